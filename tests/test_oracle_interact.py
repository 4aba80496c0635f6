"""Pins of the oracle's pair interaction (Section 2 stage PI, Table 1 terms).

Each check is fixed by a closed form, a conservation law or a lattice
identity, chosen so that a dropped term, a wrong sign, a swapped density or
a missing mass factor fails at least one of them.  Kernel values used in
expected results come from ``kernel_f``, which is pinned on its own.
"""

import math

import numpy as np
import pytest

from sph_inputs import blob, physics
from sph_inputs.dambreak import Layout


def _pair_layout(xa, xb, va, vb, rhoa, rhob, nb=0, gravity=9.81, alpha=0.1):
    ph = physics(0.01, alpha=alpha, gravity=gravity)
    x = np.array([xa, xb], dtype=float)
    v = np.array([va, vb], dtype=float)
    rho = np.array([rhoa, rhob], dtype=float)
    return Layout("pair", x, v, rho, nb, ph, np.array([-1.0] * 3), np.array([2.0] * 3))


def test_isolated_particle_feels_only_gravity(ora):
    L = _pair_layout([0.5, 0.5, 0.5], [1.5, 1.5, 1.5], [1, 2, 3], [0, 0, 0], 1003.0, 1000.0)
    P = ora.params(L.phys)
    ace, visc, nnb, npairs = ora.interact(L.x, L.v, L.rho, 0, P)
    assert npairs == 0
    assert np.array_equal(ace[0], [0.0, 0.0, -9.81, 0.0]) and visc[0] == 0.0


def test_static_pressure_pair(ora):
    # Two resting fluid particles at r = h along x, equal density rho > rho0:
    # a_a = g - m (2 P / rho^2) F(h) r_ab ; repulsive (a_a points along +x
    # when x_a > x_b); no viscosity, no density change.
    h = physics(0.01).h
    rho = 1005.0
    L = _pair_layout([0.5 + h, 0.5, 0.5], [0.5, 0.5, 0.5], [0, 0, 0], [0, 0, 0], rho, rho)
    P = ora.params(L.phys)
    ace, visc, _, npairs = ora.interact(L.x, L.v, L.rho, 0, P)
    assert npairs == 2
    m = L.phys.mass
    press = ora.pressure(P, rho)
    F = ora.kernel_f(P, h)
    ax = -m * (2 * press / rho**2) * F * h
    assert ax > 0
    assert ace[0, 0] == pytest.approx(ax, rel=1e-12)
    assert ace[1, 0] == pytest.approx(-ax, rel=1e-12)
    assert ace[0, 1] == 0.0 and ace[0, 2] == pytest.approx(-9.81, rel=1e-15)
    assert ace[0, 3] == 0.0 and visc[0] == 0.0


def test_unequal_pressure_pair_uses_both_densities(ora):
    # P_a/rho_a^2 + P_b/rho_b^2 : swapping the densities leaves the pair
    # force unchanged, and the result equals the sum of the two terms.
    h = physics(0.01).h
    r = 0.7 * h
    L = _pair_layout([0.5 + r, 0.5, 0.5], [0.5, 0.5, 0.5], [0, 0, 0], [0, 0, 0], 1002.0, 1009.0)
    P = ora.params(L.phys)
    ace, *_ = ora.interact(L.x, L.v, L.rho, 0, P)
    L2 = _pair_layout([0.5 + r, 0.5, 0.5], [0.5, 0.5, 0.5], [0, 0, 0], [0, 0, 0], 1009.0, 1002.0)
    ace2, *_ = ora.interact(L2.x, L2.v, L2.rho, 0, P)
    assert ace[0, 0] == pytest.approx(ace2[0, 0], rel=1e-14)
    m, F = L.phys.mass, ora.kernel_f(P, r)
    pa = ora.pressure(P, 1002.0) / 1002.0**2
    pb = ora.pressure(P, 1009.0) / 1009.0**2
    assert ace[0, 0] == pytest.approx(-m * (pa + pb) * F * r, rel=1e-12)


def test_approaching_pair_viscosity_and_continuity(ora):
    # rho = rho0 (P = 0); particle a at x = r moves toward b at -U.
    # v_ab . r_ab = -U r < 0 -> Monaghan term active:
    #   mu = h (-U r)/(r^2 + eta2), Pi = -alpha c0 mu / rho0 > 0,
    #   a_a = g - m Pi F r_ab  (decelerates a: a_a along +x),
    #   drho_a = m (-U r) F > 0 (compression), visc = |mu|.
    ph = physics(0.01)
    h, U = ph.h, 0.8
    r = 1.3 * h
    L = _pair_layout([0.5 + r, 0.5, 0.5], [0.5, 0.5, 0.5], [-U, 0, 0], [0, 0, 0], 1000.0, 1000.0)
    P = ora.params(L.phys)
    ace, visc, _, _ = ora.interact(L.x, L.v, L.rho, 0, P)
    m, F = ph.mass, ora.kernel_f(P, r)
    mu = h * (-U * r) / (r * r + ph.eta2)
    Pi = -ph.alpha * ph.c0 * mu / ph.rho0
    assert Pi > 0
    assert ace[0, 0] == pytest.approx(-m * Pi * F * r, rel=1e-12)
    assert ace[0, 0] > 0
    assert ace[0, 3] == pytest.approx(m * (-U * r) * F, rel=1e-12)
    assert ace[0, 3] > 0 and ace[1, 3] == pytest.approx(ace[0, 3], rel=1e-12)
    assert visc[0] == pytest.approx(abs(mu), rel=1e-12)


def _monaghan_pair_expect(ora, P, ph, r, vrel, rhoa, rhob):
    """Closed form of one approaching pair along x (x_a - x_b = r > 0,
    v_a - v_b = vrel < 0) with unequal densities: the Monaghan term of the
    Table 1 viscosity uses the arithmetic means of the two sound speeds and of
    the two densities.  Every ingredient is pinned on its own: the kernel
    factor F, the Tait pressure and the sound speed sqrt(dP/drho)."""
    m, F, h = ph.mass, ora.kernel_f(P, r), ph.h
    mu = h * (vrel * r) / (r * r + ph.eta2)
    cbar = 0.5 * (ora.sound(P, rhoa) + ora.sound(P, rhob))
    rbar = 0.5 * (rhoa + rhob)
    Pi = -ph.alpha * cbar * mu / rbar
    pa = ora.pressure(P, rhoa) / rhoa**2
    pb = ora.pressure(P, rhob) / rhob**2
    return m, F, mu, Pi, pa, pb


def test_approaching_pair_unequal_densities_means(ora):
    # rho_a = 1006, rho_b = 995: c and rho differ between the two ends, so the
    # averaging of the Monaghan term matters (max(c) or a geometric mean of
    # the densities would change Pi by about 1.6e-2 and 1.5e-5 relative).
    ph = physics(0.01)
    r, U = 1.15 * ph.h, 0.6
    rhoa, rhob = 1006.0, 995.0
    L = _pair_layout([0.5 + r, 0.5, 0.5], [0.5, 0.5, 0.5], [-U, 0, 0], [0, 0, 0], rhoa, rhob)
    P = ora.params(L.phys)
    ace, visc, _, npairs = ora.interact(L.x, L.v, L.rho, 0, P)
    assert npairs == 2
    m, F, mu, Pi, pa, pb = _monaghan_pair_expect(ora, P, ph, r, -U, rhoa, rhob)
    assert Pi > 0 and mu < 0
    ax = -m * (pa + pb + Pi) * F * r
    assert ace[0, 0] == pytest.approx(ax, rel=1e-13)
    assert ace[1, 0] == pytest.approx(-ax, rel=1e-13)       # the pair term is antisymmetric
    assert ace[0, 3] == pytest.approx(m * (-U * r) * F, rel=1e-13)
    assert ace[1, 3] == pytest.approx(ace[0, 3], rel=1e-13)
    assert visc[0] == pytest.approx(abs(mu), rel=1e-13) and visc[1] == visc[0]
    # the viscous part on its own: subtract the same pair at rest
    L0 = _pair_layout([0.5 + r, 0.5, 0.5], [0.5, 0.5, 0.5], [0, 0, 0], [0, 0, 0], rhoa, rhob)
    a0, *_ = ora.interact(L0.x, L0.v, L0.rho, 0, P)
    assert ace[0, 0] - a0[0, 0] == pytest.approx(-m * Pi * F * r, rel=1e-9)


def test_fluid_boundary_pair_unequal_densities_means(ora):
    # fluid a (rho_a = 997, P_a < 0) moves down onto boundary b (rho_b = 1012):
    # the fluid's acceleration carries the same averaged Monaghan term; the
    # boundary target gets only its continuity rate.
    ph = physics(0.01)
    r, U = 0.95 * ph.h, 0.45
    rhoa, rhob = 997.0, 1012.0
    # id 0 is the boundary particle (nb = 1), id 1 the fluid particle above it
    L = _pair_layout([0.5, 0.5, 0.5], [0.5, 0.5, 0.5 + r], [0, 0, 0], [0, 0, -U], rhob, rhoa)
    P = ora.params(L.phys)
    ace, visc, _, npairs = ora.interact(L.x, L.v, L.rho, 1, P)
    assert npairs == 2
    # seen from the fluid particle: r_ab = +r along z, v_ab = -U along z
    m, F, mu, Pi, pa, pb = _monaghan_pair_expect(ora, P, ph, r, -U, rhoa, rhob)
    assert pa < 0 < pb and Pi > 0
    assert ace[1, 2] == pytest.approx(-9.81 - m * (pa + pb + Pi) * F * r, rel=1e-13)
    assert ace[1, 0] == 0.0 and ace[1, 1] == 0.0
    assert ace[1, 3] == pytest.approx(m * (-U * r) * F, rel=1e-13)
    assert visc[1] == pytest.approx(abs(mu), rel=1e-13)
    assert np.array_equal(ace[0, :3], [0.0, 0.0, 0.0]) and visc[0] == 0.0
    assert ace[0, 3] == pytest.approx(ace[1, 3], rel=1e-13)


def test_separating_pair_has_no_viscous_force(ora):
    ph = physics(0.01)
    r = 0.9 * ph.h
    L = _pair_layout([0.5 + r, 0.5, 0.5], [0.5, 0.5, 0.5], [0.7, 0, 0], [0, 0, 0], 1000.0, 1000.0)
    P = ora.params(L.phys)
    ace, visc, _, _ = ora.interact(L.x, L.v, L.rho, 0, P)
    assert ace[0, 0] == 0.0 and ace[0, 1] == 0.0
    assert ace[0, 3] < 0  # expansion lowers density
    assert visc[0] > 0     # |mu| still reported for the time step


def test_boundary_target_continuity_only(ora):
    # id 0 is a boundary particle (nb = 1); the fluid particle approaches it.
    ph = physics(0.01)
    r, U = 1.1 * ph.h, 0.5
    L = _pair_layout([0.5, 0.5, 0.5], [0.5, 0.5, 0.5 + r], [0, 0, 0], [0, 0, -U], 1000.0, 1000.0)
    P = ora.params(L.phys)
    ace, visc, nnb, _ = ora.interact(L.x, L.v, L.rho, 1, P)
    F = ora.kernel_f(P, r)
    # a = boundary: v_ab . r_ab = (0 - (-U)) * (0 - r) = -U r
    assert np.array_equal(ace[0, :3], [0.0, 0.0, 0.0]) and visc[0] == 0.0
    assert ace[0, 3] == pytest.approx(ph.mass * (-U * r) * F, rel=1e-12) and ace[0, 3] > 0
    # the fluid particle is pushed back up by the Monaghan term (P = 0 here)
    assert ace[1, 2] > -9.81


def test_boundary_pressure_repels_fluid(ora):
    ph = physics(0.01)
    r = 1.0 * ph.h
    L = _pair_layout([0.5, 0.5, 0.5], [0.5, 0.5, 0.5 + r], [0, 0, 0], [0, 0, 0], 1010.0, 1000.0)
    P = ora.params(L.phys)
    ace, *_ = ora.interact(L.x, L.v, L.rho, 1, P)
    pb = ora.pressure(P, 1010.0) / 1010.0**2
    assert ace[1, 2] == pytest.approx(-9.81 - ph.mass * pb * ora.kernel_f(P, r) * (r), rel=1e-12)
    assert ace[1, 2] > -9.81


def test_momentum_and_angular_momentum_conservation(ora):
    # Free jittered blob with random velocities and densities, no gravity:
    # pair forces are antisymmetric and central.
    B = blob(14, 0.01, 11, vel_sigma=0.5, jitter=0.3)
    P = ora.params(B.phys)
    ace, visc, _, _ = ora.interact(B.x, B.v, B.rho, 0, P)
    a = ace[:, :3]
    assert np.abs(a.sum(0)).max() <= 1e-12 * np.abs(a).sum()
    xc = B.x - B.x.mean(0)
    L = np.cross(xc, a)
    assert np.abs(L.sum(0)).max() <= 1e-12 * np.abs(L).sum()
    # mass is conserved too: sum of drho/dt is not zero in general, but the
    # pairwise continuity terms are symmetric: m v_ab.r_ab F_ab = m v_ba.r_ba F_ba
    rp, cols = ora.neighbour_csr(B.x, 0, B.phys.h)
    assert rp[-1] > 0


def _lattice_block(ns, dp):
    g = (np.stack(np.meshgrid(*[np.arange(ns)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) * dp
    return g + 0.25


def _consistency(ora, P, dp):
    m = int(math.ceil(2 * P.h / dp)) + 1
    r = np.arange(-m, m + 1) * dp
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    d = np.linalg.norm(g, axis=1)
    sel = (d > 0) & (d < 2 * P.h)
    F = np.array([ora.kernel_f(P, x) for x in d[sel]])
    return -(g[sel, 2] ** 2 * F).sum() * dp**3


def _interior(x, dp, ns, h):
    lo, hi = x.min(0) + 2 * h, x.max(0) - 2 * h
    return np.all((x > lo) & (x < hi), axis=1)


def test_linear_pressure_field_on_lattice(ora):
    # Densities chosen so that P/rho^2 = f0 + f1 z.  On a perfect lattice the
    # interior sum gives a_z = g_z - f1 rho0 C exactly, with C the lattice
    # gradient-consistency factor; a_x = a_y = 0.
    dp, ns = 0.01, 16
    ph = physics(dp)
    P = ora.params(ph)
    x = _lattice_block(ns, dp)
    f0, f1 = 2.0e-3, -1.5e-2
    target = f0 + f1 * (x[:, 2] - x[:, 2].min())

    def solve(t):
        lo, hi = 900.0, 1100.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if ora.pressure(P, mid) / mid**2 < t:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    rho = np.array([solve(t) for t in target])
    L = Layout("lat", x, np.zeros_like(x), rho, 0, ph, x.min(0) - 1, x.max(0) + 1)
    ace, *_ = ora.interact(L.x, L.v, L.rho, 0, P)
    inner = _interior(x, dp, ns, ph.h)
    C = _consistency(ora, P, dp)
    expect = -9.81 - f1 * ph.rho0 * C
    got = ace[inner, 2]
    assert np.allclose(got, expect, rtol=1e-7, atol=1e-9)
    assert np.abs(ace[inner, :2]).max() < 1e-9


def test_continuity_rigid_motion_and_expansion(ora):
    dp, ns = 0.01, 14
    ph = physics(dp)
    P = ora.params(ph)
    x = _lattice_block(ns, dp)
    rho = np.full(len(x), 1000.0)
    inner = _interior(x, dp, ns, ph.h)
    # rigid translation + rotation: v_ab . r_ab = 0 for every pair
    w = np.array([0.3, -0.2, 0.5])
    v = np.array([0.1, 0.2, -0.3]) + np.cross(w, x - x.mean(0))
    ace, *_ = ora.interact(x, v, rho, 0, P)
    assert np.abs(ace[:, 3]).max() < 1e-9
    # uniform expansion v = eps x: drho/dt = -3 eps rho0 C on the interior
    eps = 0.05
    ace, *_ = ora.interact(x, eps * x, rho, 0, P)
    C = _consistency(ora, P, dp)
    assert np.allclose(ace[inner, 3], -3 * eps * 1000.0 * C, rtol=1e-9)


def test_viscosity_dissipates_and_is_linear_in_alpha(ora):
    # With rho = rho0 everywhere (P = 0) the only force is the Monaghan term:
    # the rate of kinetic energy sum m v.a (no gravity) must be negative, and
    # the force must scale linearly with alpha.
    B = blob(12, 0.01, 21, vel_sigma=0.3, jitter=0.3, rho_sigma=0.0)
    P1 = ora.params(B.phys, alpha=0.1)
    P2 = ora.params(B.phys, alpha=0.2)
    a1, *_ = ora.interact(B.x, B.v, B.rho, 0, P1)
    a2, *_ = ora.interact(B.x, B.v, B.rho, 0, P2)
    power = (B.v * a1[:, :3]).sum()
    assert power < 0
    assert np.allclose(a2[:, :3], 2 * a1[:, :3], rtol=1e-12, atol=1e-15)
    assert np.array_equal(a1[:, 3], a2[:, 3])
