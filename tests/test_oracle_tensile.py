"""Pins of the oracle's tensile correction (Table 3 "tensil", following the
paper's ref. [34]): R_a = 0.01 P_a/rho_a^2 for P_a > 0 and 0.2 |P_a|/rho_a^2
for P_a < 0; a pair adds (R_a + R_b) f^4, f = W(r)/W(dp), to the pressure
factor P_a/rho_a^2 + P_b/rho_b^2 of the momentum equation.

The closed forms below follow from f(dp) = 1 and f^4 = 1/16 where W(r) =
W(dp)/2, so a wrong exponent, a wrong branch constant, a missing factor of
two (R_a + R_b) or a wrong normalisation fails one of them."""

import dataclasses

import numpy as np
import pytest

from sph_inputs import blob, physics
from sph_inputs.dambreak import Layout

DP = 0.01


@pytest.fixture(params=[0, 1], ids=["wendland", "cubic"])
def kernel(request):
    return request.param


def _pair(r, rho, kernel, tensile):
    ph = dataclasses.replace(physics(DP, kernel=kernel, gravity=0.0),
                             tensile_dp=DP if tensile else 0.0)
    x = np.array([[0.5 + r, 0.5, 0.5], [0.5, 0.5, 0.5]])
    v = np.zeros((2, 3))
    return Layout("pair", x, v, np.array([rho, rho]), 0, ph, np.array([-1.0] * 3),
                  np.array([2.0] * 3))


def _ax(ora, L):
    ace, *_ = ora.interact(L.x, L.v, L.rho, 0, ora.params(L.phys))
    return ace[0, 0]


@pytest.mark.parametrize("rho,ratio", [(1004.0, 1.01), (996.0, 0.8)])
def test_ratio_at_the_particle_spacing(ora, kernel, rho, ratio):
    # r = dp: f = 1, so the pressure factor 2 P/rho^2 becomes
    # 2 P/rho^2 + 2 R with R = 0.01 P/rho^2 (P > 0) or -0.2 P/rho^2 (P < 0)
    on = _ax(ora, _pair(DP, rho, kernel, True))
    off = _ax(ora, _pair(DP, rho, kernel, False))
    assert on / off == pytest.approx(ratio, rel=1e-12)


@pytest.mark.parametrize("rho,extra", [(1004.0, 0.01), (996.0, -0.2)])
def test_ratio_where_the_kernel_halves(ora, kernel, rho, extra):
    # W(r) = W(dp)/2: f^4 = 1/16, the factor becomes 2 P/rho^2 (1 + extra/16)
    P = ora.params(physics(DP, kernel=kernel))
    w_half = 0.5 * ora.kernel_w(P, DP)
    lo, hi = DP, 2.0 * P.h  # W decreases from W(dp) to 0 on [dp, 2h]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if ora.kernel_w(P, mid) > w_half:
            lo = mid
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    on = _ax(ora, _pair(r, rho, kernel, True))
    off = _ax(ora, _pair(r, rho, kernel, False))
    assert on / off == pytest.approx(1.0 + extra / 16.0, rel=1e-9)


def test_no_contribution_at_zero_pressure_or_beyond_support(ora, kernel):
    L_on, L_off = _pair(DP, 1000.0, kernel, True), _pair(DP, 1000.0, kernel, False)
    assert _ax(ora, L_on) == _ax(ora, L_off)  # P = 0: R = 0 on both sides


def test_momentum_conserved_with_negative_pressures(ora):
    # free blob around rho0 - 5 (mostly negative pressure): the tensile term
    # is symmetric in (a, b), so the internal forces still cancel
    L = blob(8, DP, seed=41, rho_sigma=3.0)
    L.rho = L.rho - 5.0
    L.phys = dataclasses.replace(L.phys, tensile_dp=DP)
    P = ora.params(L.phys)
    ace, *_ = ora.interact(L.x, L.v, L.rho, 0, P)
    m = L.phys.mass
    tot = (m * ace[:, :3]).sum(0)
    scale = (m * np.abs(ace[:, :3])).sum()
    assert np.linalg.norm(tot) <= 1e-12 * scale
    off = ora.interact(L.x, L.v, L.rho, 0, ora.params(L.phys, tensile_dp=0.0))[0]
    assert np.abs(ace[:, :3] - off[:, :3]).max() > 1e-3 * np.abs(off[:, :3]).max()


def test_vjp_with_tensile_correction_matches_central_differences(ora, kernel):
    from sph_inputs import dam_break

    L = dam_break(0.02, 3, fluid=(0.12, 0.12, 0.12), tank=(0.2, 0.14, 0.14), vel_sigma=0.3,
                  vel_seed=4, kernel=kernel)
    L.phys = dataclasses.replace(L.phys, tensile_dp=L.phys.dp)
    rng = np.random.default_rng(5)
    L.rho = L.rho + rng.normal(0, 2.0, L.n)
    L.rho[: L.nb] = np.abs(L.rho[: L.nb] - L.phys.rho0) + L.phys.rho0
    P = ora.params(L.phys)
    n, nb = L.n, L.nb
    w = rng.normal(size=(n, 4))
    w[:nb, :3] = 0.0
    xb, vb, rb, ab = ora.interact_vjp(L.x, L.v, L.rho, nb, P, w)

    def f(x, rho):
        ace, *_ = ora.interact(x, L.v, rho, nb, P)
        return (ace * w).sum()

    for k in range(3):
        ux = rng.normal(size=(n, 3))
        ux[:nb] = 0.0
        ur = rng.normal(size=n)
        eps, s = 1e-7, L.phys.dp
        fd = (f(L.x + eps * s * ux, L.rho + eps * 10 * ur) -
              f(L.x - eps * s * ux, L.rho - eps * 10 * ur)) / (2 * eps)
        an = s * (xb * ux).sum() + 10 * (rb * ur).sum()
        assert an == pytest.approx(fd, rel=2e-6), (k, an, fd)
