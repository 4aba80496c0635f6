"""Pins of the oracle's time step, Verlet integrator and position encoding.

* Verlet (Table 1): a free particle under constant gravity is integrated
  exactly by both the regular and the corrective step.
* Variable time step (Table 1, Section 4.1): closed form for isolated
  particles.
* Dynamic boundaries: fixed position and velocity, density floored at rho0.
* Still-water column: a hydrostatic column stays at rest and keeps a
  hydrostatic pressure profile (builder-chosen tolerances; the paper gives
  none).
* Encoding: integer cell + FP32 offset round trip within half an FP32 ulp of
  the half cell.
"""

import math

import numpy as np
import pytest

from sph_inputs import cell_grid, column, named_case, physics
from sph_inputs.dambreak import Layout


def _free_layout(nf=3):
    ph = physics(0.01)
    rng = np.random.default_rng(7)
    x = np.array([[0.1, 0.1, 0.5], [0.5, 0.1, 0.5], [0.9, 0.1, 0.5]])[:nf]
    v = rng.normal(0, 0.5, size=(nf, 3))
    rho = np.full(nf, 1000.0)
    return Layout("free", x, v, rho, 0, ph, np.array([-5.0] * 3), np.array([5.0] * 3))


def test_free_fall_is_exact(ora):
    L = _free_layout()
    S = ora.State(L)
    x0, v0 = S.x.copy(), S.v.copy()
    dts = S.run(97)  # crosses two corrective steps (step 0 and 39, 79)
    dt = dts[0]
    assert np.all(dts == dt)
    t = dt * 97
    g = np.array([0, 0, -9.81])
    assert np.allclose(S.x, x0 + v0 * t + 0.5 * g * t * t, rtol=0, atol=1e-13)
    assert np.allclose(S.v, v0 + g * t, rtol=0, atol=1e-13)


def test_time_step_closed_form(ora):
    L = _free_layout()
    P = ora.params(L.phys)
    ace, visc, *_ = ora.interact(L.x, L.v, L.rho, 0, P)
    dt = ora.time_step(L.rho, ace, visc, 0, P)
    h = L.phys.h
    assert dt == pytest.approx(0.2 * min(math.sqrt(h / 9.81), h / L.phys.c0), rel=1e-15)


def test_time_step_terms(ora):
    ph = physics(0.01)
    P = ora.params(ph)
    rho = np.array([1000.0, 1020.0, 990.0])
    ace = np.array([[0, 0, 0, 0], [3.0, 4.0, 0, 1.0], [0, 0, 200.0, 0]], dtype=float)
    visc = np.array([0.0, 0.5, 3.0])
    # boundary particle 0 is ignored
    dt = ora.time_step(rho, ace, visc, 1, P)
    cands = [math.sqrt(ph.h / 5.0), math.sqrt(ph.h / 200.0),
             ph.h / (ora.sound(P, 1020.0) + 0.5), ph.h / (ora.sound(P, 990.0) + 3.0)]
    assert dt == pytest.approx(0.2 * min(cands), rel=1e-15)


def test_verlet_regular_and_corrective_updates(ora):
    L = _free_layout(1)
    S = ora.State(L)
    S.vprev[:] = [[0.3, -0.1, 0.2]]
    S.rhoprev[:] = [1001.0]
    ace = np.array([[1.0, 2.0, -3.0, 7.0]])
    S.step = 5  # regular
    x, v, vp, r, rp = S.x.copy(), S.v.copy(), S.vprev.copy(), S.rho.copy(), S.rhoprev.copy()
    dt = 1e-3
    S.verlet(ace, dt)
    assert np.allclose(S.x, x + dt * v + 0.5 * dt * dt * ace[:, :3], rtol=0, atol=1e-15)
    assert np.allclose(S.v, vp + 2 * dt * ace[:, :3], rtol=0, atol=1e-15)
    assert S.rho[0] == pytest.approx(rp[0] + 2 * dt * 7.0, rel=1e-15)
    assert np.array_equal(S.vprev, v) and S.rhoprev[0] == r[0]
    S.step = 39  # corrective: (39 + 1) % 40 == 0
    x, v, r = S.x.copy(), S.v.copy(), S.rho.copy()
    S.verlet(ace, dt)
    assert np.allclose(S.v, v + dt * ace[:, :3], rtol=0, atol=1e-15)
    assert S.rho[0] == pytest.approx(r[0] + dt * 7.0, rel=1e-15)


def test_boundary_particles_fixed_and_density_floored(ora):
    L = named_case("dam_break_8k")
    S = ora.State(L)
    S.run(5)
    assert np.array_equal(S.x[: L.nb], L.x[: L.nb])
    assert np.all(S.v[: L.nb] == 0)
    assert np.all(S.rho[: L.nb] >= L.phys.rho0)
    assert np.any(S.rho[: L.nb] > L.phys.rho0)  # loaded boundary compresses
    # without the floor, suction can bring boundary density below rho0
    L2 = named_case("dam_break_8k")
    P = ora.params(L2.phys, bound_floor=0)
    S2 = ora.State(L2, P)
    ace = np.zeros((L2.n, 4))
    ace[: L2.nb, 3] = -1.0
    S2.verlet(ace, 1e-3)
    assert np.all(S2.rho[: L2.nb] < L2.phys.rho0)
    S3 = ora.State(named_case("dam_break_8k"))
    S3.verlet(ace, 1e-3)
    assert np.all(S3.rho[: L2.nb] == L2.phys.rho0)


def test_particle_leaving_domain_is_excluded(ora):
    L = _free_layout(2)
    L.hi[:] = [5.0, 5.0, 0.5005]
    L.v[0] = [0, 0, 10.0]
    S = ora.State(L)
    S.run(3)
    assert S.excl[0] == 1 and S.excl[1] == 0
    x = S.x.copy()
    S.run(2)
    assert np.array_equal(S.x[0], x[0])


def test_still_water_column(ora):
    L = column()
    S = ora.State(L)
    S.run(2000)
    f = slice(L.nb, None)
    assert S.excl.sum() == 0
    vmax = np.linalg.norm(S.v[f], axis=1).max()
    assert vmax < 0.02 * math.sqrt(9.81 * 0.2)
    P = ora.params(L.phys)
    xf, h = S.x[f], L.phys.h
    zs = xf[:, 2].max() + 0.5 * L.phys.dp
    inner = ((xf[:, 0] > 2 * h) & (xf[:, 0] < 0.1 - 2 * h) & (xf[:, 1] > 2 * h)
             & (xf[:, 1] < 0.1 - 2 * h) & (xf[:, 2] > 2 * h) & (xf[:, 2] < zs - 2 * h))
    assert inner.sum() > 20
    pr = np.array([ora.pressure(P, r) for r in S.rho[f][inner]])
    hyd = 1000.0 * 9.81 * (zs - xf[inner, 2])
    assert np.abs(pr - hyd).max() < 0.05 * 1000.0 * 9.81 * 0.2


def test_encoding_round_trip(ora):
    L = named_case("dam_break_8k")
    for nsub in (1, 2):
        org, cell, nc = cell_grid(L, nsub)
        cidx, off = ora.encode(L.x, org, cell, nc, L.lo, L.hi)
        assert np.all(cidx != ora.EXCLUDED)
        x = ora.decode(cidx, off, org, cell, nc)
        ulp_half = np.spacing(np.float32(cell / 2)) / 2
        assert np.abs(x - L.x).max() <= ulp_half * 1.0000001 + 1e-16
        assert np.abs(off).max() <= cell / 2 + ulp_half
    # outside the domain -> excluded
    xo = np.array([[L.lo[0] - 1e-9, 0.1, 0.1], [0.1, 0.1, L.hi[2]], [0.1, 0.1, 0.1]])
    cidx, off = ora.encode(xo, org, cell, nc, L.lo, L.hi)
    assert list(cidx[:2]) == [ora.EXCLUDED] * 2 and cidx[2] != ora.EXCLUDED
