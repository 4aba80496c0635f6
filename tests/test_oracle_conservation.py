"""Pins of the oracle's global conservation sums (Section 2: the momentum and
continuity equations are evaluated pair-wise, so internal forces of fluid
pairs cancel; gravity and the boundaries are external).

Closed forms on a cubic lattice block of n^3 fluid particles at (i + 1/2) dp:
the centroid is n dp / 2 per axis, and about the centroid each axis holds
sum_i (i - (n - 1)/2)^2 dp^2 = n (n^2 - 1) dp^2 / 12 per lattice line, so the
inertia tensor of the block is I = m n^3 dp^2 (n^2 - 1) / 6 times the
identity.  Distinct components in every vector catch a transposed or
mis-signed cross product.
"""

import numpy as np
import pytest

from sph_inputs import blob, physics
from sph_inputs.dambreak import Layout


def _block(n, dp, v=None, gravity=9.81, nb_extra=0):
    ph = physics(dp, gravity=gravity)
    i = np.arange(n)
    gz, gy, gx = np.meshgrid(i, i, i, indexing="ij")
    x = np.stack([(gx.ravel() + 0.5) * dp, (gy.ravel() + 0.5) * dp, (gz.ravel() + 0.5) * dp], 1)
    if nb_extra:
        # boundary particles first (ids [0, nb)), far from the block
        xb = np.full((nb_extra, 3), -1.0) + 0.01 * np.arange(nb_extra)[:, None]
        x = np.concatenate([xb, x])
    nt = x.shape[0]
    vv = np.zeros((nt, 3)) if v is None else v
    rho = np.full(nt, ph.rho0)
    return Layout("block", x, vv, rho, nb_extra, ph, np.array([-2.0] * 3), np.array([2.0] * 3)), ph


def test_uniform_translation(ora):
    n, dp = 7, 0.01
    U = np.array([0.3, -0.7, 1.1])
    L, ph = _block(n, dp)
    v = np.tile(U, (L.n, 1))
    out = ora.conservation(L.x, v, None, 0, ora.params(ph))
    f = ora.conservation_fields(out)
    N, m = n ** 3, ph.mass
    c = np.full(3, n * dp / 2)
    assert f["count"] == N
    np.testing.assert_allclose(f["momentum"], N * m * U, rtol=1e-13)
    assert f["kinetic_energy"] == pytest.approx(0.5 * N * m * U @ U, rel=1e-13)
    np.testing.assert_allclose(f["angular_momentum"], N * m * np.cross(c, U), rtol=1e-12)
    assert np.all(f["internal_force"] == 0) and np.all(f["internal_torque"] == 0)
    assert f["force_scale"] == 0
    # the same uniform force Fc on every particle on top of gravity: the sums
    # are N m Fc, the torque N m c x Fc, the scale N m |Fc|
    Fc = np.array([2.0, -0.5, 1.25])
    ace = np.zeros((L.n, 4))
    ace[:, :3] = np.array(ph.g) + Fc
    f = ora.conservation_fields(ora.conservation(L.x, v, ace, 0, ora.params(ph)))
    np.testing.assert_allclose(f["internal_force"], N * m * Fc, rtol=1e-13)
    np.testing.assert_allclose(f["internal_torque"], N * m * np.cross(c, Fc), rtol=1e-12)
    assert f["force_scale"] == pytest.approx(N * m * np.linalg.norm(Fc), rel=1e-13)


def test_rigid_rotation_about_the_centroid(ora):
    n, dp = 6, 0.02
    w = np.array([0.4, -1.3, 2.2])
    L, ph = _block(n, dp)
    c = np.full(3, n * dp / 2)
    v = np.cross(w, L.x - c)
    f = ora.conservation_fields(ora.conservation(L.x, v, None, 0, ora.params(ph)))
    m = ph.mass
    inertia = m * n ** 3 * dp ** 2 * (n ** 2 - 1) / 6.0
    np.testing.assert_allclose(f["momentum"], 0.0, atol=1e-15)
    np.testing.assert_allclose(f["angular_momentum"], inertia * w, rtol=1e-12)
    assert f["kinetic_energy"] == pytest.approx(0.5 * inertia * w @ w, rel=1e-12)


def test_potential_energy_of_a_resting_block(ora):
    n, dp = 5, 0.01
    L, ph = _block(n, dp, gravity=9.81)
    f = ora.conservation_fields(ora.conservation(L.x, L.v, None, 0, ora.params(ph)))
    # g = (0, 0, -9.81): -m g.x summed = m 9.81 sum z = N m 9.81 (n dp / 2)
    assert f["potential_energy"] == pytest.approx(n ** 3 * ph.mass * 9.81 * n * dp / 2, rel=1e-13)
    # gravity along an oblique direction: -m N g.c
    P = ora.params(ph, g=(1.0, -2.0, 3.5))
    f2 = ora.conservation_fields(ora.conservation(L.x, L.v, None, 0, P))
    c = np.full(3, n * dp / 2)
    assert f2["potential_energy"] == pytest.approx(-n ** 3 * ph.mass * (np.array([1.0, -2.0, 3.5]) @ c),
                                                   rel=1e-13)
    assert f2["kinetic_energy"] == 0.0


def test_boundary_and_excluded_particles_are_not_summed(ora):
    n, dp = 4, 0.01
    U = np.array([0.5, 0.25, -1.0])
    L, ph = _block(n, dp, nb_extra=9)
    v = np.tile(U, (L.n, 1))
    excl = np.zeros(L.n, dtype=np.uint8)
    excl[[L.nb + 3, L.nb + 17]] = 1
    ace = np.zeros((L.n, 4))
    ace[:, :3] = 100.0  # boundary slots would dominate if summed
    ace[L.nb:, :3] = np.array(ph.g)  # fluid: gravity only, zero internal force
    f = ora.conservation_fields(ora.conservation(L.x, v, ace, L.nb, ora.params(ph), excl))
    N = n ** 3 - 2
    assert f["count"] == N
    np.testing.assert_allclose(f["momentum"], N * ph.mass * U, rtol=1e-13)
    np.testing.assert_allclose(f["internal_force"], 0.0, atol=0)
    assert f["force_scale"] == 0.0


def test_internal_force_and_torque_vanish_on_a_free_blob(ora):
    """Pair-wise central forces (pressure and Monaghan viscosity act along
    r_ab, the pair terms are antisymmetric): the internal force and torque
    sums are zero to rounding, with or without gravity, which the sums must
    subtract."""
    for gravity in (False, True):
        L = blob(10, 0.01, 123, vel_sigma=0.3, gravity=gravity)
        P = ora.params(L.phys)
        ace, *_ = ora.interact(L.x, L.v, L.rho, 0, P)
        f = ora.conservation_fields(ora.conservation(L.x, L.v, ace, 0, P))
        scale = f["force_scale"]
        assert scale > 0
        assert np.linalg.norm(f["internal_force"]) <= 1e-12 * scale
        rmax = np.abs(L.x).max()
        assert np.linalg.norm(f["internal_torque"]) <= 1e-12 * scale * rmax
    # sanity: the sums are not trivially zero (one particle's force removed)
    ace2 = ace.copy()
    ace2[5, :3] = np.array(L.phys.g)
    f2 = ora.conservation_fields(ora.conservation(L.x, L.v, ace2, 0, P))
    m = L.phys.mass
    np.testing.assert_allclose(f2["internal_force"], -m * (ace[5, :3] - np.array(L.phys.g)),
                               rtol=1e-6, atol=1e-12 * scale)
