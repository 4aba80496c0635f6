"""Position-load policy SPH_POS_ABS64 (the state keeps FP64 absolute positions,
the pair kernel forms r_ab = fp32(x_a - x_b) from them) against the FP64
oracle at the true positions, and its carrying through reorder, update and
decoding.

* Forces: relative L2 <= 1e-4 and per-target error <= 1e-3 of the rms, as for
  the default policy; both policies printed against the same reference.
* sph_build_cells gathers pos64 bitwise; sph_decode returns it.
* One whole step: positions against the oracle's FP64 Verlet update within
  the FP32 acceleration error times dt^2/2 (no FP32 offset storage term).
"""

import numpy as np
import pytest

from _helpers import parity, rel_l2
from sph_inputs import dam_break

pytestmark = pytest.mark.gpu


def _sim(lay, pos64, nsub=1):
    from paper_1110_3711_amd import sph

    return sph.Simulation(lay, nsub=nsub, pos64=pos64)


@pytest.mark.parametrize("nsub", [1, 2])
def test_abs64_forces_match_oracle(ora, nsub):
    import torch

    lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=41)
    print(f"pos64 forces dam_break_8k+v nsub={nsub} n={lay.n}", flush=True)
    P = ora.params(lay.phys)
    v32 = lay.v.astype(np.float32).astype(np.float64)
    r32 = (lay.rho - lay.phys.rho0).astype(np.float32).astype(np.float64) + lay.phys.rho0
    ref, rvisc, _, npairs = ora.interact(lay.x, v32, r32, lay.nb, P)
    f = np.arange(lay.nb, lay.n)
    out = {}
    for pos64 in (False, True):
        sim = _sim(lay, pos64, nsub)
        sim.build_cells()
        sim.npairs.zero_()
        sim.interact()
        torch.cuda.synchronize()
        assert sim.dev_status() == 0
        ace, visc = sim.by_id(sim.ace), sim.by_id(sim.visc)
        label = "ABS64" if pos64 else "OFFSET32"
        out[label] = parity(f"{label} vs oracle at the true positions", acc=(ace[f, :3], ref[f, :3]),
                            drho=(ace[:, 3], ref[:, 3]), visc=(visc, rvisc))
        got = int(sim.npairs.sum().item())
        # FP32 decisions at the cutoff may differ from FP64 by a few pairs
        assert abs(got - npairs) <= 1e-5 * npairs, (got, npairs)
    assert out["ABS64"]["acc"][0] <= 2 * out["OFFSET32"]["acc"][0] + 1e-7


def test_abs64_positions_carried_through_reorder(ora):
    import torch

    lay = dam_break(0.02, 5, vel_sigma=0.1)
    print(f"pos64 reorder n={lay.n}", flush=True)
    sim = _sim(lay, True)
    x0, _, _ = sim.decode()
    assert np.array_equal(x0, lay.x)  # encoded state keeps the FP64 input bitwise
    sim.build_cells()
    torch.cuda.synchronize()
    x1, _, _ = sim.decode()
    assert np.array_equal(x1, lay.x)
    ids = sim.a.id.cpu().numpy()
    p64 = sim.a.pos64.cpu().numpy()
    assert np.array_equal(p64, lay.x[ids])


def test_abs64_one_step_matches_oracle(ora):
    import torch

    lay = dam_break(0.01, 11103712, vel_sigma=0.1, vel_seed=3)
    print(f"pos64 one step n={lay.n}", flush=True)
    sim = _sim(lay, True)
    sim.step()
    torch.cuda.synchronize()
    assert sim.dev_status() == 0
    x, v, r = sim.decode()
    S = ora.State(lay)
    S.v[:] = lay.v.astype(np.float32).astype(np.float64)
    S.vprev[:] = S.v
    S.rho[:] = (lay.rho - lay.phys.rho0).astype(np.float32).astype(np.float64) + lay.phys.rho0
    S.rhoprev[:] = S.rho
    ace, visc, _, _ = S.interact()
    dt = ora.time_step(S.rho, ace, visc, S.nb, S.P, S.excl)
    S.verlet(ace, dt)
    assert sim.dt.item() == pytest.approx(dt, rel=1e-5)
    f = slice(lay.nb, None)
    # FP32 acceleration error times dt^2/2 and the dt error times |v|; no
    # FP32 offset storage term (the FP64 position is kept)
    tol_x = 1e-5 * dt * (np.abs(S.v[f]).max() + 1) + 1e-4 * dt * dt * np.abs(ace[f, :3]).max()
    err = np.abs(x[f] - S.x[f]).max()
    print(f"  max |x_gpu - x_oracle| = {err:.3e} m (bound {tol_x:.3e})", flush=True)
    assert err <= tol_x
    assert np.array_equal(x[: lay.nb], lay.x[: lay.nb])
    assert rel_l2(v[f], S.v[f]) <= 1e-5
    # the (cell, offset) view still encodes the same positions to FP32
    org = np.array(list(sim.grid.origin))
    cell = sim.grid.cell
    nc = [int(c) for c in sim.grid.nc]
    xo = ora.decode(sim.a.cell.cpu().numpy(), sim.a.pos.cpu().numpy()[:, :3], org, cell, nc)
    ids = sim.a.id.cpu().numpy()
    xo_id = np.empty_like(xo)
    xo_id[ids] = xo
    assert np.abs(xo_id - x).max() <= np.spacing(np.float32(cell))
