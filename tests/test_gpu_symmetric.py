"""Symmetric evaluation of fluid-fluid pairs (SPH_PI_SYMMETRIC, Section 3.1 and
the "Symmetric" variant of Section 3.4) against the FP64 oracle and against
the gather kernel on the same encoded state.

* Forces: relative L2 <= 1e-4 against the oracle, like the gather kernel.
* Pair counts: a pair evaluated once counts as its two directed interactions
  and is decided once, in the frame of the cell it is computed from; the
  totals equal the oracle's FP32 count under that rule exactly (the gather
  kernel's under the per-target rule; the two differ only on pairs within
  rounding of the cutoff).
* Reproducibility: reactions are added in LDS by several wavefronts in an
  order that varies, so two launches agree to FP32 rounding only.
* Several staging tiles per cell (a compressed layout), excluded particles,
  fluid against the walls, and the split fluid part.
"""

import numpy as np
import pytest

from _helpers import grid_tuple, oracle_view, rel_l2
from sph_inputs import blob, dam_break, named_case

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _sim(lay):
    import torch

    from paper_1110_3711_amd import sph

    sim = sph.Simulation(lay, nsub=1)
    sim.build_cells()
    torch.cuda.synchronize()
    return sim


def _interact(sim, parts):
    import torch

    npairs = torch.zeros(2, dtype=torch.int64, device=sim.device)
    sim.ace.fill_(7.0)
    sim.visc.fill_(7.0)
    sim.interact(parts=parts, npairs=npairs)
    torch.cuda.synchronize()
    return sim.ace.clone(), sim.visc.clone(), npairs.cpu().numpy()


def _check(ora, lay, tol=TOL):
    from paper_1110_3711_amd import sph

    sim = _sim(lay)
    ace_g, visc_g, np_g = _interact(sim, sph.SPH_PI_ALL)
    ace_s, visc_s, np_s = _interact(sim, sph.SPH_PI_ALL | sph.SPH_PI_SYMMETRIC)
    gt = grid_tuple(sim)
    xq, vq, rq, excl, cidx, off = oracle_view(ora, lay.x, lay.v, lay.rho, lay.phys.rho0, gt,
                                              lay.lo, lay.hi)
    ref, rvisc, _, _ = ora.interact(xq, vq, rq, lay.nb, ora.params(lay.phys), excl=excl)
    rc2 = np.float32(4.0 * lay.phys.h * lay.phys.h)
    _, _, tot_g = ora.count_f32(cidx, off, lay.nb, gt[2], np.float32(gt[1]), rc2)
    _, _, tot_s = ora.count_f32(cidx, off, lay.nb, gt[2], np.float32(gt[1]), rc2, once=True)
    print(f"  pairs: gather {np_g.tolist()} symmetric {np_s.tolist()}", flush=True)
    assert int(np_g.sum()) == tot_g and int(np_s.sum()) == tot_s
    assert np_g[1] == np_s[1]  # boundary targets: the same gather either way
    ace = sim.by_id(ace_s)
    visc = sim.by_id(visc_s)
    f = np.arange(lay.nb, lay.n)
    f = f[excl[f] == 0]
    e_a = rel_l2(ace[f, :3], ref[f, :3])
    e_d = rel_l2(ace[:, 3], ref[:, 3])
    e_v = rel_l2(visc, rvisc)
    print(f"  rel L2 vs oracle: acc {e_a:.2e} drho {e_d:.2e} visc {e_v:.2e}", flush=True)
    assert e_a <= tol and e_d <= tol and e_v <= tol
    assert np.all(ace[excl == 1] == 0)
    assert np.all(ace[: lay.nb, :3] == 0) and np.all(visc[: lay.nb] == 0)
    # the gather kernel on the same state, element by element (|mu| of a
    # pair from the other frame differs in the last bits only)
    ag = sim.by_id(ace_g)
    assert rel_l2(ace[f, :3], ag[f, :3]) <= 1e-5 and rel_l2(ace[:, 3], ag[:, 3]) <= 1e-5
    assert rel_l2(visc, sim.by_id(visc_g)) <= 1e-6
    return sim


def test_symmetric_8k_moving(ora):
    lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=77)
    print("symmetric forces dam_break_8k+v", flush=True)
    _check(ora, lay)


def test_symmetric_8k_rest(ora):
    lay = named_case("dam_break_8k")
    print("symmetric forces dam_break_8k rest", flush=True)
    _check(ora, lay)


def test_symmetric_blob_with_excluded(ora):
    lay = blob(20, 0.01, 4, vel_sigma=0.3, jitter=0.3)
    lay.x[:50, 0] = lay.hi[0] + 1.0  # outside the domain: excluded
    print("symmetric forces blob", flush=True)
    _check(ora, lay)


def test_symmetric_several_tiles_per_cell(ora):
    # positions pulled together by 0.6: about 4.6 times the lattice density,
    # so a cell stages some 5,000 candidates (several tiles)
    lay = blob(14, 0.01, 6, vel_sigma=0.3, jitter=0.3)
    c = lay.x.mean(0)
    lay.x = c + 0.6 * (lay.x - c)
    print(f"symmetric forces compressed blob n={lay.n}", flush=True)
    _check(ora, lay)


def test_symmetric_cubic_tensile(ora):
    import dataclasses

    lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=79, kernel=1)
    lay.phys = dataclasses.replace(lay.phys, alpha=0.25, tensile_dp=lay.phys.dp)
    rng = np.random.default_rng(9)
    lay.rho = lay.rho + rng.normal(0.0, 3.0, lay.n)  # both signs of pressure
    print("symmetric forces cubic + tensile", flush=True)
    _check(ora, lay)


def test_symmetric_momentum_and_determinism(ora):
    import torch

    from paper_1110_3711_amd import sph

    lay = blob(16, 0.01, 8, vel_sigma=0.3, jitter=0.3)
    print("symmetric momentum + determinism blob", flush=True)
    sim = _sim(lay)
    sym = sph.SPH_PI_ALL | sph.SPH_PI_SYMMETRIC
    a1, v1, _ = _interact(sim, sym)
    a2, v2, _ = _interact(sim, sym)
    assert torch.equal(v1, v2)  # a maximum does not depend on the order
    assert rel_l2(a1.cpu().numpy(), a2.cpu().numpy()) <= 1e-6
    a = sim.by_id(a1)[:, :3].astype(np.float64)
    assert np.abs(a.sum(0)).max() <= 1e-5 * np.abs(a).sum()


def test_symmetric_split_parts(ora):
    """SPH_PI_FLUID | SYMMETRIC then SPH_PI_BOUNDARY equals the fused
    symmetric launch to FP32 rounding (bitwise for the boundary targets)."""
    import torch

    from paper_1110_3711_amd import sph

    lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=78)
    print("symmetric split vs fused dam_break_8k+v", flush=True)
    sim = _sim(lay)
    ace_a, visc_a, np_a = _interact(sim, sph.SPH_PI_ALL | sph.SPH_PI_SYMMETRIC)
    np_s = torch.zeros(2, dtype=torch.int64, device=sim.device)
    sim.ace.fill_(7.0)
    sim.visc.fill_(7.0)
    sim.interact(parts=sph.SPH_PI_FLUID | sph.SPH_PI_SYMMETRIC, npairs=np_s)
    sim.interact(parts=sph.SPH_PI_BOUNDARY, npairs=np_s)
    torch.cuda.synchronize()
    assert torch.equal(visc_a, sim.visc)
    assert rel_l2(sim.ace.cpu().numpy(), ace_a.cpu().numpy()) <= 1e-6
    assert torch.equal(ace_a[: lay.nb], sim.ace[: lay.nb])
    assert np.array_equal(np_a, np_s.cpu().numpy())


def test_symmetric_1m_matches_gather(ora):
    """The 1.65M-particle dam break with seeded velocities against the gather
    kernel on the same state: forces within 1e-5, visc within 1e-6, the same
    boundary-target pair count, and fluid-target counts that differ only by
    pairs within rounding of the cutoff (the oracle subset check at this size
    is in test_gpu_large)."""
    from paper_1110_3711_amd import sph

    lay = named_case("dam_break_1m")
    rng = np.random.default_rng(21)
    lay.v = lay.v + rng.normal(0.0, 0.05, lay.v.shape)
    lay.v[: lay.nb] = 0.0
    print(f"symmetric dam_break_1m sampled n={lay.n}", flush=True)
    sim = _sim(lay)
    ace_g, visc_g, np_g = _interact(sim, sph.SPH_PI_ALL)
    ace_s, visc_s, np_s = _interact(sim, sph.SPH_PI_ALL | sph.SPH_PI_SYMMETRIC)
    print(f"  pairs: gather {np_g.tolist()} symmetric {np_s.tolist()}", flush=True)
    assert np_g[1] == np_s[1] and abs(int(np_g[0]) - int(np_s[0])) <= 1e-6 * int(np_g[0])
    assert rel_l2(visc_s.cpu().numpy(), visc_g.cpu().numpy()) <= 1e-6
    ag = sim.by_id(ace_g)
    asym = sim.by_id(ace_s)
    f = slice(lay.nb, None)
    e_a = rel_l2(asym[f, :3], ag[f, :3])
    e_d = rel_l2(asym[:, 3], ag[:, 3])
    print(f"  rel L2 vs gather: acc {e_a:.2e} drho {e_d:.2e}", flush=True)
    assert e_a <= 1e-5 and e_d <= 1e-5
