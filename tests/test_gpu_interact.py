"""sph_interact on the GPU against the FP64 oracle on the same encoded state.

* Neighbour sets: per-target count and id hash lie between the oracle's FP64
  cell-list sets at the cutoff moved by -1e-5 and +1e-5 (relative, in r^2):
  exact for every target without a pair in that tie band.
* Forces: relative L2 <= 1e-4 and per-target error <= 1e-3 of the rms for
  fluid accelerations, drho/dt and visc.
* Determinism: two launches are bitwise identical.
"""

import dataclasses

import numpy as np
import pytest

from _helpers import band_sets, check_sets_in_band, compress, grid_tuple, oracle_view, parity
from sph_inputs import blob, dam_break, named_case

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _run(lay, nsub, stats=False):
    import torch

    from paper_1110_3711_amd import sph

    sim = sph.Simulation(lay, nsub=nsub)
    sim.build_cells()
    st = torch.zeros(2 * lay.n, dtype=torch.int32, device=sim.device) if stats else None
    sim.npairs.zero_()
    sim.interact(stats=st)
    torch.cuda.synchronize()
    return sim, st


def _compare_forces(ora, lay, sim, tol=TOL):
    gt = grid_tuple(sim)
    xq, vq, rq, excl, _, _ = oracle_view(ora, lay.x, lay.v, lay.rho, lay.phys.rho0, gt, lay.lo,
                                         lay.hi)
    ref, rvisc, _, npairs = ora.interact(xq, vq, rq, lay.nb, ora.params(lay.phys), excl=excl)
    ace = sim.by_id(sim.ace)
    visc = sim.by_id(sim.visc)
    f = np.arange(lay.nb, lay.n)
    f = f[excl[f] == 0]
    parity(f"{lay.name} n={lay.n}", tol=tol, acc=(ace[f, :3], ref[f, :3]),
           drho=(ace[:, 3], ref[:, 3]), visc=(visc, rvisc))
    assert np.all(ace[excl == 1] == 0)
    assert np.all(ace[: lay.nb, :3] == 0) and np.all(visc[: lay.nb] == 0)
    return npairs


@pytest.mark.parametrize("nsub", [1, 2])
def test_neighbour_sets_within_tie_band(ora, nsub):
    lay = named_case("dam_break_8k")
    print(f"interact stats dam_break_8k nsub={nsub}", flush=True)
    sim, st = _run(lay, nsub, stats=True)
    gt = grid_tuple(sim)
    xq, _, _, excl, _, _ = oracle_view(ora, lay.x, lay.v, lay.rho, lay.phys.rho0, gt, lay.lo,
                                       lay.hi)
    inner, outer = band_sets(ora, xq, lay.nb, lay.phys.h, excl=excl)
    s = sim.by_id(st.view(-1, 2))
    tied, nband = check_sets_in_band(s[:, 0], s[:, 1].view(np.uint32), inner, outer)
    total = int(sim.npairs.sum().item())
    print(f"  {total:,} directed pairs; {nband} FP64 pairs in the tie band on {tied} targets",
          flush=True)
    assert int(s[:, 0].sum()) == total
    assert inner[0][-1] <= total <= outer[0][-1]


@pytest.mark.parametrize("nsub", [1, 2])
def test_forces_8k_moving(ora, nsub):
    lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=77)
    print(f"interact forces dam_break_8k+v nsub={nsub}", flush=True)
    sim, _ = _run(lay, nsub)
    _compare_forces(ora, lay, sim)


def test_forces_8k_rest(ora):
    lay = named_case("dam_break_8k")
    print("interact forces dam_break_8k rest", flush=True)
    sim, _ = _run(lay, 1)
    gt = grid_tuple(sim)
    xq, vq, rq, excl, _, _ = oracle_view(ora, lay.x, lay.v, lay.rho, lay.phys.rho0, gt, lay.lo,
                                         lay.hi)
    ref, rvisc, _, _ = ora.interact(xq, vq, rq, lay.nb, ora.params(lay.phys), excl=excl)
    ace = sim.by_id(sim.ace)
    f = slice(lay.nb, None)
    parity("dam_break_8k rest", acc=(ace[f, :3], ref[f, :3]))
    assert np.all(ace[:, 3] == 0) and np.all(ref[:, 3] == 0)  # at rest: no density change


def test_forces_blob_with_excluded(ora):
    lay = blob(20, 0.01, 4, vel_sigma=0.3, jitter=0.3)
    lay.x[:50, 0] = lay.hi[0] + 1.0  # outside the domain: excluded
    print("interact forces blob", flush=True)
    sim, _ = _run(lay, 1)
    _compare_forces(ora, lay, sim)


def test_forces_compressed_several_tiles(ora):
    # the 1,728-fluid dam break with positions pulled together by 0.5 (8x the
    # lattice density): the stencils hold some 4,000 candidates (two or three
    # staging tiles) and boundary cells hundreds of targets, beyond the ones
    # staged in LDS
    lay = compress(dam_break(0.01, 7, fluid=(0.12, 0.12, 0.12), tank=(0.2, 0.14, 0.14),
                             vel_sigma=0.2, vel_seed=5), 0.5)
    print(f"interact forces compressed dam break n={lay.n}", flush=True)
    sim, _ = _run(lay, 1)
    cells = sim.start.cpu().numpy()
    assert np.diff(cells[: sim.ncell + 1]).max() > 128  # a boundary cell beyond the staged targets
    _compare_forces(ora, lay, sim)


@pytest.mark.parametrize("which", ["dam_break_8k", "dam_break_8k_nsub2", "compressed",
                                   "cubic_tensile"])
def test_range_table_path_bitwise(ora, which):
    """With the precomputed interaction ranges the pair kernels read each
    cell's runs from its row: forces, visc, pair counts and the pair VJP are
    bitwise those of the default path (and within the bar of the oracle)."""
    import torch

    from paper_1110_3711_amd import sph

    if which == "compressed":
        lay = compress(dam_break(0.01, 7, fluid=(0.12, 0.12, 0.12), tank=(0.2, 0.14, 0.14),
                                 vel_sigma=0.2, vel_seed=5), 0.5)
    else:
        lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=77)
    if which == "cubic_tensile":
        lay.phys = dataclasses.replace(lay.phys, kernel=1, alpha=0.25, tensile_dp=lay.phys.dp)
    nsub = 2 if which.endswith("nsub2") else 1
    print(f"interact range table {which} n={lay.n}", flush=True)
    out = []
    for ranges in (False, True):
        sim = sph.Simulation(lay, nsub=nsub, ranges=ranges)
        sim.build_cells()
        sim.npairs.zero_()
        sim.interact()
        rng = np.random.default_rng(21)
        w = torch.as_tensor(rng.normal(size=(lay.n, 4)), dtype=torch.float32,
                            device=sim.device)[sim.a.id.long()].contiguous()
        xb = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
        vb = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
        ab = torch.zeros(1, dtype=torch.float64, device=sim.device)
        sph.sph_interact_backward(sim.grid, sim.params, sim.a.c(), sim.cells(), w, xb, vb, ab,
                                  sim.ws)
        torch.cuda.synchronize()
        out.append((sim, sim.ace.clone(), sim.visc.clone(), sim.npairs.clone(), xb, vb, ab))
    (_, *a), (sim_rt, *b) = out
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    _compare_forces(ora, lay, sim_rt)


def test_momentum_conservation_gpu(ora):
    # pair forces are antisymmetric; the sum of the FP32 internal forces over a
    # free blob (no gravity, no boundary) vanishes to FP32 rounding
    lay = blob(16, 0.01, 8, vel_sigma=0.3, jitter=0.3)
    print("interact momentum blob", flush=True)
    sim, _ = _run(lay, 1)
    a = sim.by_id(sim.ace)[:, :3].astype(np.float64)
    res = np.abs(a.sum(0)).max() / np.abs(a).sum()
    print(f"  |sum m a| / sum |m a| = {res:.2e}", flush=True)
    assert res <= 1e-6


@pytest.mark.parametrize("which", ["dam_break", "compressed"])
def test_determinism(ora, which):
    """Repeated launches are bitwise identical, also on the compressed layout,
    whose stencils span several staging tiles filled with kept candidates."""
    import torch

    if which == "compressed":
        lay = compress(dam_break(0.01, 7, fluid=(0.12, 0.12, 0.12), tank=(0.2, 0.14, 0.14),
                                 vel_sigma=0.2, vel_seed=5), 0.4)
    else:
        lay = dam_break(0.01, 5, vel_sigma=0.2)
    print(f"interact determinism {which} n={lay.n}", flush=True)
    sim, _ = _run(lay, 1)
    a1 = sim.ace.clone()
    v1 = sim.visc.clone()
    for _ in range(3):
        sim.interact()
        torch.cuda.synchronize()
        assert torch.equal(a1, sim.ace) and torch.equal(v1, sim.visc)


def test_split_parts_match_fused_launch(ora):
    """SPH_PI_FLUID then SPH_PI_BOUNDARY (two launches) and SPH_PI_ALL (one
    fused launch) give bitwise identical outputs and the same pair counts."""
    import torch

    from paper_1110_3711_amd import sph

    lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=78)
    print("interact split vs fused dam_break_8k+v", flush=True)
    sim = sph.Simulation(lay, nsub=1)
    sim.build_cells()
    st_a = torch.zeros(2 * lay.n, dtype=torch.int32, device=sim.device)
    np_a = torch.zeros(2, dtype=torch.int64, device=sim.device)
    sim.interact(stats=st_a, parts=sph.SPH_PI_ALL, npairs=np_a)
    ace_a, visc_a = sim.ace.clone(), sim.visc.clone()
    sim.ace.fill_(7.0)
    sim.visc.fill_(7.0)
    st_s = torch.zeros_like(st_a)
    np_s = torch.zeros(2, dtype=torch.int64, device=sim.device)
    sim.interact(stats=st_s, parts=sph.SPH_PI_FLUID, npairs=np_s)
    sim.interact(stats=st_s, parts=sph.SPH_PI_BOUNDARY, npairs=np_s)
    torch.cuda.synchronize()
    assert torch.equal(ace_a, sim.ace) and torch.equal(visc_a, sim.visc)
    assert torch.equal(st_a, st_s)
    assert torch.equal(np_a, np_s) and int(np_a[1]) > 0
