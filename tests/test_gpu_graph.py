"""One whole step (sph_build_cells -> sph_interact -> sph_step) captured in a
HIP graph through torch and replayed: the library enqueues only kernels on
the caller's stream (no allocation, no memset), so every replay must give
bitwise the step's eager result.  Replays alternate with eager work and
synchronisations, and each one is checked."""

import pytest

from sph_inputs import SEED_BASE, dam_break

pytestmark = pytest.mark.gpu


def _snapshot(sim):
    return [t.clone() for t in (sim.a.cell, sim.a.pos, sim.a.velrho, sim.a.velrho_prev, sim.a.id)]


def _restore(sim, snap):
    for t, s in zip((sim.a.cell, sim.a.pos, sim.a.velrho, sim.a.velrho_prev, sim.a.id), snap):
        t.copy_(s)


def _result(sim):
    # the current side after a step (build_cells swaps the two sides)
    return [t.clone() for t in (sim.a.cell, sim.a.pos, sim.a.velrho, sim.a.velrho_prev, sim.a.id,
                                sim.ace, sim.visc, sim.dt)]


def test_step_graph_replays_match_eager():
    import torch

    from paper_1110_3711_amd import sph

    lay = dam_break(0.02, SEED_BASE + 11, vel_sigma=0.1, vel_seed=SEED_BASE + 110)
    print(f"graph: n={lay.n}", flush=True)
    sim = sph.Simulation(lay, nsub=1)
    for _ in range(3):  # a few eager steps first (warm-up of every kernel)
        sim.step()
    torch.cuda.synchronize()
    a0, b0 = sim.a, sim.b
    snap = _snapshot(sim)
    k0 = sim.step_index

    # eager reference of one step from the snapshot
    sim.step()
    torch.cuda.synchronize()
    ref = _result(sim)
    sim.a, sim.b, sim.step_index = a0, b0, k0
    _restore(sim, snap)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            sim.build_cells()
            sim.interact(npairs=None)
            sim.update()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # capture only recorded the work; the buffers now hold the captured side
    sim.step_index = k0
    for rep in range(4):
        # the graph reads a0 and writes b0, whatever side Python holds as current
        for t, sv in zip((a0.cell, a0.pos, a0.velrho, a0.velrho_prev, a0.id), snap):
            t.copy_(sv)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in (b0.cell, b0.pos, b0.velrho, b0.velrho_prev, b0.id,
                                   sim.ace, sim.visc, sim.dt)]
        for u, v in zip(ref, got):
            assert torch.equal(u, v), f"replay {rep} differs from the eager step"
        # eager work between replays
        x = torch.randn(1000, device=sim.device)
        float((x * x).sum().item())
    assert sim.dev_status() == 0
    print("  4 replays bitwise equal to the eager step", flush=True)
