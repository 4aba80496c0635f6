"""The Python binding refuses device arrays the C ABI cannot check itself
(wrong dtype, too small, not contiguous, not on the device) before any
kernel is enqueued; a valid call afterwards still works."""

import pytest

from sph_inputs import dam_break

pytestmark = pytest.mark.gpu


def test_binding_rejects_bad_device_arrays():
    import torch

    from paper_1110_3711_amd import sph

    lay = dam_break(0.02, 11103711 + 9)
    print(f"binding checks n={lay.n}", flush=True)
    sim = sph.Simulation(lay, nsub=1)
    sim.build_cells()
    n = lay.n
    dev = sim.device
    good = dict(ace=sim.ace, visc=sim.visc, npairs=sim.npairs)
    bad = [
        ("ace", torch.empty((n, 4), dtype=torch.float64, device=dev)),       # dtype
        ("ace", torch.empty((n - 1, 4), dtype=torch.float32, device=dev)),   # too small
        ("ace", torch.empty((4, n), dtype=torch.float32, device=dev).t()),   # not contiguous
        ("ace", torch.empty((n, 4), dtype=torch.float32)),                   # host memory
        ("visc", torch.empty(n - 1, dtype=torch.float32, device=dev)),
        ("npairs", torch.zeros(1, dtype=torch.int64, device=dev)),
    ]
    for name, t in bad:
        args = dict(good)
        args[name] = t
        with pytest.raises(sph.SphError):
            sph.sph_interact(sim.grid, sim.params, sim.a.c(), sim.cells(), args["ace"],
                             args["visc"], args["npairs"], sim.ws)
    with pytest.raises(sph.SphError):
        sph.sph_step(sim.grid, sim.params, sim.a.c(), sim.ace, sim.visc,
                     torch.zeros(1, dtype=torch.float32, device=dev), 0, 0, sim.ws, sim.status)
    sim.interact()
    sim.update()
    torch.cuda.synchronize()
    assert sim.dev_status() == 0
