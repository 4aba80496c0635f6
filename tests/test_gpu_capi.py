"""The library driven from plain C: ``paper_1110_3711_amd/sph_run`` (built from
``csrc/sph_run.c`` by the package build, host code that calls only the C ABI
and the HIP runtime) runs whole steps on an input file.  Its final state must
be bitwise the state the Python binding reaches from the same input."""

import os
import struct
import subprocess

import numpy as np
import pytest

from sph_inputs import SEED_BASE, dam_break

pytestmark = pytest.mark.gpu

RUNNER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_1110_3711_amd", "sph_run")


def _write_input(path, lay, grid, params, steps):
    with open(path, "wb") as f:
        f.write(struct.pack("<3i", lay.n, lay.nb, steps))
        f.write(struct.pack("<7d", *grid.origin, *grid.hi, grid.cell))
        f.write(struct.pack("<4i", *grid.nc, grid.nsub))
        f.write(struct.pack("<11d", params.h, params.rho0, params.gamma, params.c0, params.alpha,
                            params.eta2, *params.g, params.mass, params.cfl))
        f.write(struct.pack("<3i", params.kernel, params.verlet_ns, params.bound_floor))
        f.write(struct.pack("<d", params.tensile_dp))
        for a in (lay.x, lay.v, lay.rho):
            f.write(np.ascontiguousarray(a, dtype="<f8").tobytes())


@pytest.mark.parametrize("steps", [1, 60])
def test_c_program_matches_binding(tmp_path, steps):
    import torch

    from paper_1110_3711_amd import sph

    assert os.access(RUNNER, os.X_OK), f"{RUNNER} is not built (run the package build)"
    lay = dam_break(0.02, SEED_BASE + 9, vel_sigma=0.1, vel_seed=SEED_BASE + 90)
    sim = sph.Simulation(lay, nsub=1)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    _write_input(inp, lay, sim.grid, sim.params, steps)
    print(f"capi: sph_run n={lay.n} steps={steps}", flush=True)
    res = subprocess.run([RUNNER, str(inp), str(out)], capture_output=True, text=True,
                         timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    n = lay.n
    raw = out.read_bytes()
    assert len(raw) == 8 * (7 * n + 1) + 4
    arr = np.frombuffer(raw[: 8 * (7 * n + 1)], dtype="<f8")
    cx = arr[: 3 * n].reshape(n, 3)
    cv = arr[3 * n: 6 * n].reshape(n, 3)
    cr = arr[6 * n: 7 * n]
    ct = arr[7 * n]
    (cstatus,) = struct.unpack("<i", raw[-4:])

    tsum = torch.zeros(1, dtype=torch.float64, device=sim.device)
    for _ in range(steps):
        sim.step()
        tsum += sim.dt
    torch.cuda.synchronize()
    x, v, r = sim.decode()
    print(f"  t {ct:.9g} / {float(tsum.item()):.9g}", flush=True)
    assert cstatus == sim.dev_status() == 0
    assert np.array_equal(cx, x) and np.array_equal(cv, v) and np.array_equal(cr, r)
    assert ct == float(tsum.item())
