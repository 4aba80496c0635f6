"""Tensile correction on the GPU (sph_params.tensile_dp = dp) against the FP64
oracle on the same encoded state: forces <= 1e-4 relative L2 for both kernel
shapes, the pair VJP <= 1e-4, and rollout gradients vs central differences
of the oracle <= 1e-3.  Densities are perturbed around rho0 so that both
pressure signs (both branches of R) occur."""

import dataclasses

import numpy as np
import pytest

from _helpers import grid_tuple, oracle_view, parity, rel_l2
from sph_inputs import SEED_BASE, dam_break

pytestmark = pytest.mark.gpu


def _layout(kernel=0, dp=0.01, seed=SEED_BASE + 1, vel=0.2, vel_seed=79, rho_sigma=3.0, **kw):
    L = dam_break(dp, seed, vel_sigma=vel, vel_seed=vel_seed, kernel=kernel, name="tensile", **kw)
    L.phys = dataclasses.replace(L.phys, tensile_dp=dp)
    rng = np.random.default_rng(seed + 7)
    L.rho = L.rho + rng.normal(0, rho_sigma, L.n)
    L.rho[: L.nb] = np.abs(L.rho[: L.nb] - L.phys.rho0) + L.phys.rho0
    return L


@pytest.mark.parametrize("kernel,nsub", [(0, 1), (1, 1), (0, 2)],
                         ids=["wendland", "cubic", "wendland_nsub2"])
def test_tensile_forces_match_oracle(ora, kernel, nsub):
    import torch

    from paper_1110_3711_amd import sph

    lay = _layout(kernel)
    print(f"tensile interact kernel={kernel} nsub={nsub} n={lay.n}", flush=True)
    sim = sph.Simulation(lay, nsub=nsub)
    sim.build_cells()
    sim.npairs.zero_()
    sim.interact()
    torch.cuda.synchronize()
    xq, vq, rq, excl, _, _ = oracle_view(ora, lay.x, lay.v, lay.rho, lay.phys.rho0,
                                         grid_tuple(sim), lay.lo, lay.hi)
    P = ora.params(lay.phys)
    assert P.tensile_dp == lay.phys.dp
    ref, rvisc, _, npairs = ora.interact(xq, vq, rq, lay.nb, P, excl=excl)
    ace, visc = sim.by_id(sim.ace), sim.by_id(sim.visc)
    f = np.arange(lay.nb, lay.n)
    parity(f"tensile kernel={kernel} nsub={nsub}", acc=(ace[f, :3], ref[f, :3]),
           drho=(ace[:, 3], ref[:, 3]), visc=(visc, rvisc))
    e_a = rel_l2(ace[f, :3], ref[f, :3])
    e_d = rel_l2(ace[:, 3], ref[:, 3])
    e_v = rel_l2(visc, rvisc)
    off, *_ = ora.interact(xq, vq, rq, lay.nb, ora.params(lay.phys, tensile_dp=0.0), excl=excl)
    e_off = rel_l2(ace[f, :3], off[f, :3])
    print(f"  rel L2: acc {e_a:.2e} drho {e_d:.2e} visc {e_v:.2e}; vs tensile off {e_off:.2e}",
          flush=True)
    assert e_a <= 1e-4 and e_d <= 1e-4 and e_v <= 1e-4
    assert e_off > 1e-3  # the correction reached the kernel
    assert int(sim.npairs.sum().item()) == npairs


@pytest.mark.parametrize("kernel,nsub", [(0, 1), (1, 1), (1, 2)],
                         ids=["wendland", "cubic", "cubic_nsub2"])
def test_tensile_interact_backward_matches_oracle(ora, kernel, nsub):
    import torch

    from paper_1110_3711_amd import sph

    lay = _layout(kernel, dp=0.02, seed=3, vel=0.3, vel_seed=4, rho_sigma=2.0,
                  fluid=(0.12, 0.12, 0.12), tank=(0.2, 0.14, 0.14))
    print(f"tensile interact_backward kernel={kernel} nsub={nsub} n={lay.n}", flush=True)
    sim = sph.Simulation(lay, nsub=nsub)
    sim.build_cells()
    rng = np.random.default_rng(21)
    w = rng.normal(size=(lay.n, 4))
    w[: lay.nb, :3] = 0.0
    ids = sim.a.id.long()
    wd = torch.as_tensor(w, dtype=torch.float32, device=sim.device)[ids].contiguous()
    xb = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
    vb = torch.zeros_like(xb)
    ab = torch.zeros(1, dtype=torch.float64, device=sim.device)
    sph.sph_interact_backward(sim.grid, sim.params, sim.a.c(), sim.cells(), wd, xb, vb, ab,
                              sim.ws)
    torch.cuda.synchronize()
    xq, vq, rq, excl, _, _ = oracle_view(ora, lay.x, lay.v, lay.rho, lay.phys.rho0,
                                         grid_tuple(sim), lay.lo, lay.hi)
    w32 = w.astype(np.float32).astype(np.float64)
    oxb, ovb, orb, oab = ora.interact_vjp(xq, vq, rq, lay.nb, ora.params(lay.phys), w32, excl)
    gx, gv = sim.by_id(xb), sim.by_id(vb)
    fs = slice(lay.nb, None)
    parity(f"tensile VJP kernel={kernel} nsub={nsub}", xbar=(gx[fs, :3], oxb[fs]),
           vbar=(gv[fs, :3], ovb[fs]), rhobar=(gv[:, 3], orb))
    ex, ev = rel_l2(gx[fs, :3], oxb[fs]), rel_l2(gv[fs, :3], ovb[fs])
    er, ea = rel_l2(gv[:, 3], orb), abs(ab.item() - oab) / abs(oab)
    print(f"  rel L2: xbar {ex:.2e} vbar {ev:.2e} rhobar {er:.2e} alphabar {ea:.2e}", flush=True)
    assert ex <= 1e-4 and ev <= 1e-4 and er <= 1e-4 and ea <= 1e-4


def test_tensile_rollout_gradient(ora):
    import torch

    from paper_1110_3711_amd.rollout import Rollout, SphRollout

    lay = _layout(0, dp=0.02, seed=5, vel=0.2, vel_seed=6, rho_sigma=0.0,
                  fluid=(0.12, 0.12, 0.12), tank=(0.2, 0.14, 0.14))
    K, C = 20, 5
    dts = np.full(K, 2.0e-4)
    rng = np.random.default_rng(7)
    target = lay.x[lay.nb:].mean(0) + rng.uniform(-0.01, 0.01, 3)
    u = rng.normal(size=(lay.nf, 3))
    print(f"tensile rollout n={lay.n} K={K} C={C}", flush=True)
    roll = Rollout(lay, K, C, nsub=1, dts=dts)
    alpha = torch.tensor(lay.phys.alpha, dtype=torch.float64, requires_grad=True)
    v0 = torch.as_tensor(lay.v[lay.nb:], dtype=torch.float64, device=roll.device)
    v0.requires_grad_(True)
    xk = SphRollout.apply(alpha, v0, roll)
    tgt = torch.as_tensor(target, dtype=torch.float64, device=roll.device)
    loss = ((xk.mean(0) - tgt) ** 2).sum() / 3.0
    loss.backward()
    ga = float(alpha.grad)
    gv = float((v0.grad.detach().cpu().numpy() * u).sum())

    def loss_of(alpha_v, v0f):
        P = ora.params(lay.phys, alpha=alpha_v)
        vv = lay.v.copy()
        vv[lay.nb:] = v0f
        _, S = ora.rollout(lay, dts, P, v0=vv)
        c = S.x[lay.nb:].mean(0)
        return ((c - target) ** 2).sum() / 3.0

    a0, vf = lay.phys.alpha, lay.v[lay.nb:]
    fa = (loss_of(a0 + 1e-4, vf) - loss_of(a0 - 1e-4, vf)) / 2e-4
    fv = (loss_of(a0, vf + 1e-6 * u) - loss_of(a0, vf - 1e-6 * u)) / 2e-6
    print(f"  alpha: gpu {ga:.6e} fd {fa:.6e}; v0: gpu {gv:.6e} fd {fv:.6e}", flush=True)
    assert ga == pytest.approx(fa, rel=1e-3)
    assert gv == pytest.approx(fv, rel=1e-3)
