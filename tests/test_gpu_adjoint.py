"""GPU adjoint against the FP64 oracle.

* sph_interact_backward vs the oracle's VJP on the same encoded state and the
  same seeded adjoint input (relative L2 per output).
* sph_step(SPH_ADJOINT) vs the oracle's Verlet transpose.
* Rollout gradients (alpha and initial fluid velocities, checkpoint every C
  steps) vs central finite differences of the FP64 oracle rollout with the
  same frozen time steps: <= 1e-3 relative.
"""

import numpy as np
import pytest

from _helpers import compress, grid_tuple, oracle_view, parity, rel_l2
from sph_inputs import dam_break, named_case

pytestmark = pytest.mark.gpu


def _case(seed=3, dp=0.02, vel=0.3, rho_sigma=2.0):
    L = dam_break(dp, seed, fluid=(0.12, 0.12, 0.12), tank=(0.2, 0.14, 0.14),
                  vel_sigma=vel, vel_seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    L.rho = L.rho + rng.normal(0, rho_sigma, L.n)
    L.rho[: L.nb] = np.abs(L.rho[: L.nb] - L.phys.rho0) + L.phys.rho0
    return L


def _oracle_state(ora, lay, sim):
    return oracle_view(ora, lay.x, lay.v, lay.rho, lay.phys.rho0, grid_tuple(sim), lay.lo, lay.hi)


@pytest.mark.parametrize("which", ["small", "dam_break_8k", "dam_break_8k_nsub2", "compressed"])
def test_interact_backward_matches_oracle(ora, which):
    import torch

    from paper_1110_3711_amd import sph

    if which == "small":
        lay = _case()
    elif which == "compressed":  # stencils over several adjoint staging tiles
        lay = compress(_case(dp=0.01), 0.5)
    else:
        lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=9)
    print(f"interact_backward {which} n={lay.n}", flush=True)
    sim = sph.Simulation(lay, nsub=2 if which.endswith("nsub2") else 1)
    sim.build_cells()
    rng = np.random.default_rng(21)
    w = rng.normal(size=(lay.n, 4))
    w[: lay.nb, :3] = 0.0
    ids = sim.a.id.long()
    wd = torch.as_tensor(w, dtype=torch.float32, device=sim.device)[ids].contiguous()
    xb = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
    vb = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
    ab = torch.zeros(1, dtype=torch.float64, device=sim.device)
    sph.sph_interact_backward(sim.grid, sim.params, sim.a.c(), sim.cells(), wd, xb, vb, ab,
                              sim.ws)
    torch.cuda.synchronize()
    gx = sim.by_id(xb)
    gv = sim.by_id(vb)
    xq, vq, rq, excl, _, _ = _oracle_state(ora, lay, sim)
    w32 = w.astype(np.float32).astype(np.float64)
    oxb, ovb, orb, oab = ora.interact_vjp(xq, vq, rq, lay.nb, ora.params(lay.phys), w32, excl)
    f = slice(lay.nb, None)
    parity(f"VJP {which}", xbar=(gx[f, :3], oxb[f]), vbar=(gv[f, :3], ovb[f]),
           rhobar=(gv[:, 3], orb))
    ex = rel_l2(gx[f, :3], oxb[f])
    ev = rel_l2(gv[f, :3], ovb[f])
    er = rel_l2(gv[:, 3], orb)
    ea = abs(ab.item() - oab) / abs(oab)
    print(f"  rel L2: xbar {ex:.2e} vbar {ev:.2e} rhobar {er:.2e} alphabar {ea:.2e}", flush=True)
    assert ex <= 1e-4 and ev <= 1e-4 and er <= 1e-4 and ea <= 1e-4
    assert np.all(gx[: lay.nb, :3] == 0) and np.all(gv[: lay.nb, :3] == 0)


@pytest.mark.parametrize("which", ["dam_break_8k", "compressed"])
def test_interact_backward_deterministic(ora, which):
    """Three launches of the pair VJP on the same inputs are bitwise identical
    (no float atomics; alpha_bar is a fixed-order FP64 sum).  The compressed
    layout fills whole adjoint staging tiles with kept candidates."""
    import torch

    from paper_1110_3711_amd import sph

    if which == "compressed":
        lay = compress(_case(dp=0.01), 0.5)
    else:
        lay = dam_break(0.01, 11103711 + 1, vel_sigma=0.2, vel_seed=9)
    print(f"interact_backward determinism {which} n={lay.n}", flush=True)
    sim = sph.Simulation(lay, nsub=1)
    sim.build_cells()
    rng = np.random.default_rng(22)
    wd = torch.as_tensor(rng.normal(size=(lay.n, 4)), dtype=torch.float32, device=sim.device)
    outs = []
    for _ in range(3):
        xb = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
        vb = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
        ab = torch.zeros(1, dtype=torch.float64, device=sim.device)
        sph.sph_interact_backward(sim.grid, sim.params, sim.a.c(), sim.cells(), wd, xb, vb, ab,
                                  sim.ws)
        torch.cuda.synchronize()
        outs.append((xb, vb, ab))
    for later in outs[1:]:
        for u, v in zip(outs[0], later):
            assert torch.equal(u, v)


@pytest.mark.parametrize("step_index", [0, 7])
def test_verlet_adjoint_matches_oracle(ora, step_index):
    import torch

    from paper_1110_3711_amd import sph

    lay = _case(seed=8)
    rng = np.random.default_rng(13)
    vprev = lay.v + rng.normal(0, 0.01, lay.v.shape)
    vprev[: lay.nb] = 0
    rhoprev = lay.rho + rng.normal(0, 0.05, lay.n)
    rhoprev[: lay.nb] = lay.phys.rho0 + 1e-3
    print(f"verlet adjoint step={step_index}", flush=True)
    sim = sph.Simulation(lay, nsub=1)
    sim.upload_prev(vprev, rhoprev)
    sim.build_cells()
    sim.interact()
    dt = 2.5e-4
    sim.dt.fill_(dt)
    ids = sim.a.id.long()
    # seeded level-(n+1) adjoints, id order -> slot order
    xin = rng.normal(size=(lay.n, 3))
    vin = rng.normal(size=(lay.n, 4))
    pin = rng.normal(size=(lay.n, 4))

    def dev(a4):
        t = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
        t[:, : a4.shape[1]] = torch.as_tensor(a4, dtype=torch.float32, device=sim.device)
        return t[ids].contiguous()

    xb, vb, vpb = dev(xin), dev(vin), dev(pin)
    ab = torch.zeros((lay.n, 4), dtype=torch.float32, device=sim.device)
    adj = sph.Adjoint()
    adj.pos_bar, adj.velrho_bar, adj.velrho_prev_bar, adj.ace_bar = (
        xb.data_ptr(), vb.data_ptr(), vpb.data_ptr(), ab.data_ptr())
    sph.sph_step(sim.grid, sim.params, sim.a.c(), sim.ace, sim.visc, sim.dt, step_index,
                 sph.SPH_ADJOINT, sim.ws, sim.status, adj=adj)
    torch.cuda.synchronize()
    # oracle on the same encoded state
    xq, vq, rq, excl, _, _ = _oracle_state(ora, lay, sim)
    rpq = (rhoprev - lay.phys.rho0).astype(np.float32).astype(np.float64) + lay.phys.rho0
    P = ora.params(lay.phys)
    ace, *_ = ora.interact(xq, vq, rq, lay.nb, P, excl)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32).astype(np.float64)
    oxb, ovb, orb = f32(xin), f32(vin[:, :3]), f32(vin[:, 3])
    ovpb, orpb = f32(pin[:, :3]), f32(pin[:, 3])
    oab = ora.verlet_vjp(rq, rpq, ace, dt, step_index, lay.nb, P, excl, oxb, ovb, orb, ovpb, orpb)
    gab = sim.by_id(ab)
    f = slice(lay.nb, None)
    assert rel_l2(gab[f, :3], oab[f, :3]) <= 1e-6
    assert rel_l2(gab[:, 3], oab[:, 3]) <= 1e-6
    gvb = sim.by_id(vb)
    gvpb = sim.by_id(vpb)
    assert rel_l2(gvb[f, :3], ovb[f]) <= 1e-6
    assert rel_l2(gvb[:, 3], orb) <= 1e-6
    assert rel_l2(gvpb[f, :3], ovpb[f]) <= 1e-6
    assert rel_l2(gvpb[:, 3], orpb) <= 1e-6


def _centroid(xf, target):
    c = xf.mean(0)
    return ((c - target) ** 2).sum() / 3.0


def _gpu_grad(lay, K, C, dts, target, u_dirs):
    import torch

    from paper_1110_3711_amd.rollout import Rollout, SphRollout

    roll = Rollout(lay, K, C, nsub=1, dts=dts)
    alpha = torch.tensor(lay.phys.alpha, dtype=torch.float64, requires_grad=True)
    v0 = torch.as_tensor(lay.v[lay.nb:], dtype=torch.float64, device=roll.device)
    v0.requires_grad_(True)
    xk = SphRollout.apply(alpha, v0, roll)
    tgt = torch.as_tensor(target, dtype=torch.float64, device=roll.device)
    loss = ((xk.mean(0) - tgt) ** 2).sum() / 3.0
    loss.backward()
    ga = float(alpha.grad)
    gv = v0.grad.detach().cpu().numpy()
    return ga, [float((gv * u).sum()) for u in u_dirs], roll


def _oracle_fd(ora, lay, dts, target, u_dirs, eps_a=1e-4, eps_v=1e-6):
    def loss_of(alpha=None, v0=None):
        P = ora.params(lay.phys, alpha=lay.phys.alpha if alpha is None else alpha)
        vv = None
        if v0 is not None:
            vv = lay.v.copy()
            vv[lay.nb:] = v0
        _, S = ora.rollout(lay, dts, P, v0=vv)
        return _centroid(S.x[lay.nb:], target)

    a0 = lay.phys.alpha
    fa = (loss_of(alpha=a0 + eps_a) - loss_of(alpha=a0 - eps_a)) / (2 * eps_a)
    fv = []
    for u in u_dirs:
        vf = lay.v[lay.nb:]
        fv.append((loss_of(v0=vf + eps_v * u) - loss_of(v0=vf - eps_v * u)) / (2 * eps_v))
    return fa, fv


def test_rollout_gradient_small_fixed_dt(ora):
    lay = _case(seed=5, vel=0.2, rho_sigma=0.0)
    K, C = 24, 5
    dts = np.full(K, 2.0e-4)
    rng = np.random.default_rng(4)
    target = lay.x[lay.nb:].mean(0) + rng.uniform(-0.01, 0.01, 3)
    u_dirs = [rng.normal(size=(lay.nf, 3)) for _ in range(3)]
    print(f"rollout small n={lay.n} K={K} C={C}", flush=True)
    ga, gv, _ = _gpu_grad(lay, K, C, dts, target, u_dirs)
    fa, fv = _oracle_fd(ora, lay, dts, target, u_dirs)
    print(f"  alpha: gpu {ga:.6e} fd {fa:.6e}; v0: {list(zip(gv, fv))}", flush=True)
    assert ga == pytest.approx(fa, rel=1e-3)
    for g, fdv in zip(gv, fv):
        assert g == pytest.approx(fdv, rel=1e-3)


def test_rollout_gradient_64k_short(ora):
    """64k-fluid dam break (64,000 fluid particles, seeded initial velocities), 30 steps
    with a checkpoint every 10; each side freezes its own CFL time steps."""
    import torch

    lay = named_case("dam_break_64k")
    K, C = 30, 10
    rng = np.random.default_rng(11103711 + 4)
    target = lay.x[lay.nb:].mean(0) + rng.uniform(-0.01, 0.01, 3)
    u_dirs = [rng.normal(size=(lay.nf, 3))]
    print(f"rollout dam_break_64k n={lay.n} K={K} C={C}", flush=True)
    ga, gv, roll = _gpu_grad(lay, K, C, None, target, u_dirs)
    gpu_dts = roll.dts.cpu().numpy()
    S = ora.State(lay)
    dts = S.run(K)  # the oracle's own FP64 CFL time steps
    assert np.allclose(gpu_dts, dts, rtol=1e-4)
    fa, fv = _oracle_fd(ora, lay, dts, target, u_dirs)
    print(f"  alpha: gpu {ga:.6e} fd {fa:.6e}; v0: gpu {gv[0]:.6e} fd {fv[0]:.6e}", flush=True)
    assert ga == pytest.approx(fa, rel=1e-3)
    assert gv[0] == pytest.approx(fv[0], rel=1e-3)
    torch.cuda.synchronize()


@pytest.mark.timeout(1500)
def test_rollout_gradient_64k_full(ora):
    """The differentiable-rollout workload at full length: 64k-fluid dam break, K = 200
    steps, checkpoint every 20, each side with its own CFL time steps (frozen
    for the gradient); alpha and one seeded v0 direction vs central FD of the
    FP64 oracle rollout."""
    lay = named_case("dam_break_64k")
    K, C = 200, 20
    rng = np.random.default_rng(11103711 + 4)
    target = lay.x[lay.nb:].mean(0) + rng.uniform(-0.01, 0.01, 3)
    u_dirs = [rng.normal(size=(lay.nf, 3))]
    print(f"rollout dam_break_64k n={lay.n} K={K} C={C}", flush=True)
    ga, gv, roll = _gpu_grad(lay, K, C, None, target, u_dirs)
    gpu_dts = roll.dts.cpu().numpy()
    S = ora.State(lay)
    dts = S.run(K)
    print(f"  dt: gpu {gpu_dts[0]:.6e}..{gpu_dts[-1]:.6e}, oracle {dts[0]:.6e}..{dts[-1]:.6e}",
          flush=True)
    assert np.allclose(gpu_dts, dts, rtol=1e-3)
    fa, fv = _oracle_fd(ora, lay, dts, target, u_dirs)
    print(f"  alpha: gpu {ga:.6e} fd {fa:.6e} rel {abs(ga - fa) / abs(fa):.2e}; "
          f"v0: gpu {gv[0]:.6e} fd {fv[0]:.6e} rel {abs(gv[0] - fv[0]) / abs(fv[0]):.2e}",
          flush=True)
    assert ga == pytest.approx(fa, rel=1e-3)
    assert gv[0] == pytest.approx(fv[0], rel=1e-3)


def test_rollout_gradient_vector_matches_oracle_adjoint(ora):
    """Whole gradient vectors on the 64k-fluid dam break: 5 steps with a fixed
    time step, checkpoint every 2 (three segments); GPU dL/dv0 (every fluid
    particle and component) and dL/dalpha against the FP64 oracle's own
    reverse pass over its FP64 rollout (relative L2 <= 1e-3)."""
    import torch

    lay = named_case("dam_break_64k")
    K, C = 5, 2
    dts = np.full(K, 1.4e-4)
    rng = np.random.default_rng(11103711 + 4)
    target = lay.x[lay.nb:].mean(0) + rng.uniform(-0.01, 0.01, 3)
    print(f"rollout vector dam_break_64k n={lay.n} K={K} C={C}", flush=True)
    from paper_1110_3711_amd.rollout import Rollout, SphRollout

    roll = Rollout(lay, K, C, nsub=1, dts=dts)
    alpha = torch.tensor(lay.phys.alpha, dtype=torch.float64, requires_grad=True)
    v0 = torch.as_tensor(lay.v[lay.nb:], dtype=torch.float64, device=roll.device)
    v0.requires_grad_(True)
    xk = SphRollout.apply(alpha, v0, roll)
    tgt = torch.as_tensor(target, dtype=torch.float64, device=roll.device)
    loss = ((xk.mean(0) - tgt) ** 2).sum() / 3.0
    loss.backward()
    ga = float(alpha.grad)
    gv = v0.grad.detach().cpu().numpy()

    P = ora.params(lay.phys)
    tape, S = ora.rollout(lay, dts, P)
    c = S.x[lay.nb:].mean(0)
    xbar = np.zeros((lay.n, 3))
    xbar[lay.nb:] = 2.0 / 3.0 * (c - target) / lay.nf
    vbar0, abar = ora.rollout_vjp(lay, tape, dts, P, xbar)
    ev = rel_l2(gv, vbar0[lay.nb:])
    ea = abs(ga - abar) / abs(abar)
    print(f"  dL/dv0 rel L2 {ev:.2e}; dL/dalpha gpu {ga:.6e} oracle {abar:.6e} rel {ea:.2e}",
          flush=True)
    assert ev <= 1e-3 and ea <= 1e-3
