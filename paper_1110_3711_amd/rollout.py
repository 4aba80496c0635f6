"""Differentiable rollout: K Verlet steps with checkpoint-and-recompute.

Forward: K whole steps (sph_build_cells -> sph_interact -> sph_step) on the
device; the state is checkpointed every C steps and the time-step sequence is
recorded (or taken from the caller) and then held fixed.  Backward: for each
segment, newest first, restore its checkpoint, replay its C steps with the
recorded time steps while keeping each step's sorted state, permutation, cell
arrays and (a, D), then walk the segment backwards:

    sph_step(SPH_ADJOINT)        transpose of the Verlet update
    sph_interact_backward        VJP of the pair interaction (+= into the adjoints)
    sph_build_cells_backward     transpose of the reorder

Every step runs in the HIP library; this module only sequences the calls and
holds the device buffers.  ``SphRollout`` wraps the driver as a
``torch.autograd.Function`` with inputs (alpha, initial fluid velocities) and
output the fluid positions at step K (FP64, id order).
"""

from __future__ import annotations

import numpy as np

from . import sph


class _Tape:
    """Device buffers of one replayed step, allocated once and reused by every
    segment: the sorted state before the Verlet update (written directly by
    sph_build_cells), its cell arrays and permutation, and its (a, D)."""

    def __init__(self, sim):
        import torch

        n, dev = sim.n, sim.device
        self.st = sph.DeviceState(n, sim.nb, dev)
        self.start = torch.empty(2 * sim.ncell + 2, dtype=torch.int32, device=dev)
        self.list = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self.info = torch.zeros(4, dtype=torch.int32, device=dev)
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self.ace = torch.empty((max(n, 1), 4), dtype=torch.float32, device=dev)
        c = sph.Cells()
        c.start, c.list, c.info = self.start.data_ptr(), self.list.data_ptr(), self.info.data_ptr()
        self._cells = c

    def state(self) -> sph.State:
        return self.st.c()

    def cells(self) -> sph.Cells:
        return self._cells


def _adjoint_struct(xb, vb, vpb, ab) -> sph.Adjoint:
    A = sph.Adjoint()
    A.pos_bar = xb.data_ptr()
    A.velrho_bar = vb.data_ptr()
    A.velrho_prev_bar = vpb.data_ptr()
    A.ace_bar = 0 if ab is None else ab.data_ptr()
    return A


class Rollout:
    """Checkpointed forward/backward driver for one layout."""

    def __init__(self, layout, steps: int, checkpoint_every: int, nsub: int = 1,
                 device="cuda:0", dts=None):
        import torch

        if steps < 1 or checkpoint_every < 1:
            raise ValueError("steps and checkpoint_every must be positive")
        self.layout = layout
        self.K = int(steps)
        self.C = int(checkpoint_every)
        self.sim = sph.Simulation(layout, nsub=nsub, device=device)
        self.device = self.sim.device
        self.fixed_dts = None
        if dts is not None:
            self.fixed_dts = torch.as_tensor(np.asarray(dts, dtype=np.float64)).to(self.device)
            if self.fixed_dts.numel() != self.K:
                raise ValueError("dts must have one entry per step")
        self.dts = torch.zeros(self.K, dtype=torch.float64, device=self.device)
        self.ckpt = {}
        self.tapes = []
        self.alpha = float(layout.phys.alpha)

    # -- state helpers
    def _snapshot(self):
        a = self.sim.a
        return [t.clone() for t in (a.cell, a.pos, a.velrho, a.velrho_prev, a.id)]

    def _restore(self, snap):
        a = self.sim.a
        for dst, src in zip((a.cell, a.pos, a.velrho, a.velrho_prev, a.id), snap):
            dst.copy_(src)

    def _one_step(self, n, tape=None):
        """One step from the state in sim.a.  With a tape, the sorted state,
        cell arrays, permutation and (a, D) of the step are kept in it and
        the time step is the recorded (or given) one."""
        sim = self.sim
        fixed = self.fixed_dts if self.fixed_dts is not None else (self.dts if tape is not None else None)
        if tape is None:
            sim.build_cells()
            sim.interact()
            ace = sim.ace
        else:
            sph.sph_build_cells(sim.grid, sim.a.c(), tape.state(), tape.cells(), tape.perm,
                                sim.ws, sim.status)
            sph.sph_interact(sim.grid, sim.params, tape.state(), tape.cells(), tape.ace,
                             sim.visc, sim.npairs, sim.ws)
            # the Verlet update works in place: give it a copy, keep the tape
            a, t = sim.a, tape.st
            for dst, src in ((a.cell, t.cell), (a.pos, t.pos), (a.velrho, t.velrho),
                             (a.velrho_prev, t.velrho_prev), (a.id, t.id)):
                dst.copy_(src)
            ace = tape.ace
        sim.step_index = n
        if fixed is not None:
            sim.dt.copy_(fixed[n:n + 1])
            sph.sph_step(sim.grid, sim.params, sim.a.c(), ace, sim.visc, sim.dt, n,
                         sph.SPH_FIXED_DT, sim.ws, sim.status)
        else:
            sph.sph_step(sim.grid, sim.params, sim.a.c(), ace, sim.visc, sim.dt, n, 0, sim.ws,
                         sim.status)
            self.dts[n:n + 1].copy_(sim.dt)

    def forward(self, alpha: float, v0_fluid):
        """v0_fluid: device FP64 [nf, 3] initial fluid velocities (id order).
        Returns device FP64 [nf, 3] fluid positions after K steps (id order)."""
        import torch

        lay = self.layout
        self.alpha = float(alpha)
        self.sim.params.alpha = self.alpha
        x = torch.as_tensor(np.ascontiguousarray(lay.x, dtype=np.float64)).to(self.device)
        v = torch.zeros((lay.n, 3), dtype=torch.float64, device=self.device)
        v[lay.nb:] = v0_fluid.to(self.device, torch.float64)
        rho = torch.as_tensor(np.ascontiguousarray(lay.rho, dtype=np.float64)).to(self.device)
        sph.sph_encode(self.sim.grid, self.sim.params, x, v, rho, self.sim.a.c(), self.sim.status)
        self.ckpt = {}
        for n in range(self.K):
            if n % self.C == 0:
                self.ckpt[n // self.C] = self._snapshot()
            self._one_step(n)
        return self.fluid_positions()

    def fluid_positions(self):
        import torch

        sim, lay = self.sim, self.layout
        xs = torch.empty((lay.n, 3), dtype=torch.float64, device=self.device)
        vs = torch.empty((lay.n, 3), dtype=torch.float64, device=self.device)
        rs = torch.empty(lay.n, dtype=torch.float64, device=self.device)
        sph.sph_decode(sim.grid, sim.params, sim.a.c(), xs, vs, rs)
        out = torch.empty_like(xs)
        out[sim.a.id.long()] = xs
        return out[lay.nb:]

    def backward(self, grad_x_fluid):
        """Adjoint of the fluid positions at step K (device [nf, 3], id order)
        -> (d/d alpha, d/d v0_fluid [nf, 3] id order)."""
        import torch

        sim, lay = self.sim, self.layout
        n, nb = lay.n, lay.nb
        dev = self.device
        f32 = torch.float32
        gx = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        gx[nb:] = grad_x_fluid.to(dev, torch.float64)
        bufs = [[torch.zeros((n, 4), dtype=f32, device=dev) for _ in range(3)] for _ in range(2)]
        ace_bar = torch.zeros((n, 4), dtype=f32, device=dev)
        cur = 0
        # seed in the slot order of the final state
        bufs[cur][0][:, :3] = gx[sim.a.id.long()].to(f32)
        alpha_bar = torch.zeros(1, dtype=torch.float64, device=dev)
        nseg = (self.K + self.C - 1) // self.C
        if len(self.tapes) < min(self.C, self.K):
            self.tapes = [_Tape(sim) for _ in range(min(self.C, self.K))]
        for s in reversed(range(nseg)):
            n0, n1 = s * self.C, min(self.K, (s + 1) * self.C)
            self._restore(self.ckpt[s])
            for k in range(n0, n1):
                self._one_step(k, self.tapes[k - n0])
            for k in reversed(range(n0, n1)):
                t = self.tapes[k - n0]
                st = t.state()
                xb, vb, vpb = bufs[cur]
                adj = _adjoint_struct(xb, vb, vpb, ace_bar)
                dt = self.dts if self.fixed_dts is None else self.fixed_dts
                sph.sph_step(sim.grid, sim.params, st, t.ace, sim.visc, dt[k:k + 1], k,
                             sph.SPH_ADJOINT, sim.ws, sim.status, adj=adj)
                sph.sph_interact_backward(sim.grid, sim.params, st, t.cells(), ace_bar, xb, vb,
                                          alpha_bar, sim.ws)
                nxt = 1 - cur
                sph.sph_build_cells_backward(t.perm, n, adj, _adjoint_struct(*bufs[nxt], None))
                cur = nxt
        xb, vb, vpb = bufs[cur]
        # the initial state sets v^{-1} = v^0: both adjoints belong to v0
        gv0 = (vb[nb:, :3] + vpb[nb:, :3]).to(torch.float64)
        return alpha_bar[0], gv0


def _autograd_function():
    import torch

    class SphRollout(torch.autograd.Function):
        """x_K = SphRollout.apply(alpha, v0_fluid, rollout)."""

        @staticmethod
        def forward(ctx, alpha, v0_fluid, roll):
            ctx.roll = roll
            ctx.alpha_like = (alpha.device, alpha.dtype, alpha.shape)
            ctx.v_like = (v0_fluid.device, v0_fluid.dtype)
            return roll.forward(float(alpha), v0_fluid.detach())

        @staticmethod
        def backward(ctx, grad_x):
            ga, gv = ctx.roll.backward(grad_x.detach())
            dev, dt, shape = ctx.alpha_like
            return (ga.to(device=dev, dtype=dt).reshape(shape), gv.to(*ctx.v_like), None)

    return SphRollout


def __getattr__(name):
    if name == "SphRollout":
        return _autograd_function()
    raise AttributeError(name)
