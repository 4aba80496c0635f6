"""ctypes binding of ``libsph.so`` (include/sph.h) plus a small driver.

The binding only marshals arguments: every stage of the step runs in the HIP
kernels of the library.  PyTorch provides device memory (tensors) and the HIP
stream (``torch.cuda.current_stream()``).  If the library has not been built,
``load()`` (called by every entry point and by ``Simulation``) raises; there is
no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK, SPH_ERR_ARG, SPH_ERR_WORKSPACE, SPH_ERR_HIP = 0, 1, 2, 3
SPH_DEV_OUT_OF_GRID, SPH_DEV_NONFINITE, SPH_DEV_BOUNDARY_OUT = 1, 2, 4
SPH_FIXED_DT, SPH_ADJOINT = 1, 2
SPH_PI_FLUID, SPH_PI_BOUNDARY, SPH_PI_ALL = 1, 2, 3
SPH_EXCLUDED = 2**31 - 1
SPH_POS_OFFSET32, SPH_POS_ABS64 = 0, 1
ABI_VERSION = 8
STATIC_SCRATCH_BYTES = 64 << 20  # SPH_STATIC_SCRATCH_BYTES

EXPORTS = ["sph_workspace_bytes", "sph_ranges_bytes", "sph_abi_version", "sph_encode", "sph_decode",
           "sph_build_cells", "sph_interact", "sph_step", "sph_interact_backward",
           "sph_build_cells_backward", "sph_conservation", "sph_build_cells_static"]


class Grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("hi", C.c_double * 3), ("cell", C.c_double),
                ("nc", C.c_int32 * 3), ("nsub", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("h", C.c_double), ("rho0", C.c_double), ("gamma", C.c_double),
                ("c0", C.c_double), ("alpha", C.c_double), ("eta2", C.c_double),
                ("g", C.c_double * 3), ("mass", C.c_double), ("cfl", C.c_double),
                ("kernel", C.c_int32), ("verlet_ns", C.c_int32), ("bound_floor", C.c_int32),
                ("pos_policy", C.c_int32), ("tensile_dp", C.c_double)]


class State(C.Structure):
    _fields_ = [("n", C.c_int32), ("nb", C.c_int32), ("cell", C.c_void_p), ("pos", C.c_void_p),
                ("velrho", C.c_void_p), ("velrho_prev", C.c_void_p), ("id", C.c_void_p),
                ("pos64", C.c_void_p)]


class Cells(C.Structure):
    _fields_ = [("start", C.c_void_p), ("list", C.c_void_p), ("info", C.c_void_p),
                ("ranges", C.c_void_p)]


class Adjoint(C.Structure):
    _fields_ = [("pos_bar", C.c_void_p), ("velrho_bar", C.c_void_p),
                ("velrho_prev_bar", C.c_void_p), ("ace_bar", C.c_void_p)]


class SphError(RuntimeError):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load libsph.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SphError(f"{path} not found: build the HIP library first "
                       "(python -m paper_1110_3711_amd.build)")
    L = C.CDLL(path)
    vp, sz = C.c_void_p, C.c_size_t
    P = C.POINTER
    L.sph_workspace_bytes.argtypes = [P(Grid), C.c_int32]
    L.sph_workspace_bytes.restype = sz
    L.sph_ranges_bytes.argtypes = [P(Grid)]
    L.sph_ranges_bytes.restype = sz
    L.sph_abi_version.argtypes = []
    L.sph_abi_version.restype = C.c_int32
    L.sph_encode.argtypes = [P(Grid), P(Params), vp, vp, vp, P(State), vp, vp]
    L.sph_decode.argtypes = [P(Grid), P(Params), P(State), vp, vp, vp, vp]
    L.sph_build_cells.argtypes = [P(Grid), P(State), P(State), P(Cells), vp, vp, sz, vp, vp]
    L.sph_build_cells_static.argtypes = [P(Grid), P(State), P(State), P(Cells), vp, vp, vp]
    L.sph_interact.argtypes = [P(Grid), P(Params), P(State), P(Cells), C.c_uint, vp, vp, vp, vp,
                               vp, sz, vp]
    L.sph_step.argtypes = [P(Grid), P(Params), P(State), vp, vp, vp, C.c_longlong, C.c_uint,
                           P(Adjoint), vp, sz, vp, vp]
    L.sph_interact_backward.argtypes = [P(Grid), P(Params), P(State), P(Cells), vp, vp, vp, vp,
                                        vp, sz, vp]
    L.sph_build_cells_backward.argtypes = [vp, C.c_int32, P(Adjoint), P(Adjoint), vp]
    L.sph_conservation.argtypes = [P(Grid), P(Params), P(State), vp, vp, vp, sz, vp]
    for f in ["sph_encode", "sph_decode", "sph_build_cells", "sph_build_cells_static",
              "sph_interact", "sph_step",
              "sph_interact_backward", "sph_build_cells_backward", "sph_conservation"]:
        getattr(L, f).restype = C.c_int
    if L.sph_abi_version() != ABI_VERSION:
        raise SphError("libsph.so ABI version mismatch")
    _lib = L
    return L


def _check(st, what):
    if st != SPH_OK:
        names = {1: "SPH_ERR_ARG", 2: "SPH_ERR_WORKSPACE", 3: "SPH_ERR_HIP"}
        raise SphError(f"{what} failed: {names.get(st, st)}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, count, name, optional=False):
    """A device array passed to the C ABI must be a contiguous CUDA tensor of
    the expected dtype with at least `count` elements (the library cannot
    check device buffer sizes itself)."""
    import torch

    if t is None:
        if optional:
            return
        raise SphError(f"{name}: a device array is required")
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise SphError(f"{name}: expected a CUDA tensor")
    if t.dtype != dtype:
        raise SphError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise SphError(f"{name}: expected a contiguous tensor")
    if t.numel() < count:
        raise SphError(f"{name}: {t.numel()} elements, need at least {count}")


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------
# entry points with the C names (argument marshalling only)

def sph_workspace_bytes(grid: Grid, n: int) -> int:
    return load().sph_workspace_bytes(C.byref(grid), int(n))


def sph_ranges_bytes(grid: Grid) -> int:
    return load().sph_ranges_bytes(C.byref(grid))


def sph_encode(grid, params, x, v, rho, state, dev_status, stream=None):
    import torch

    n = state.n
    _need(x, torch.float64, 3 * n, "x")
    _need(v, torch.float64, 3 * n, "v")
    _need(rho, torch.float64, n, "rho")
    _need(dev_status, torch.int32, 1, "dev_status")
    _check(load().sph_encode(C.byref(grid), C.byref(params), _ptr(x), _ptr(v), _ptr(rho),
                             C.byref(state), _ptr(dev_status), _stream(stream)), "sph_encode")


def sph_decode(grid, params, state, x, v, rho, stream=None):
    import torch

    n = state.n
    _need(x, torch.float64, 3 * n, "x")
    _need(v, torch.float64, 3 * n, "v")
    _need(rho, torch.float64, n, "rho")
    _check(load().sph_decode(C.byref(grid), C.byref(params), C.byref(state), _ptr(x), _ptr(v),
                             _ptr(rho), _stream(stream)), "sph_decode")


def sph_build_cells(grid, src, dst, cells, perm, ws, dev_status, stream=None):
    import torch

    _need(perm, torch.int32, src.n, "perm")
    _need(ws, torch.uint8, 1, "ws")
    _need(dev_status, torch.int32, 1, "dev_status")
    _check(load().sph_build_cells(C.byref(grid), C.byref(src), C.byref(dst), C.byref(cells),
                                  _ptr(perm), _ptr(ws), ws.numel(), _ptr(dev_status),
                                  _stream(stream)), "sph_build_cells")


def sph_build_cells_static(grid, src, dst, cells, perm, dev_status, stream=None):
    """sph_build_cells in the library's static device scratch (no workspace
    argument, nothing allocated)."""
    import torch

    _need(perm, torch.int32, src.n, "perm")
    _need(dev_status, torch.int32, 1, "dev_status")
    _check(load().sph_build_cells_static(C.byref(grid), C.byref(src), C.byref(dst),
                                         C.byref(cells), _ptr(perm), _ptr(dev_status),
                                         _stream(stream)), "sph_build_cells_static")


def sph_interact(grid, params, state, cells, ace, visc, npairs, ws, nbr_stats=None,
                 parts=SPH_PI_ALL, stream=None):
    import torch

    n = state.n
    _need(ace, torch.float32, 4 * n, "ace")
    _need(visc, torch.float32, n, "visc")
    _need(npairs, torch.int64, 2, "npairs (fluid-target, boundary-target pairs)", optional=True)
    _need(nbr_stats, torch.int32, 2 * n, "nbr_stats", optional=True)
    _need(ws, torch.uint8, 1, "ws")
    _check(load().sph_interact(C.byref(grid), C.byref(params), C.byref(state), C.byref(cells),
                               int(parts), _ptr(ace), _ptr(visc), _ptr(npairs), _ptr(nbr_stats),
                               _ptr(ws), ws.numel(), _stream(stream)), "sph_interact")


def sph_step(grid, params, state, ace, visc, dt, step, flags, ws, dev_status, adj=None,
             stream=None):
    import torch

    n = state.n
    _need(ace, torch.float32, 4 * n, "ace")
    _need(visc, torch.float32, n, "visc")
    _need(dt, torch.float64, 1, "dt")
    _need(ws, torch.uint8, 1, "ws")
    _need(dev_status, torch.int32, 1, "dev_status")
    _check(load().sph_step(C.byref(grid), C.byref(params), C.byref(state), _ptr(ace), _ptr(visc),
                           _ptr(dt), int(step), int(flags), C.byref(adj) if adj else None,
                           _ptr(ws), ws.numel(), _ptr(dev_status), _stream(stream)), "sph_step")


def sph_interact_backward(grid, params, state, cells, ace_bar, pos_bar, velrho_bar, alpha_bar,
                          ws, stream=None):
    import torch

    n = state.n
    _need(ace_bar, torch.float32, 4 * n, "ace_bar")
    _need(pos_bar, torch.float32, 4 * n, "pos_bar")
    _need(velrho_bar, torch.float32, 4 * n, "velrho_bar")
    _need(alpha_bar, torch.float64, 1, "alpha_bar")
    _need(ws, torch.uint8, 1, "ws")
    _check(load().sph_interact_backward(C.byref(grid), C.byref(params), C.byref(state),
                                        C.byref(cells), _ptr(ace_bar), _ptr(pos_bar),
                                        _ptr(velrho_bar), _ptr(alpha_bar), _ptr(ws), ws.numel(),
                                        _stream(stream)), "sph_interact_backward")


def sph_build_cells_backward(perm, n, dst_bar, src_bar, stream=None):
    import torch

    _need(perm, torch.int32, n, "perm")
    _check(load().sph_build_cells_backward(_ptr(perm), int(n), C.byref(dst_bar),
                                           C.byref(src_bar), _stream(stream)),
           "sph_build_cells_backward")


def sph_conservation(grid, params, state, ace, out, ws, stream=None):
    import torch

    _need(ace, torch.float32, 4 * state.n, "ace", optional=True)
    _need(out, torch.float64, 16, "out")
    _need(ws, torch.uint8, 1, "ws")
    _check(load().sph_conservation(C.byref(grid), C.byref(params), C.byref(state), _ptr(ace),
                                   _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "sph_conservation")


CONSERVATION_FIELDS = ("momentum", "internal_force", "kinetic_energy", "potential_energy",
                       "angular_momentum", "internal_torque", "count", "force_scale")


# ----------------------------------------------------------------------------
# host-side description helpers

def make_grid(origin, hi, cell, nc, nsub) -> Grid:
    g = Grid()
    for d in range(3):
        g.origin[d] = float(origin[d])
        g.hi[d] = float(hi[d])
        g.nc[d] = int(nc[d])
    g.cell = float(cell)
    g.nsub = int(nsub)
    return g


def make_params(phys, pos_policy: int = SPH_POS_OFFSET32) -> Params:
    p = Params()
    p.pos_policy = int(pos_policy)
    p.h, p.rho0, p.gamma, p.c0 = phys.h, phys.rho0, phys.gamma, phys.c0
    p.alpha, p.eta2, p.mass, p.cfl = phys.alpha, phys.eta2, phys.mass, phys.cfl
    for d in range(3):
        p.g[d] = phys.g[d]
    p.kernel, p.verlet_ns, p.bound_floor = phys.kernel, phys.verlet_ns, phys.bound_floor
    p.tensile_dp = phys.tensile_dp
    return p


class DeviceState:
    """Device arrays of one side of the double-buffered particle state."""

    def __init__(self, n, nb, device, pos64=False):
        import torch

        self.n, self.nb = n, nb
        # optional FP64 absolute positions (position-load policy SPH_POS_ABS64)
        self.pos64 = torch.empty((n, 3), dtype=torch.float64, device=device) if pos64 else None
        self.cell = torch.empty(n, dtype=torch.int32, device=device)
        self.pos = torch.empty((n, 4), dtype=torch.float32, device=device)
        self.velrho = torch.empty((n, 4), dtype=torch.float32, device=device)
        self.velrho_prev = torch.empty((n, 4), dtype=torch.float32, device=device)
        self.id = torch.empty(n, dtype=torch.int32, device=device)

    def c(self) -> State:
        """The C descriptor of these arrays (built once: the tensors are never
        reallocated)."""
        if getattr(self, "_c", None) is None:
            s = State()
            s.n, s.nb = self.n, self.nb
            s.cell, s.pos = self.cell.data_ptr(), self.pos.data_ptr()
            s.velrho, s.velrho_prev = self.velrho.data_ptr(), self.velrho_prev.data_ptr()
            s.id = self.id.data_ptr()
            s.pos64 = None if self.pos64 is None else self.pos64.data_ptr()
            self._c = s
        return self._c


class Simulation:
    """Owns the device buffers of one particle set and runs NL -> PI -> SU.

    ``layout`` is a host layout (FP64 arrays indexed by particle id); it is
    copied to the device once and encoded there.  Nothing in ``step`` leaves
    the device.
    """

    def __init__(self, layout, nsub: int = 1, device="cuda:0", grid=None, ranges=False,
                 pos64=False):
        import torch

        from sph_inputs import cell_grid

        load()
        self.device = torch.device(device)
        self.layout = layout
        if grid is None:
            org, cell, nc = cell_grid(layout, nsub)
            grid = make_grid(org, layout.hi, cell, nc, nsub)
        self.grid = grid
        # pos64: the state keeps FP64 absolute positions and the pair kernel
        # forms r_ab from them (SPH_POS_ABS64); otherwise cell + FP32 offset
        self.params = make_params(layout.phys, SPH_POS_ABS64 if pos64 else SPH_POS_OFFSET32)
        n, nb = layout.n, layout.nb
        self.n, self.nb = n, nb
        self.ncell = int(grid.nc[0]) * int(grid.nc[1]) * int(grid.nc[2])
        self.a = DeviceState(n, nb, self.device, pos64)   # current (sorted after build)
        self.b = DeviceState(n, nb, self.device, pos64)   # scratch side
        self.ws = torch.empty(max(sph_workspace_bytes(grid, n), 1), dtype=torch.uint8,
                              device=self.device)
        if self.ws.numel() <= 1 and n > 0:
            raise SphError("invalid grid for the workspace query")
        self.start = torch.empty(2 * self.ncell + 2, dtype=torch.int32, device=self.device)
        self.list = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self.info = torch.zeros(4, dtype=torch.int32, device=self.device)
        # optional precomputed interaction ranges (144 B per cell with nsub = 1)
        self.ranges = None
        if ranges:
            self.ranges = torch.zeros(sph_ranges_bytes(grid) // 4, dtype=torch.int32,
                                      device=self.device)
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self.ace = torch.empty((max(n, 1), 4), dtype=torch.float32, device=self.device)
        self.visc = torch.empty(max(n, 1), dtype=torch.float32, device=self.device)
        self.npairs = torch.zeros(2, dtype=torch.int64, device=self.device)  # fluid, boundary targets
        self.dt = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.step_index = 0
        self.upload(layout.x, layout.v, layout.rho)

    # -- cells struct
    def cells(self) -> Cells:
        if getattr(self, "_cells", None) is None:
            c = Cells()
            c.start, c.list, c.info = (self.start.data_ptr(), self.list.data_ptr(),
                                       self.info.data_ptr())
            c.ranges = None if self.ranges is None else self.ranges.data_ptr()
            self._cells = c
        return self._cells

    def upload(self, x, v, rho):
        import torch

        xd = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).to(self.device)
        vd = torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)).to(self.device)
        rd = torch.as_tensor(np.ascontiguousarray(rho, dtype=np.float64)).to(self.device)
        sph_encode(self.grid, self.params, xd, vd, rd, self.a.c(), self.status)
        torch.cuda.current_stream().synchronize()
        if self.dev_status() & SPH_DEV_BOUNDARY_OUT:
            raise SphError("a boundary particle lies outside the domain: boundary particles "
                           "must lie inside the grid (they never move)")

    def upload_prev(self, v_prev, rho_prev):
        """Set level n-1 (velrho_prev) from FP64 arrays in id order (current
        state must be unsorted, i.e. straight after upload)."""
        import torch

        vr = np.zeros((self.n, 4), dtype=np.float32)
        vr[:, :3] = np.asarray(v_prev, dtype=np.float64)
        vr[:, 3] = np.asarray(rho_prev, dtype=np.float64) - self.layout.phys.rho0
        self.a.velrho_prev.copy_(torch.as_tensor(vr))

    def build_cells(self):
        sph_build_cells(self.grid, self.a.c(), self.b.c(), self.cells(), self.perm, self.ws,
                        self.status)
        self.a, self.b = self.b, self.a

    def interact(self, stats=None, parts=SPH_PI_ALL, npairs=None):
        sph_interact(self.grid, self.params, self.a.c(), self.cells(), self.ace, self.visc,
                     self.npairs if npairs is None else npairs, self.ws, nbr_stats=stats,
                     parts=parts)

    def update(self, fixed_dt: float | None = None):
        flags = 0
        if fixed_dt is not None:
            self.dt.fill_(fixed_dt)
            flags |= SPH_FIXED_DT
        sph_step(self.grid, self.params, self.a.c(), self.ace, self.visc, self.dt,
                 self.step_index, flags, self.ws, self.status)
        self.step_index += 1

    def step(self):
        self.build_cells()
        self.interact()
        self.update()

    def run(self, k: int):
        for _ in range(k):
            self.step()

    # -- readback (host, id order)
    def decode(self):
        import torch

        x = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        r = torch.empty(self.n, dtype=torch.float64, device=self.device)
        sph_decode(self.grid, self.params, self.a.c(), x, v, r)
        ids = self.a.id.cpu().numpy()
        out_x = np.empty((self.n, 3))
        out_v = np.empty((self.n, 3))
        out_r = np.empty(self.n)
        out_x[ids] = x.cpu().numpy()
        out_v[ids] = v.cpu().numpy()
        out_r[ids] = r.cpu().numpy()
        return out_x, out_v, out_r

    def by_id(self, t):
        """Reorder a per-slot tensor into id order (host numpy)."""
        ids = self.a.id.cpu().numpy()
        a = t.detach().cpu().numpy()
        out = np.empty_like(a)
        out[ids] = a
        return out

    def conservation(self, with_forces=True):
        """FP64 conservation sums of the current state on the device
        (sph_conservation), as a dict of named fields."""
        import torch

        out = torch.zeros(16, dtype=torch.float64, device=self.device)
        sph_conservation(self.grid, self.params, self.a.c(), self.ace if with_forces else None,
                         out, self.ws)
        o = out.cpu().numpy()
        return {"momentum": o[0:3], "internal_force": o[3:6], "kinetic_energy": float(o[6]),
                "potential_energy": float(o[7]), "angular_momentum": o[8:11],
                "internal_torque": o[11:14], "count": float(o[14]), "force_scale": float(o[15])}

    def dev_status(self) -> int:
        return int(self.status.item())

    def check_status(self) -> int:
        """Device status bits (synchronises); raises on SPH_DEV_BOUNDARY_OUT,
        which means the sorted state is invalid."""
        st = self.dev_status()
        if st & SPH_DEV_BOUNDARY_OUT:
            raise SphError("a boundary particle lies outside the domain")
        return st
