"""FP64 CPU oracle of the WCSPH particle step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_1110_3711_amd``); neither imports the other.  The arithmetic lives in
``sph_oracle.c`` (plain C, FP64, OpenMP over targets); this module only
compiles it with gcc and marshals numpy arrays through ctypes.

Parity status: every function is pinned by an independent check in
``tests/test_oracle_*.py``; none is "parity unpinned" except long-horizon
rollout agreement, which the method does not define (chaotic dynamics).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
EXCLUDED = 2**31 - 1


class Params(C.Structure):
    _fields_ = [("h", C.c_double), ("rho0", C.c_double), ("gamma", C.c_double),
                ("c0", C.c_double), ("alpha", C.c_double), ("eta2", C.c_double),
                ("g", C.c_double * 3), ("mass", C.c_double), ("cfl", C.c_double),
                ("kernel", C.c_int32), ("verlet_ns", C.c_int32),
                ("bound_floor", C.c_int32), ("pad_", C.c_int32), ("tensile_dp", C.c_double)]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-mfma", "-mavx2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fvisibility=hidden",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp, ip, i64p, u8p = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int64), C.POINTER(C.c_uint8))
        fp, pp = C.POINTER(C.c_float), C.POINTER(Params)
        L.ora_w.argtypes = [pp, C.c_double]
        L.ora_w.restype = C.c_double
        L.ora_f.argtypes = [pp, C.c_double]
        L.ora_f.restype = C.c_double
        L.ora_pressure.argtypes = [pp, C.c_double]
        L.ora_pressure.restype = C.c_double
        L.ora_sound.argtypes = [pp, C.c_double]
        L.ora_sound.restype = C.c_double
        L.ora_interact.argtypes = [C.c_int, C.c_int, dp, dp, dp, u8p, pp, C.c_int, C.c_int, ip,
                                   dp, dp, ip]
        L.ora_interact.restype = C.c_longlong
        L.ora_neighbour_csr.argtypes = [C.c_int, C.c_int, dp, u8p, C.c_double, C.c_int, i64p, ip]
        L.ora_neighbour_csr.restype = C.c_longlong
        L.ora_dt.argtypes = [C.c_int, C.c_int, dp, dp, dp, u8p, pp]
        L.ora_dt.restype = C.c_double
        L.ora_verlet.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, C.c_double,
                                 C.c_longlong, dp, dp, u8p, pp]
        L.ora_verlet.restype = None
        L.ora_run.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, u8p, dp, dp, pp,
                              C.c_longlong, C.c_int, dp]
        L.ora_run.restype = None
        L.ora_encode.argtypes = [C.c_int, dp, dp, C.c_double, ip, dp, dp, ip, fp]
        L.ora_encode.restype = None
        L.ora_decode.argtypes = [C.c_int, ip, fp, dp, C.c_double, ip, dp]
        L.ora_decode.restype = None
        L.ora_fprime.argtypes = [pp, C.c_double]
        L.ora_fprime.restype = C.c_double
        L.ora_interact_vjp.argtypes = [C.c_int, C.c_int, dp, dp, dp, u8p, pp, dp, dp, dp, dp, dp]
        L.ora_interact_vjp.restype = None
        L.ora_verlet_vjp.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_longlong, u8p,
                                     pp, dp, dp, dp, dp, dp, dp]
        L.ora_verlet_vjp.restype = None
        L.ora_conservation.argtypes = [C.c_int, C.c_int, dp, dp, dp, u8p, pp, dp]
        L.ora_conservation.restype = None
        L.ora_num_threads.argtypes = []
        L.ora_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def params(phys, **override) -> Params:
    """Oracle parameter struct from a layout's physics constants."""
    d = dict(h=phys.h, rho0=phys.rho0, gamma=phys.gamma, c0=phys.c0, alpha=phys.alpha,
             eta2=phys.eta2, g=tuple(phys.g), mass=phys.mass, cfl=phys.cfl, kernel=phys.kernel,
             verlet_ns=phys.verlet_ns, bound_floor=phys.bound_floor,
             tensile_dp=phys.tensile_dp)
    d.update(override)
    P = Params()
    for k, v in d.items():
        if k == "g":
            P.g[0], P.g[1], P.g[2] = v
        else:
            setattr(P, k, v)
    return P


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def kernel_w(P, r):
    return lib().ora_w(C.byref(P), float(r))


def kernel_f(P, r):
    return lib().ora_f(C.byref(P), float(r))


def kernel_fprime(P, r):
    return lib().ora_fprime(C.byref(P), float(r))


def pressure(P, rho):
    return lib().ora_pressure(C.byref(P), float(rho))


def sound(P, rho):
    return lib().ora_sound(C.byref(P), float(rho))


def in_domain(x, lo, hi):
    x = np.asarray(x)
    return np.all((x >= lo) & (x < hi), axis=1)


def interact(x, v, rho, nb, P, excl=None, mode=1, targets=None):
    """Returns (ace[nt,4], visc[nt], nnb[nt], npairs)."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    rho = _f64(rho)
    n = x.shape[0]
    if excl is None:
        excl = np.zeros(n, dtype=np.uint8)
    excl = np.ascontiguousarray(excl, dtype=np.uint8)
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int32)
        nt, tp = targets.size, _p(targets, C.c_int32)
    ace = np.zeros((nt, 4))
    visc = np.zeros(nt)
    nnb = np.zeros(nt, dtype=np.int32)
    npairs = lib().ora_interact(n, nb, _p(x, C.c_double), _p(v, C.c_double), _p(rho, C.c_double),
                                _p(excl, C.c_uint8), C.byref(P), mode, nt, tp,
                                _p(ace, C.c_double), _p(visc, C.c_double), _p(nnb, C.c_int32))
    return ace, visc, nnb, npairs


def neighbour_csr(x, nb, h, excl=None, mode=1):
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    if excl is None:
        excl = np.zeros(n, dtype=np.uint8)
    excl = np.ascontiguousarray(excl, dtype=np.uint8)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    L = lib()
    nnz = L.ora_neighbour_csr(n, nb, _p(x, C.c_double), _p(excl, C.c_uint8), h, mode,
                              _p(rowptr, C.c_int64), None)
    cols = np.zeros(max(nnz, 1), dtype=np.int32)
    L.ora_neighbour_csr(n, nb, _p(x, C.c_double), _p(excl, C.c_uint8), h, mode,
                        _p(rowptr, C.c_int64), _p(cols, C.c_int32))
    return rowptr, cols[:nnz]


def time_step(rho, ace, visc, nb, P, excl=None):
    rho = _f64(rho)
    n = rho.size
    ace = _f64(ace, (-1, 4))
    visc = _f64(visc)
    if excl is None:
        excl = np.zeros(n, dtype=np.uint8)
    excl = np.ascontiguousarray(excl, dtype=np.uint8)
    return lib().ora_dt(n, nb, _p(rho, C.c_double), _p(ace, C.c_double), _p(visc, C.c_double),
                        _p(excl, C.c_uint8), C.byref(P))


CONSERVATION_FIELDS = ("momentum", "internal_force", "kinetic_energy", "potential_energy",
                       "angular_momentum", "internal_torque", "count", "force_scale")


def conservation(x, v, ace, nb, P, excl=None):
    """Global sums of the conservation laws over the fluid (sph_oracle.c
    ora_conservation): a [16] array, see there.  ace may be None."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    n = x.shape[0]
    if excl is None:
        excl = np.zeros(n, dtype=np.uint8)
    excl = np.ascontiguousarray(excl, dtype=np.uint8)
    out = np.zeros(16)
    a4 = None if ace is None else _f64(ace, (-1, 4))
    ap = None if a4 is None else _p(a4, C.c_double)
    lib().ora_conservation(n, nb, _p(x, C.c_double), _p(v, C.c_double), ap, _p(excl, C.c_uint8),
                           C.byref(P), _p(out, C.c_double))
    return out


def conservation_fields(out):
    """Named views of a [16] conservation array."""
    o = np.asarray(out, dtype=np.float64)
    return {"momentum": o[0:3], "internal_force": o[3:6], "kinetic_energy": float(o[6]),
            "potential_energy": float(o[7]), "angular_momentum": o[8:11],
            "internal_torque": o[11:14], "count": float(o[14]), "force_scale": float(o[15])}


class State:
    """Mutable FP64 state of the oracle integrator (levels n and n-1)."""

    def __init__(self, layout, P=None):
        self.x = _f64(layout.x, (-1, 3)).copy()
        self.v = _f64(layout.v, (-1, 3)).copy()
        self.rho = _f64(layout.rho).copy()
        self.vprev = self.v.copy()
        self.rhoprev = self.rho.copy()
        self.nb = int(layout.nb)
        self.lo = _f64(layout.lo).copy()
        self.hi = _f64(layout.hi).copy()
        self.excl = (~in_domain(self.x, self.lo, self.hi)).astype(np.uint8)
        self.P = P if P is not None else params(layout.phys)
        self.step = 0

    @property
    def n(self):
        return self.x.shape[0]

    def interact(self, mode=1, targets=None):
        return interact(self.x, self.v, self.rho, self.nb, self.P, self.excl, mode, targets)

    def verlet(self, ace, dt):
        lib().ora_verlet(self.n, self.nb, _p(self.x, C.c_double), _p(self.v, C.c_double),
                         _p(self.rho, C.c_double), _p(self.vprev, C.c_double),
                         _p(self.rhoprev, C.c_double), _p(_f64(ace, (-1, 4)), C.c_double),
                         float(dt), self.step, _p(self.lo, C.c_double), _p(self.hi, C.c_double),
                         _p(self.excl, C.c_uint8), C.byref(self.P))
        self.step += 1

    def run(self, nsteps):
        dts = np.zeros(max(nsteps, 1))
        lib().ora_run(self.n, self.nb, _p(self.x, C.c_double), _p(self.v, C.c_double),
                      _p(self.rho, C.c_double), _p(self.vprev, C.c_double),
                      _p(self.rhoprev, C.c_double), _p(self.excl, C.c_uint8),
                      _p(self.lo, C.c_double), _p(self.hi, C.c_double), C.byref(self.P),
                      self.step, nsteps, _p(dts, C.c_double))
        self.step += nsteps
        return dts[:nsteps]


def encode(x, origin, cell, nc, lo, hi):
    """Integer cell + FP32 offset encoding (own implementation)."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    org = _f64(origin)
    ncv = np.ascontiguousarray(nc, dtype=np.int32)
    lo = _f64(lo)
    hi = _f64(hi)
    cidx = np.zeros(n, dtype=np.int32)
    off = np.zeros((n, 3), dtype=np.float32)
    lib().ora_encode(n, _p(x, C.c_double), _p(org, C.c_double), float(cell), _p(ncv, C.c_int32),
                     _p(lo, C.c_double), _p(hi, C.c_double), _p(cidx, C.c_int32),
                     _p(off, C.c_float))
    return cidx, off


def decode(cidx, off, origin, cell, nc):
    cidx = np.ascontiguousarray(cidx, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.float32).reshape(-1, 3)
    n = cidx.size
    org = _f64(origin)
    ncv = np.ascontiguousarray(nc, dtype=np.int32)
    x = np.zeros((n, 3))
    lib().ora_decode(n, _p(cidx, C.c_int32), _p(off, C.c_float), _p(org, C.c_double),
                     float(cell), _p(ncv, C.c_int32), _p(x, C.c_double))
    return x


def interact_vjp(x, v, rho, nb, P, abar, excl=None):
    """(xbar[n,3], vbar[n,3], rhobar[n], alphabar) = J^T abar for abar[n,4]."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    rho = _f64(rho)
    n = x.shape[0]
    if excl is None:
        excl = np.zeros(n, dtype=np.uint8)
    excl = np.ascontiguousarray(excl, dtype=np.uint8)
    abar = _f64(abar, (-1, 4))
    xb = np.zeros((n, 3))
    vb = np.zeros((n, 3))
    rb = np.zeros(n)
    al = np.zeros(1)
    lib().ora_interact_vjp(n, nb, _p(x, C.c_double), _p(v, C.c_double), _p(rho, C.c_double),
                           _p(excl, C.c_uint8), C.byref(P), _p(abar, C.c_double),
                           _p(xb, C.c_double), _p(vb, C.c_double), _p(rb, C.c_double),
                           _p(al, C.c_double))
    return xb, vb, rb, float(al[0])


def verlet_vjp(rho, rhoprev, ace, dt, step, nb, P, excl, xb, vb, rb, vpb, rpb):
    """Transpose of one Verlet step (in place on the adjoint arrays); returns
    abar[n,4], the adjoint of (A, D) of that step."""
    rho = _f64(rho)
    n = rho.size
    rhoprev = _f64(rhoprev)
    ace = _f64(ace, (-1, 4))
    excl = np.ascontiguousarray(excl, dtype=np.uint8)
    for a in (xb, vb, rb, vpb, rpb):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    abar = np.zeros((n, 4))
    lib().ora_verlet_vjp(n, nb, _p(rho, C.c_double), _p(rhoprev, C.c_double),
                         _p(ace, C.c_double), float(dt), int(step), _p(excl, C.c_uint8),
                         C.byref(P), _p(xb, C.c_double), _p(vb, C.c_double), _p(rb, C.c_double),
                         _p(vpb, C.c_double), _p(rpb, C.c_double), _p(abar, C.c_double))
    return abar


def rollout(layout, dts, P=None, v0=None, step0=0):
    """FP64 forward rollout with a given time-step sequence; returns the list
    of per-step records (state before the step, its (A, D)) and the final
    State.  Used by the adjoint checks (the time step is frozen)."""
    S = State(layout, P)
    if v0 is not None:
        S.v[:] = v0
        S.vprev[:] = v0
    S.step = step0
    tape = []
    for dt in dts:
        ace, visc, _, _ = S.interact()
        tape.append((S.x.copy(), S.v.copy(), S.rho.copy(), S.rhoprev.copy(), S.excl.copy(),
                     ace, S.step))
        S.verlet(ace, dt)
    return tape, S


def rollout_vjp(layout, tape, dts, P, xbar_final):
    """Reverse pass over a tape from ``rollout``: adjoint of the final
    positions -> (vbar0 [n,3] of the initial velocity, alphabar)."""
    n = layout.n
    xb = np.ascontiguousarray(xbar_final, dtype=np.float64).copy()
    vb = np.zeros((n, 3))
    rb = np.zeros(n)
    vpb = np.zeros((n, 3))
    rpb = np.zeros(n)
    alpha = 0.0
    for (x, v, rho, rhoprev, excl, ace, step), dt in zip(reversed(tape), reversed(dts)):
        abar = verlet_vjp(rho, rhoprev, ace, dt, step, layout.nb, P, excl, xb, vb, rb, vpb, rpb)
        gx, gv, gr, ga = interact_vjp(x, v, rho, layout.nb, P, abar, excl)
        f = slice(layout.nb, None)
        xb[f] += gx[f]
        vb[f] += gv[f]
        rb += gr
        alpha += ga
    # v^{-1} = v^0 at the start: both levels are the initial velocity
    return vb + vpb, alpha


def num_threads():
    return lib().ora_num_threads()
