"""The C ABI library loads and exports every symbol declared in include/sph.h;
host-side validation rejects bad arguments before touching the device.  No
compute call is made (runs without a GPU)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sph.h")).read()
    return sorted(set(re.findall(r"SPH_API\s+[\w\s\*]+?\b(sph_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1110_3711_amd import sph

    if not os.path.exists(sph.LIB_PATH):
        pytest.fail("libsph.so is not built (run __graft_entry__.build())")
    return sph.load()


def test_header_declares_the_four_calls():
    names = _declared()
    for f in ["sph_build_cells", "sph_interact", "sph_step", "sph_interact_backward"]:
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1110_3711_amd import sph

    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(sph.EXPORTS) == _declared()
    assert lib.sph_abi_version() == 8


def test_library_resolves_every_symbol_at_load():
    """Loading with immediate binding fails on any undefined symbol (for
    instance a kernel whose host stub was not emitted), which lazy binding
    would only report at the first launch."""
    import ctypes

    from paper_1110_3711_amd import sph

    ctypes.CDLL(sph.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)


def _grid():
    from paper_1110_3711_amd import sph

    return sph.make_grid([0, 0, 0], [1, 1, 1], 0.05, [20, 20, 20], 1)


def test_workspace_query(lib):
    from paper_1110_3711_amd import sph

    g = _grid()
    assert sph.sph_workspace_bytes(g, 1000) > 16 * 1000
    assert sph.sph_workspace_bytes(g, 0) > 0
    bad = sph.make_grid([0, 0, 0], [1, 1, 1], 0.05, [20, 20, 20], 3)
    assert sph.sph_workspace_bytes(bad, 1000) == 0
    small = sph.make_grid([0, 0, 0], [1, 1, 1], 0.01, [20, 20, 20], 1)  # does not cover
    assert sph.sph_workspace_bytes(small, 1000) == 0
    assert sph.sph_workspace_bytes(g, -1) == 0


def test_ctypes_structs_match_header(tmp_path):
    """The binding's ctypes structures have the sizes and member offsets that a
    C compiler gives the structs of include/sph.h."""
    import shutil
    import subprocess

    from paper_1110_3711_amd import sph

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    structs = {"sph_grid": sph.Grid, "sph_params": sph.Params, "sph_state": sph.State,
               "sph_cells": sph.Cells, "sph_adjoint": sph.Adjoint}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "sph.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + inc, "-o",
                    str(exe), str(src)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            cname, key, val = ln.split()
            got[(cname, key)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_range_table_size(lib):
    """Interaction ranges (Section 4.4, optimisation D): 9 X-runs x 2 particle
    types x (first, end) = 144 bytes per cell with cells of side 2h, 25 runs
    (400 bytes) with cells of side h."""
    from paper_1110_3711_amd import sph

    assert sph.sph_ranges_bytes(_grid()) == 20 ** 3 * 144
    g2 = sph.make_grid([0, 0, 0], [1, 1, 1], 0.025, [40, 40, 40], 2)
    assert sph.sph_ranges_bytes(g2) == 40 ** 3 * 400
    bad = sph.make_grid([0, 0, 0], [1, 1, 1], 0.05, [20, 20, 20], 3)
    assert sph.sph_ranges_bytes(bad) == 0


def test_validation_errors_before_any_device_work(lib):
    from paper_1110_3711_amd import sph
    from sph_inputs import physics

    g = _grid()
    p = sph.make_params(physics(0.01))  # 2h = 0.0416 < cell 0.05 -> ok
    st = sph.State()
    st.n, st.nb = 10, 11  # nb > n
    cells = sph.Cells()
    assert lib.sph_build_cells(C.byref(g), C.byref(st), C.byref(st), C.byref(cells), None, None,
                               0, None, None) == sph.SPH_ERR_ARG
    assert lib.sph_interact(None, C.byref(p), C.byref(st), C.byref(cells), 3, None, None, None,
                            None, None, 0, None) == sph.SPH_ERR_ARG
    st.nb = 0
    # non-null fake pointers: validation must still stop at the workspace size
    fake = C.c_void_p(16)
    st.cell = st.pos = st.velrho = st.velrho_prev = st.id = 16
    st2 = sph.State()
    st2.n, st2.nb = 10, 0
    st2.cell = st2.pos = st2.velrho = st2.velrho_prev = st2.id = 32
    cells.start = cells.list = cells.info = 16
    assert lib.sph_build_cells(C.byref(g), C.byref(st), C.byref(st2), C.byref(cells), fake, fake, 8,
                               fake, None) == sph.SPH_ERR_WORKSPACE
    # src and dst may not alias
    assert lib.sph_build_cells(C.byref(g), C.byref(st), C.byref(st), C.byref(cells), fake, fake,
                               1 << 40, fake, None) == sph.SPH_ERR_ARG
    # stencil smaller than the support: cell * nsub < 2h
    p2 = sph.make_params(physics(0.02))  # 2h = 0.083 > 0.05
    assert lib.sph_interact(C.byref(g), C.byref(p2), C.byref(st), C.byref(cells), 3, fake, fake,
                            None, None, fake, 1 << 40, None) == sph.SPH_ERR_ARG
    # unknown parts selectors
    for parts in (0, 4, 8, 3 | 4, 3 | 8):
        assert lib.sph_interact(C.byref(g), C.byref(p), C.byref(st), C.byref(cells), parts, fake,
                                fake, None, None, fake, 1 << 40, None) == sph.SPH_ERR_ARG
    # gamma other than 7 and unknown kernels are rejected
    p3 = sph.make_params(physics(0.01))
    p3.gamma = 5.0
    assert lib.sph_interact(C.byref(g), C.byref(p3), C.byref(st), C.byref(cells), 3, fake, fake,
                            None, None, fake, 1 << 40, None) == sph.SPH_ERR_ARG
    p5 = sph.make_params(physics(0.01))
    for bad in (-0.01, 2.0 * p5.h, float("nan")):  # tensile spacing outside [0, 2h)
        p5.tensile_dp = bad
        assert lib.sph_interact(C.byref(g), C.byref(p5), C.byref(st), C.byref(cells), 3, fake,
                                fake, None, None, fake, 1 << 40, None) == sph.SPH_ERR_ARG
    p4 = sph.make_params(physics(0.01))
    p4.kernel = 2  # only SPH_WENDLAND5 (0) and SPH_CUBIC_SPLINE (1) exist
    assert lib.sph_step(C.byref(g), C.byref(p4), C.byref(st), fake, fake, fake, 0, 0, None, fake,
                        1 << 40, fake, None) == sph.SPH_ERR_ARG
    # unknown flags, negative step
    assert lib.sph_step(C.byref(g), C.byref(p), C.byref(st), fake, fake, fake, 0, 64, None, fake,
                        1 << 40, fake, None) == sph.SPH_ERR_ARG
    assert lib.sph_step(C.byref(g), C.byref(p), C.byref(st), fake, fake, fake, -1, 0, None, fake,
                        1 << 40, fake, None) == sph.SPH_ERR_ARG


def test_static_scratch_entry_rejects_before_any_device_call(lib):
    """sph_build_cells_static checks its arguments and the size of its
    workspace against the static scratch before it touches a device (this
    runs without one): bad arguments give SPH_ERR_ARG, a particle count whose
    workspace exceeds the scratch gives SPH_ERR_WORKSPACE."""
    from paper_1110_3711_amd import sph

    g = _grid()
    src, dst, cells = sph.State(), sph.State(), sph.Cells()
    fake = C.c_void_p(16)
    n_big = 1 << 30
    for st, ptr in ((src, 16), (dst, 4096)):
        st.n, st.nb = n_big, 0
        st.cell = st.pos = st.velrho = st.velrho_prev = st.id = ptr
    cells.start = cells.list = cells.info = 16
    assert sph.sph_workspace_bytes(g, n_big) > sph.STATIC_SCRATCH_BYTES
    assert lib.sph_build_cells_static(C.byref(g), C.byref(src), C.byref(dst), C.byref(cells),
                                      fake, fake, None) == sph.SPH_ERR_WORKSPACE
    # the largest particle count that fits this grid is accepted up to the
    # device call (not made here); one beyond is refused
    lo, hi = 0, n_big
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if sph.sph_workspace_bytes(g, mid) <= sph.STATIC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid
    assert lo > 1_000_000
    src.n = dst.n = hi
    assert lib.sph_build_cells_static(C.byref(g), C.byref(src), C.byref(dst), C.byref(cells),
                                      fake, fake, None) == sph.SPH_ERR_WORKSPACE
    # argument errors: src and dst alias, missing dev_status, nb > n
    assert lib.sph_build_cells_static(C.byref(g), C.byref(src), C.byref(src), C.byref(cells),
                                      fake, fake, None) == sph.SPH_ERR_ARG
    assert lib.sph_build_cells_static(C.byref(g), C.byref(src), C.byref(dst), C.byref(cells),
                                      fake, None, None) == sph.SPH_ERR_ARG
    src.nb = src.n + 1
    assert lib.sph_build_cells_static(C.byref(g), C.byref(src), C.byref(dst), C.byref(cells),
                                      fake, fake, None) == sph.SPH_ERR_ARG


def test_position_policy_validation(lib):
    """SPH_POS_ABS64 is a forward variant of the default kernel: the entry
    points refuse it with per-pair statistics, the cubic spline, the tensile
    correction, a state without pos64, in the adjoint, and refuse a reorder
    with pos64 on one side only (no device work: fake pointers)."""
    from paper_1110_3711_amd import sph
    from sph_inputs import physics

    g = _grid()
    fake = C.c_void_p(16)
    st = sph.State()
    st.n, st.nb = 10, 0
    st.cell = st.pos = st.velrho = st.velrho_prev = st.id = 16
    cells = sph.Cells()
    cells.start = cells.list = cells.info = 16
    big = 1 << 40

    def interact(p, s, stats=None):
        return lib.sph_interact(C.byref(g), C.byref(p), C.byref(s), C.byref(cells), 3, fake, fake,
                                None, stats, fake, big, None)

    p = sph.make_params(physics(0.01), sph.SPH_POS_ABS64)
    assert interact(p, st) == sph.SPH_ERR_ARG  # no pos64 in the state
    st.pos64 = 64
    for bad in ("stats", "cubic", "tensile"):
        q = sph.make_params(physics(0.01), sph.SPH_POS_ABS64)
        stats = None
        if bad == "stats":
            stats = fake
        elif bad == "cubic":
            q.kernel = 1
        else:
            q.tensile_dp = 0.01
        assert interact(q, st, stats) == sph.SPH_ERR_ARG, bad
    q = sph.make_params(physics(0.01), 2)  # unknown policy
    assert interact(q, st) == sph.SPH_ERR_ARG
    assert lib.sph_interact_backward(C.byref(g), C.byref(p), C.byref(st), C.byref(cells), fake,
                                     fake, fake, fake, fake, big, None) == sph.SPH_ERR_ARG
    # reorder: pos64 on both sides or on neither
    st2 = sph.State()
    st2.n, st2.nb = 10, 0
    st2.cell = st2.pos = st2.velrho = st2.velrho_prev = st2.id = 32
    assert lib.sph_build_cells(C.byref(g), C.byref(st), C.byref(st2), C.byref(cells), fake, fake,
                               big, fake, None) == sph.SPH_ERR_ARG
    st2.pos64 = 64  # the same array on both sides
    assert lib.sph_build_cells(C.byref(g), C.byref(st), C.byref(st2), C.byref(cells), fake, fake,
                               big, fake, None) == sph.SPH_ERR_ARG


def test_product_path_has_no_cpu_fallback():
    # the package must not import the oracle anywhere
    pkg = os.path.join(ROOT, "paper_1110_3711_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "sph_oracle" not in txt, f


def test_c_driver_rejects_bad_input(tmp_path):
    """The plain-C driver checks its input before it touches a device: usage,
    a header with nb > n and a truncated file end with an error status."""
    import struct
    import subprocess

    exe = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1110_3711_amd", "sph_run")
    if not os.access(exe, os.X_OK):
        pytest.skip("sph_run is not built")
    out = tmp_path / "out.bin"
    assert subprocess.run([exe], capture_output=True, timeout=60).returncode == 2
    bad = tmp_path / "bad.bin"
    bad.write_bytes(struct.pack("<3i", 5, 9, 1))
    r = subprocess.run([exe, str(bad), str(out)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "bad header" in r.stderr
    short = tmp_path / "short.bin"
    short.write_bytes(struct.pack("<3i", 5, 2, 1) + b"\0" * 16)
    r = subprocess.run([exe, str(short), str(out)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "too short" in r.stderr
    assert not out.exists()
