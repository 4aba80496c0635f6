"""Pins of the oracle's neighbour search and of its FP32 decision variant.

* The O(N^2) brute force and the cell list find identical neighbour sets, and
  with id-ordered summation give bit-identical FP64 forces (Section 2 stage NL
  is only an accelerator of the pair search).
* No boundary-boundary pairs (Section 2).
* The FP32 decision variant (the precision the GPU decides in) agrees with the
  FP64 sets except on pairs whose distance is within rounding of the cutoff.
"""

import numpy as np

from sph_inputs import blob, cell_grid, dam_break, named_case


def test_brute_equals_cells_8k(ora):
    L = named_case("dam_break_8k")
    P = ora.params(L.phys)
    rb, cb = ora.neighbour_csr(L.x, L.nb, L.phys.h, mode=0)
    rc, cc = ora.neighbour_csr(L.x, L.nb, L.phys.h, mode=1)
    assert np.array_equal(rb, rc)
    assert np.array_equal(cb, cc)
    a0, v0, n0, p0 = ora.interact(L.x, L.v, L.rho, L.nb, P, mode=0)
    a1, v1, n1, p1 = ora.interact(L.x, L.v, L.rho, L.nb, P, mode=1)
    assert p0 == p1 == rb[-1]
    assert np.array_equal(a0, a1) and np.array_equal(v0, v1) and np.array_equal(n0, n1)


def test_brute_equals_cells_blob_with_velocities(ora):
    B = blob(12, 0.01, 5, jitter=0.45)
    P = ora.params(B.phys)
    a0, v0, n0, p0 = ora.interact(B.x, B.v, B.rho, 0, P, mode=0)
    a1, v1, n1, p1 = ora.interact(B.x, B.v, B.rho, 0, P, mode=1)
    assert p0 == p1 and np.array_equal(a0, a1) and np.array_equal(v0, v1)


def test_neighbour_sets_by_definition(ora):
    # tiny case: sets equal the definition evaluated with numpy
    B = dam_break(0.02, 3, fluid=(0.1, 0.1, 0.1), tank=(0.14, 0.12, 0.12))
    rp, cols = ora.neighbour_csr(B.x, B.nb, B.phys.h, mode=1)
    d2 = ((B.x[:, None, :] - B.x[None, :, :]) ** 2).sum(-1)
    for a in range(B.n):
        ok = d2[a] < 4 * B.phys.h**2
        ok[a] = False
        if a < B.nb:
            ok[: B.nb] = False
        assert np.array_equal(np.nonzero(ok)[0], cols[rp[a]:rp[a + 1]])


def test_no_boundary_boundary_pairs(ora):
    L = named_case("dam_break_8k")
    xb = L.x[: L.nb]
    rp, cols = ora.neighbour_csr(xb, L.nb, L.phys.h, mode=1)
    assert rp[-1] == 0
    rp, cols = ora.neighbour_csr(L.x, L.nb, L.phys.h, mode=1)
    for a in range(0, L.nb, 53):
        assert np.all(cols[rp[a]:rp[a + 1]] >= L.nb)


def test_excluded_particles_never_interact(ora):
    L = named_case("dam_break_8k")
    P = ora.params(L.phys)
    excl = np.zeros(L.n, dtype=np.uint8)
    excl[L.nb + 100:L.nb + 200] = 1
    ace, visc, nnb, _ = ora.interact(L.x, L.v, L.rho, L.nb, P, excl=excl)
    assert np.all(nnb[excl == 1] == 0) and np.all(ace[excl == 1] == 0)
    rp, cols = ora.neighbour_csr(L.x, L.nb, L.phys.h, excl=excl)
    assert not np.isin(cols, np.arange(L.nb + 100, L.nb + 200)).any()


def test_fp32_decision_matches_fp64_sets(ora):
    L = named_case("dam_break_8k")
    for nsub in (1, 2):
        org, cell, nc = cell_grid(L, nsub)
        cidx, off = ora.encode(L.x, org, cell, nc, L.lo, L.hi)
        x = ora.decode(cidx, off, org, cell, nc)
        rc2 = np.float32(4.0 * L.phys.h * L.phys.h)
        cnt, hs, tot = ora.count_f32(cidx, off, L.nb, nc, np.float32(cell), rc2)
        rp, cols = ora.neighbour_csr(x, L.nb, L.phys.h, mode=1)
        c64 = np.diff(rp)
        bad = np.nonzero(c64 != cnt)[0]
        # every disagreement is a pair within rounding of the cutoff
        for a in bad:
            d2 = ((x[a] - x) ** 2).sum(1)
            near = np.abs(d2 / (4 * L.phys.h**2) - 1.0) < 1e-6
            assert abs(int(c64[a]) - int(cnt[a])) <= near.sum()
        assert len(bad) <= 4
        # hashes of agreeing sets agree
        ids = np.arange(L.n, dtype=np.uint64)
        hh = (ids * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)
        for a in range(0, L.n, 211):
            if a in bad:
                continue
            s = int(hh[cols[rp[a]:rp[a + 1]]].sum()) & 0xFFFFFFFF
            assert s == int(hs[a])


def test_stencil_superset(ora):
    # With offsets |o| <= cell/2, a pair inside the support lies within
    # (2 nsub + 1)^3 cells: check every FP64 neighbour pair of the 8k-fluid dam break.
    L = named_case("dam_break_8k")
    for nsub in (1, 2):
        org, cell, nc = cell_grid(L, nsub)
        cidx, off = ora.encode(L.x, org, cell, nc, L.lo, L.hi)
        assert np.abs(off).max() <= np.float32(cell / 2)
        k = np.stack([cidx % nc[0], (cidx // nc[0]) % nc[1], cidx // (nc[0] * nc[1])], 1)
        rp, cols = ora.neighbour_csr(L.x, L.nb, L.phys.h, mode=1)
        rows = np.repeat(np.arange(L.n), np.diff(rp))
        assert np.abs(k[cols] - k[rows]).max() <= nsub
