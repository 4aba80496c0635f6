"""Shared test helpers.  The oracle side of every comparison is computed from
the seeded layout by the oracle's own encoding (never from GPU output)."""

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


ELEM_TOL = 1e-3   # per-element bound: max_i |dev_i - ref_i| / rms_i(|ref_i|)


def elem_err(a, b):
    """Largest per-element error relative to the rms of the reference: rows of
    a 2-D array are vectors (per-target Euclidean norm), a 1-D array holds
    scalars.  A localised mistake (a few wrong targets among many) shows here
    even when the relative L2 over all targets stays small."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b) if a.ndim == 1 else np.linalg.norm(a - b, axis=1)
    r = np.abs(b) if b.ndim == 1 else np.linalg.norm(b, axis=1)
    if d.size == 0:
        return 0.0
    rms = float(np.sqrt(np.mean(r * r)))
    return float(d.max() / rms) if rms > 0 else float(d.max())


def parity(label, tol=1e-4, elem_tol=ELEM_TOL, **fields):
    """Print and assert, for each named (device, reference) pair, the relative
    L2 error (<= tol) and the per-element error (<= elem_tol).  Returns
    {name: (rel L2, per-element)}."""
    out = {k: (rel_l2(a, b), elem_err(a, b)) for k, (a, b) in fields.items()}
    print(f"  {label}: " + ", ".join(f"{k} L2 {e:.2e} max {m:.2e}" for k, (e, m) in out.items()),
          flush=True)
    for k, (e, m) in out.items():
        assert e <= tol, f"{label} {k}: relative L2 {e:.3e} > {tol:.0e}"
        assert m <= elem_tol, f"{label} {k}: per-element error {m:.3e} > {elem_tol:.0e}"
    return out


def oracle_view(ora, x, v, rho, rho0, grid_tuple, lo, hi):
    """FP64 state the device holds after encoding (x, v, rho): positions
    quantised to (cell, FP32 offset), velocity and rho - rho0 rounded to FP32.
    Returns (x, v, rho, excl, cidx, off)."""
    org, cell, nc = grid_tuple
    cidx, off = ora.encode(x, org, cell, nc, lo, hi)
    xq = ora.decode(cidx, off, org, cell, nc)
    excl = (cidx == ora.EXCLUDED).astype(np.uint8)
    xq[excl == 1] = np.asarray(x)[excl == 1]
    vq = np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)
    rq = (np.asarray(rho, dtype=np.float64) - rho0).astype(np.float32).astype(np.float64) + rho0
    return xq, vq, rq, excl, cidx, off


def grid_tuple(sim):
    return (np.array(list(sim.grid.origin)), float(sim.grid.cell), [int(c) for c in sim.grid.nc])


def compress(lay, factor):
    """Positions pulled toward the domain's lower corner by `factor` (< 1): the
    density rises by factor**-3, so a cell's stencil spans several staging
    tiles and boundary cells hold more targets than are staged in LDS."""
    lay.x = lay.lo + factor * (lay.x - lay.lo)
    return lay


# ---------------------------------------------------------------------------
# Neighbour sets against the FP64 definition with an explicit tie band.
#
# The device decides r^2 < 4h^2 in FP32 from the encoded positions; the FP64
# definition on the same (decoded) positions can only disagree for pairs whose
# r^2 lies within rounding of the cutoff.  The oracle's FP64 cell-list sets at
# the cutoff moved by -delta and +delta (relative, in r^2) bracket every valid
# answer: inner <= device set <= outer.  The device reports, per target, the
# neighbour count and sum_b uint32(id_b * HASH_MUL) (mod 2^32).

HASH_MUL = 2654435761
BAND = 1e-5   # relative half-width of the tie band in r^2 (FP32 rounding of r^2 is ~1e-6)


def id_hash(ids):
    ids = np.asarray(ids, dtype=np.uint64)
    return (ids * np.uint64(HASH_MUL)) & np.uint64(0xFFFFFFFF)


def band_sets(ora, x, nb, h, excl=None, delta=BAND):
    """FP64 neighbour sets (CSR over ids) with r^2 < 4h^2 (1 - delta) and with
    r^2 < 4h^2 (1 + delta)."""
    inner = ora.neighbour_csr(x, nb, h * np.sqrt(1.0 - delta), excl=excl)
    outer = ora.neighbour_csr(x, nb, h * np.sqrt(1.0 + delta), excl=excl)
    return inner, outer


def _row_hash(rp, cols):
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    s = np.bincount(rows, weights=id_hash(cols).astype(np.float64), minlength=n)
    return (s.astype(np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def check_sets_in_band(count, hsum, inner, outer, max_band=16):
    """Assert that each target's device set S (count, id hash) satisfies
    inner <= S <= outer.  Targets without band pairs must match exactly; for
    the others, S minus inner must be a subset of the band pairs (found by
    enumeration).  Returns (targets with band pairs, band pairs in total)."""
    from itertools import combinations

    count = np.asarray(count).astype(np.int64)
    hsum = np.asarray(hsum).astype(np.uint32)
    (ri, ci), (ro, co) = inner, outer
    ni, no = np.diff(ri), np.diff(ro)
    hi = _row_hash(ri, ci)
    exact = ni == no
    bad = exact & ((count != ni) | (hsum != hi))
    assert not bad.any(), f"{int(bad.sum())} targets differ from the FP64 sets outside the tie band " \
                          f"(first {np.nonzero(bad)[0][:5]})"
    tied = np.nonzero(~exact)[0]
    for a in tied:
        I = set(ci[ri[a]:ri[a + 1]].tolist())
        band = [b for b in co[ro[a]:ro[a + 1]].tolist() if b not in I]
        assert len(I) + len(band) == no[a] and len(band) <= max_band
        k = int(count[a]) - int(ni[a])
        assert 0 <= k <= len(band), f"target {a}: count {count[a]} outside [{ni[a]}, {no[a]}]"
        want = (int(hsum[a]) - int(hi[a])) % (1 << 32)
        hb = [int(v) for v in id_hash(band)]
        ok = any(sum(hb[i] for i in c) % (1 << 32) == want for c in combinations(range(len(band)), k))
        assert ok, f"target {a}: no subset of its {len(band)} band pairs matches the device set"
    return len(tied), int((no - ni).sum())


def check_every_cell_once(lay, label, nsub=1):
    """The pair kernel's work queue hands out every cell exactly once: with
    every output slot pre-filled with NaN, the fused forward launch writes
    every slot (a cell never taken leaves NaN), and its directed pair count
    equals the sum of the per-target counts of the statistics kernel on the
    same state (a cell taken twice would add its pairs twice to the count,
    while its per-target outputs would only be written again)."""
    import torch

    from paper_1110_3711_amd import sph

    sim = sph.Simulation(lay, nsub=nsub)
    sim.build_cells()
    sim.ace.fill_(float("nan"))
    sim.visc.fill_(float("nan"))
    sim.npairs.zero_()
    sim.interact()
    torch.cuda.synchronize()
    total = int(sim.npairs.sum().item())
    ace = sim.by_id(sim.ace)
    visc = sim.by_id(sim.visc)
    st = torch.zeros(2 * lay.n, dtype=torch.int32, device=sim.device)
    sim.npairs.zero_()
    sim.interact(stats=st)
    torch.cuda.synchronize()
    counted = int(st.view(-1, 2)[:, 0].to(torch.int64).sum().item())
    total_stats = int(sim.npairs.sum().item())
    unwritten = int((~np.isfinite(ace)).any(axis=1).sum() + (~np.isfinite(visc)).sum())
    del sim
    torch.cuda.empty_cache()
    print(f"  {label}: {total:,} directed pairs (default kernel), {counted:,} summed per target "
          f"(statistics kernel, which counts {total_stats:,}); unwritten output slots {unwritten}",
          flush=True)
    assert unwritten == 0
    assert total == counted == total_stats
