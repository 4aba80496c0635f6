// build_cells.hip -- neighbour-list stage (Section 4.1): cell keys, a stable
// LSD radix sort of (key, slot), the cell start array, the list of non-empty
// keys, the reorder of every particle array into cell order and, on request,
// the interaction ranges of every occupied cell (Section 4.4, optimisation D).
//
// Keys: boundary cell k -> k, fluid cell k -> ncell + k, excluded -> 2 ncell,
// so the sorted order is boundary cells, then fluid cells, then excluded
// particles, each cell contiguous and cells X fastest (the X-run property
// used by the interaction stencil, Section 4.4).
#include <algorithm>

#include "sph_internal.h"

namespace sph {

// ---------------------------------------------------------------------------
// keys (computed on the fly by the first radix pass)

struct KeySrc {
    const uint32_t *keys;   // later passes: keys of the previous pass
    const int32_t *cell;    // first pass: cell of slot i (keys == nullptr)
    int32_t nb, ncell;
};

__device__ inline uint32_t key_of(const KeySrc &S, int64_t i)
{
    if (S.keys) return S.keys[i];
    const int32_t c = S.cell[i];
    if (c == SPH_EXCLUDED) return 2u * (uint32_t)S.ncell;
    return (uint32_t)c + (i < S.nb ? 0u : (uint32_t)S.ncell);
}

// ---------------------------------------------------------------------------
// radix sort: per-block digit histograms, digit-major so that one exclusive
// scan gives every (digit, block) its global output offset.  A pass sorts by
// a digit of at most 11 bits; the key width (bit length of 2 ncell) is split
// into the fewest such passes (two for a 20-bit key).  A block takes a tile
// of kSortTile consecutive keys; wave w of the block takes the w-th quarter of
// the tile, 64 keys per round, in input order.

// Runs of equal values in a wave (consecutive lanes, nearly sorted input) are
// counted once: lanes whose left neighbour holds another value are heads, and
// each head adds the length of its run through add(value, length).
template <class Add>
__device__ inline void add_runs(bool valid, uint32_t val, Add &&add)
{
    const int lane = lane_id();
    const uint32_t d = valid ? val : 0xffffffffu;
    const uint32_t dprev = __shfl_up(d, 1);
    const bool head = valid && (lane == 0 || dprev != d);
    const unsigned long long heads = ballot(head);
    const unsigned long long vmask = ballot(valid);
    if (head) {
        const unsigned long long after = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
        const int end = after ? __ffsll((long long)after) - 1 : 64 - __clzll((long long)vmask);
        add(val, (uint32_t)(end - lane));
    }
}

__device__ inline void add_digit_runs(uint32_t *h, bool valid, uint32_t dig)
{
    add_runs(valid, dig, [&](uint32_t d, uint32_t c) { atomicAdd(&h[d], c); });
}

__device__ inline int64_t sort_elem(int round, int wave, int lane)
{
    // element of (round, wave, lane) inside the block's tile
    return (int64_t)wave * (kSortTile / (kSortThreads / kWave)) + (int64_t)round * kWave + lane;
}

// zero, zero32 (optional, first pass): a u64 and a u32 array cleared on the
// side, grid-stride
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(int32_t n, int shift, int dbits,
                                                             KeySrc keys,
                                                             uint32_t *__restrict__ hist,
                                                             int nblk, int32_t *dev_status,
                                                             unsigned long long *__restrict__ zero,
                                                             int64_t nzero,
                                                             uint32_t *__restrict__ zero32,
                                                             int64_t nzero32)
{
    __shared__ uint32_t h[kRadixMax];
    const int ndig = 1 << dbits;
    const uint32_t dmask = (uint32_t)ndig - 1u;
    for (int d = threadIdx.x; d < ndig; d += kSortThreads) h[d] = 0;
    if (zero) {
        for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < nzero;
             i += (int64_t)gridDim.x * kSortThreads)
            zero[i] = 0ull;
    }
    if (zero32) {
        for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < nzero32;
             i += (int64_t)gridDim.x * kSortThreads)
            zero32[i] = 0u;
    }
    __syncthreads();
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t e = base + sort_elem(j, wave, lane);
        const bool valid = e < n;
        uint32_t dig = 0;
        if (valid) {
            dig = (key_of(keys, e) >> shift) & dmask;
            // first pass: a boundary slot must hold a particle inside the grid
            if (!keys.keys && e < keys.nb && keys.cell[e] == SPH_EXCLUDED)
                atomicOr(dev_status, SPH_DEV_BOUNDARY_OUT);
        }
        add_digit_runs(h, valid, dig);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ndig; d += kSortThreads)
        hist[(int64_t)d * nblk + blockIdx.x] = h[d];
}

// Stable scatter.  Each wave ranks its own quarter of the tile round by round:
// lanes with equal digits are matched with ballots, and a per-wave running
// count per digit (LDS) gives each key its place among the wave's keys of
// that digit.  After one barrier the per-wave counts become per-wave offsets
// (waves in order), and every key goes to
// global offset of (digit, block) + offset of its wave + its rank.
// counts (last pass): every key is also counted, ks[key] += count << 32, one
// atomic per run of equal keys in a wave (the input of the last pass is
// sorted by the lower digits, so a cell's keys arrive together).
// next (first of two or more passes): the digit histogram of the next pass,
// next[digit * nblk + tile of the output slot] += count, taken here from the
// output slots instead of by a histogram launch of its own (equal keys go to
// consecutive slots, so again one atomic per run); next starts from zero.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    int32_t n, int shift, int dbits, KeySrc keys_in, const uint32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
    const uint32_t *__restrict__ offs, int nblk, unsigned long long *__restrict__ counts,
    uint32_t *__restrict__ next)
{
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint16_t wcnt[NW][kRadixMax];
    __shared__ uint32_t sbase[kRadixMax];
    const int ndig = 1 << dbits;
    const uint32_t dmask = (uint32_t)ndig - 1u;
    const int t = threadIdx.x;
    const int wave = t / kWave, lane = t % kWave;
    for (int d = t; d < NW * ndig; d += kSortThreads) wcnt[d / ndig][d % ndig] = 0;
    for (int d = t; d < ndig; d += kSortThreads) sbase[d] = offs[(int64_t)d * nblk + blockIdx.x];
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    uint32_t key[kSortItems], val[kSortItems];
    uint16_t rank[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t e = tile + sort_elem(j, wave, lane);
        const bool valid = e < n;
        uint32_t k = 0, v = 0, dig = 0;
        if (valid) {
            k = key_of(keys_in, e);
            v = vals_in ? vals_in[e] : (uint32_t)e;  // first pass: slot index
            dig = (k >> shift) & dmask;
        }
        unsigned long long peers = ballot(valid);
        for (int b = 0; b < dbits; ++b) {
            const bool bit = (dig >> b) & 1u;
            const unsigned long long m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        const unsigned rk = lane_rank(peers);
        if (counts)
            add_runs(valid, k, [&](uint32_t key, uint32_t c) {
                atomicAdd(&counts[key], (unsigned long long)c << 32);
            });
        uint32_t before = 0;
        if (valid) before = wcnt[wave][dig];
        // the wave's LDS accesses complete in order: every peer has read the
        // count before the first peer writes it back
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (valid && rk == 0) wcnt[wave][dig] = (uint16_t)(before + (uint32_t)__popcll(peers));
        key[j] = k;
        val[j] = v;
        rank[j] = (uint16_t)(valid ? before + rk : 0xffffu);
    }
    __syncthreads();
    // per-wave counts -> offsets of each wave among the block's keys of a digit
    for (int d = t; d < ndig; d += kSortThreads) {
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = wcnt[w][d];
            wcnt[w][d] = (uint16_t)run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const bool valid = rank[j] != 0xffffu;
        const uint32_t dig = (key[j] >> shift) & dmask;
        const uint32_t pos = valid ? sbase[dig] + wcnt[wave][dig] + rank[j] : 0u;
        if (next) {
            const uint32_t dn = (key[j] >> (shift + dbits)) & dmask;
            const uint32_t tn = pos / (uint32_t)kSortTile;
            add_runs(valid, (tn << kRadixBitsMax) | dn, [&](uint32_t, uint32_t c) {
                atomicAdd(&next[(int64_t)dn * nblk + tn], c);
            });
        }
        if (!valid) continue;
        keys_out[pos] = key[j];
        vals_out[pos] = val[j];
    }
}

// ---------------------------------------------------------------------------
// exclusive scan (reduce -> scan partials -> apply), in place

template <typename T>
__device__ T block_exclusive_scan(T v, T *sh, T *total)
{
    // sh: kScanThreads entries
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T add = t >= off ? sh[t - off] : (T)0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const T incl = sh[t];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

// MARK: the scanned value of element e is a[e] | 1 when a[e] != 0 (the
// packed (count << 32 | non-empty) key counts), applied on load.
template <typename T, bool MARK>
__device__ inline T scan_load(const T *a, int64_t e, int64_t len)
{
    if (e >= len) return (T)0;
    const T v = a[e];
    return MARK ? (v ? (T)(v | (T)1) : (T)0) : v;
}

// zero1 (optional): one int cleared on the side
template <typename T, bool MARK>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(int64_t len, const T *__restrict__ a,
                                                              unsigned long long *__restrict__ part,
                                                              int32_t *__restrict__ zero1)
{
    __shared__ T sh[kScanThreads];
    if (zero1 && blockIdx.x == 0 && threadIdx.x == 0) *zero1 = 0;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
    for (int j = 0; j < kScanItems; ++j)
        s += scan_load<T, MARK>(a, base + (int64_t)j * kScanThreads + threadIdx.x, len);
    T tot;
    block_exclusive_scan<T>(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = (unsigned long long)tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(int64_t np,
                                                                unsigned long long *__restrict__ part)
{
    __shared__ unsigned long long sh[kScanThreads];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < np; base += (int64_t)kScanThreads * kScanItems) {
        // each thread scans kScanItems consecutive partials serially
        unsigned long long loc[kScanItems];
        unsigned long long s = 0;
        const int64_t first = base + (int64_t)threadIdx.x * kScanItems;
        for (int j = 0; j < kScanItems; ++j) {
            const int64_t e = first + j;
            loc[j] = e < np ? part[e] : 0ull;
            s += loc[j];
        }
        unsigned long long tot;
        const unsigned long long ex = block_exclusive_scan<unsigned long long>(s, sh, &tot);
        unsigned long long run = carry + ex;
        for (int j = 0; j < kScanItems; ++j) {
            const int64_t e = first + j;
            if (e < np) part[e] = run;
            run += loc[j];
        }
        carry += tot;
        __syncthreads();
    }
}

// PREFIX: part[] holds tile totals and each block sums those before its own
// tile (few tiles); otherwise part[] already holds the exclusive prefixes.
template <typename T, bool MARK, bool PREFIX>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int64_t len, T *__restrict__ a,
                                                             const unsigned long long *__restrict__ part)
{
    // blocked: thread t owns kScanItems consecutive elements
    __shared__ T sh[kScanThreads];
    __shared__ unsigned long long sp[kScanThreads];
    unsigned long long base;
    if (PREFIX) {
        unsigned long long pre = 0;
        for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) pre += part[i];
        sp[threadIdx.x] = pre;
        __syncthreads();
        for (int o = kScanThreads / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sp[threadIdx.x] += sp[threadIdx.x + o];
            __syncthreads();
        }
        base = sp[0];
    } else {
        base = part[blockIdx.x];
    }
    const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T loc[kScanItems];
    T s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        loc[j] = scan_load<T, MARK>(a, first + j, len);
        s += loc[j];
    }
    T tot;
    const T ex = block_exclusive_scan<T>(s, sh, &tot);
    T run = (T)base + ex;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t e = first + j;
        if (e < len) a[e] = run;
        run += loc[j];
    }
}

// The reduce step above sums a strided layout and the apply step a blocked
// one; both cover exactly the tile [b * kScanTile, (b + 1) * kScanTile), so
// the per-tile totals agree.  Up to kScanFusedTiles tiles the apply blocks add
// up the tile totals themselves (two launches); beyond, one block scans them.
constexpr int64_t kScanFusedTiles = 1024;

template <typename T, bool MARK = false>
static hipError_t exclusive_scan(T *a, int64_t len, unsigned long long *part, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    const int64_t nblk = (len + kScanTile - 1) / kScanTile;
    k_scan_reduce<T, MARK><<<(unsigned)nblk, kScanThreads, 0, s>>>(len, a, part, nullptr);
    if (nblk <= kScanFusedTiles) {
        k_scan_apply<T, MARK, true><<<(unsigned)nblk, kScanThreads, 0, s>>>(len, a, part);
    } else {
        k_scan_partials<<<1, kScanThreads, 0, s>>>(nblk, part);
        k_scan_apply<T, MARK, false><<<(unsigned)nblk, kScanThreads, 0, s>>>(len, a, part);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cell ranges

__global__ void k_fill_u64(int64_t len, unsigned long long *__restrict__ a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] = 0ull;
}

// Cell ranges from the key counts: the apply step of the exclusive scan of
// the packed counts (count << 32 | non-empty mark), written out at once.  For
// key k the exclusive prefix is (first slot of k) << 32 | (number of non-empty
// keys before k): start[k] gets the first, a non-empty key gets list slot of
// the second; info[1] (fluid cells) is li(2 ncell) - li(ncell), added up by
// the two blocks holding those keys (the reduce step cleared it).
template <bool PREFIX>
__global__ __launch_bounds__(kScanThreads) void k_scan_emit(
    int64_t nkeys, int32_t n, int32_t ncell, const unsigned long long *__restrict__ ks,
    const unsigned long long *__restrict__ part, int32_t *__restrict__ start,
    int32_t *__restrict__ list, int32_t *__restrict__ info)
{
    using T = unsigned long long;
    __shared__ T sh[kScanThreads];
    __shared__ T sp[kScanThreads];
    const int64_t len = nkeys + 1;
    T base;
    if (PREFIX) {
        T pre = 0;
        for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) pre += part[i];
        sp[threadIdx.x] = pre;
        __syncthreads();
        for (int o = kScanThreads / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sp[threadIdx.x] += sp[threadIdx.x + o];
            __syncthreads();
        }
        base = sp[0];
    } else {
        base = part[blockIdx.x];
    }
    const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T raw[kScanItems], loc[kScanItems];
    T s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        raw[j] = first + j < len ? ks[first + j] : 0ull;
        loc[j] = scan_load<T, true>(ks, first + j, len);
        s += loc[j];
    }
    T tot;
    const T ex = block_exclusive_scan<T>(s, sh, &tot);
    T run = base + ex;
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t k = first + j;
        if (k > nkeys) break;
        const int32_t st = (int32_t)(run >> 32);
        const int32_t li = (int32_t)(run & 0xffffffffull);
        start[k] = st;
        if (k < nkeys) {
            if ((raw[j] >> 32) > 0 && k < 2 * (int64_t)ncell) list[li] = (int32_t)k;
            if (k == ncell) {
                info[0] = li;                  // boundary cells
                atomicAdd(&info[1], -li);
            }
            if (k == 2 * (int64_t)ncell) {
                atomicAdd(&info[1], li);       // fluid cells
                info[2] = n - st;              // excluded particles
                info[3] = 0;
            }
        }
        run += loc[j];
    }
}

// Interaction ranges (Section 4.4, optimisation D): for every cell with
// particles, the slot range [first, end) of each X-run of its stencil, per
// particle type.  Rows are indexed by cell, 2 (2n+1)^2 (first, end) pairs
// each; a cell that holds both boundary and fluid particles is written from
// its fluid key only, so every row has one writer.
__global__ void k_range_rows(int32_t ncell, int32_t nc0, int32_t nc1, int32_t nc2, int32_t nsub,
                             const int32_t *__restrict__ start, const int32_t *__restrict__ list,
                             const int32_t *__restrict__ info, int2 *__restrict__ rows)
{
    const int side = 2 * nsub + 1;
    const int per = 2 * side * side;
    const int64_t nlist = (int64_t)max(info[0], 0) + max(info[1], 0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nlist * per; t += stride) {
        const int64_t p = t / per;
        const int r = (int)(t - p * per);
        const int32_t key = list[p];
        const bool fluid = key >= ncell;
        const int32_t c = fluid ? key - ncell : key;
        if (!fluid && start[ncell + c + 1] > start[ncell + c]) continue;
        const int32_t cx = c % nc0, cy = (c / nc0) % nc1, cz = c / (nc0 * nc1);
        const int type = r / (side * side);
        const int rr = r - type * side * side;
        const int32_t y = cy + rr % side - nsub, z = cz + rr / side - nsub;
        int2 v = make_int2(0, 0);
        if (y >= 0 && y < nc1 && z >= 0 && z < nc2) {
            const int32_t x0 = max(cx - nsub, 0), x1 = min(cx + nsub, nc0 - 1);
            const int32_t k0 = (type ? ncell : 0) + x0 + nc0 * (y + nc1 * z);
            v = make_int2(start[k0], start[k0 + (x1 - x0 + 1)]);
        }
        rows[(int64_t)c * per + r] = v;
    }
}

// ---------------------------------------------------------------------------
// gather into sorted order

__global__ void k_gather(int32_t n, const uint32_t *__restrict__ perm,
                         const int32_t *__restrict__ cell_in, const float4 *__restrict__ pos_in,
                         const float4 *__restrict__ vr_in, const float4 *__restrict__ vp_in,
                         const int32_t *__restrict__ id_in, const double *__restrict__ x64_in,
                         int32_t *__restrict__ cell_out, float4 *__restrict__ pos_out,
                         float4 *__restrict__ vr_out, float4 *__restrict__ vp_out,
                         int32_t *__restrict__ id_out, double *__restrict__ x64_out,
                         int32_t *__restrict__ perm_out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    if (x64_in) {
        for (int d = 0; d < 3; ++d) x64_out[3 * (int64_t)i + d] = x64_in[3 * (int64_t)j + d];
    }
    cell_out[i] = cell_in[j];
    pos_out[i] = pos_in[j];
    vr_out[i] = vr_in[j];
    vp_out[i] = vp_in[j];
    id_out[i] = id_in[j];
    perm_out[i] = (int32_t)j;
}

hipError_t launch_build_cells(const sph_grid *g, const sph_state *src, sph_state *dst,
                              sph_cells *cells, int32_t *perm, const Workspace &w,
                              int32_t *dev_status, hipStream_t s)
{
    const int32_t n = src->n;
    const int32_t ncell = (int32_t)ncell_of(g);
    const int64_t nkeys = 2 * (int64_t)ncell + 1;  // keys 0 .. 2 ncell
    const int threads = 256;
    dst->n = src->n;
    dst->nb = src->nb;

    // 1-2. radix sort over the bits of the largest key, in the fewest passes
    // of at most kRadixBitsMax bits; the first pass reads the keys from the
    // cell array (and clears the key counts of step 3), the values are the slots
    int bits = 0;
    while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)(2 * (int64_t)ncell)) ++bits;
    const int npass = (bits + kRadixBitsMax - 1) / kRadixBitsMax;
    const int dbits = npass > 0 ? (bits + npass - 1) / npass : 0;
    uint32_t *kin = nullptr, *vin = nullptr, *kout = w.keys0, *vout = w.vals0;
    const int nblk = nblk_sort(n);
    const int64_t lenks = nkeys + 1;
    // The first pass's scatter takes the second pass's histogram (into hist2);
    // a third pass, if any, has a histogram launch of its own.
    bool cleared = false;
    const int64_t nhist = ((int64_t)1 << dbits) * nblk;
    for (int shift = 0, p = 0; shift < bits && n > 0; shift += dbits, ++p) {
        const KeySrc ks{kin, src->cell, src->nb, ncell};
        uint32_t *hist = p == 1 ? w.hist2 : w.hist;
        if (p != 1)
            k_radix_hist<<<nblk, kSortThreads, 0, s>>>(
                n, shift, dbits, ks, hist, nblk, dev_status, cleared ? nullptr : w.keyscan, lenks,
                p == 0 && npass > 1 ? w.hist2 : nullptr, nhist);
        cleared = true;
        hipError_t e = exclusive_scan<uint32_t>(hist, nhist, w.partials, s);
        if (e != hipSuccess) return e;
        const bool last = shift + dbits >= bits;
        k_radix_scatter<<<nblk, kSortThreads, 0, s>>>(n, shift, dbits, ks, vin, kout, vout, hist,
                                                      nblk, last ? w.keyscan : nullptr,
                                                      p == 0 && npass > 1 ? w.hist2 : nullptr);
        if (kin == nullptr) {
            kin = kout;
            vin = vout;
            kout = w.keys1;
            vout = w.vals1;
        } else {
            uint32_t *t;
            t = kin; kin = kout; kout = t;
            t = vin; vin = vout; vout = t;
        }
    }
    // 3. key counts (taken by the last pass) -> exclusive scan of the packed
    //    (count, non-empty) values, whose apply step writes the ranges
    if (!cleared)
        k_fill_u64<<<(unsigned)((lenks + threads - 1) / threads), threads, 0, s>>>(lenks, w.keyscan);
    {
        const int64_t nts = (lenks + kScanTile - 1) / kScanTile;
        k_scan_reduce<unsigned long long, true><<<(unsigned)nts, kScanThreads, 0, s>>>(
            lenks, w.keyscan, w.partials, cells->info + 1);
        if (nts <= kScanFusedTiles) {
            k_scan_emit<true><<<(unsigned)nts, kScanThreads, 0, s>>>(
                nkeys, n, ncell, w.keyscan, w.partials, cells->start, cells->list, cells->info);
        } else {
            k_scan_partials<<<1, kScanThreads, 0, s>>>(nts, w.partials);
            k_scan_emit<false><<<(unsigned)nts, kScanThreads, 0, s>>>(
                nkeys, n, ncell, w.keyscan, w.partials, cells->start, cells->list, cells->info);
        }
    }
    if (cells->ranges && n > 0) {
        // at most n listed keys, 2 (2n+1)^2 runs each
        const int side = 2 * g->nsub + 1;
        const int64_t work = (int64_t)n * 2 * side * side;
        const unsigned blocks = (unsigned)std::min<int64_t>((work + threads - 1) / threads, 4096);
        k_range_rows<<<blocks, threads, 0, s>>>(ncell, g->nc[0], g->nc[1], g->nc[2], g->nsub,
                                                cells->start, cells->list, cells->info,
                                                (int2 *)cells->ranges);
    }
    // 4. gather
    if (n > 0)
        k_gather<<<(n + threads - 1) / threads, threads, 0, s>>>(
            n, vin, src->cell, (const float4 *)src->pos, (const float4 *)src->velrho,
            (const float4 *)src->velrho_prev, src->id, src->pos64, dst->cell, (float4 *)dst->pos,
            (float4 *)dst->velrho, (float4 *)dst->velrho_prev, dst->id, dst->pos64, perm);
    return hipGetLastError();
}

}  // namespace sph
