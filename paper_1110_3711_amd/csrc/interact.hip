// interact.hip -- particle-interaction stage (Section 2 "PI"): fluid targets
// (F-F and F-B fused, Section 4.5) and boundary targets (B-F), and the
// vector-Jacobian product of the same pair terms.
//
// Work decomposition (gfx950, wave64):
//   * one workgroup per non-empty target cell, taken from device work queues
//     (dynamic scheduling, like the OpenMP dynamic scheduler of Section 3.4):
//     the fluid cell list is cut into one chunk per XCD, so that cells with
//     common stencil neighbours run on the XCD that caches them; a full stage
//     is one launch in which the boundary cells with fluid in reach are
//     interleaved with the fluid cells;
//   * the (2n+1)^2 X-runs of the stencil (Section 4.4: three consecutive
//     cells along X are one contiguous range of the sorted arrays) are staged
//     into LDS in the frame of the target cell: each candidate's offset gets
//     (k_b - k_a) * cell added once, in FP32 (the shift is exact for
//     |k_b - k_a| <= 2, the sum is rounded once), and the staged candidates
//     are ordered by 32 bins of their x, so that a
//     target scans only the window of bins within 2h of its own x;
//   * one wavefront per target: 64 candidates per step are tested for
//     r^2 < (2h)^2, survivors are compacted with a ballot into a per-wave ring
//     in LDS, and every full batch of 64 survivors is evaluated with all lanes
//     busy.  This removes the divergence of a thread-per-target loop (the
//     "code divergence" problem of Section 4) without any neighbour list in
//     HBM;
//   * per-lane partial sums are reduced across the wave once per target (DPP
//     butterflies) and written once (Section 4.5: accumulate in registers,
//     write at the end).  No float atomics: results are bitwise reproducible.
//
// The target itself is one of its staged candidates: it passes the distance
// test with r = 0 and contributes exactly zero to every sum (r_ab = 0,
// v_ab = 0, mu = 0), so it is not filtered per candidate; it is only removed
// from the pair count.
//
// Template parameters of the kernels: the work-list kind (fluid, boundary,
// or both in one launch; forward or adjoint), per-pair diagnostics (STATS),
// the kernel shape (KER: Wendland quintic or cubic spline) and the tensile
// correction (TENS).
#include "sph_internal.h"

namespace sph {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / kWave;
constexpr int kTile = 2048;          // candidates staged per pass (multiple of 64)
constexpr int kRing = 256;           // per-wave ring of compacted candidates
constexpr int kMaxRuns = 2 * 25;     // types x (2n+1)^2, n <= 2
constexpr float kFar = 1.0e30f;      // padding position: never within the support
constexpr int kXcds = 8;             // MI355X: workgroups are dealt to 8 XCDs round robin
constexpr int kPad = 3 * kWave;      // padding entries after the placed candidates
constexpr int kBinBits = 5;          // staged candidates are ordered by 32 bins of x
constexpr int kBins = 1 << kBinBits;
// work queue of a list: kXcds chunk counters, the pool counter, the flag word
// (counter slots, kCounterStride ints apart)
constexpr int kQPool = kXcds;
constexpr int kQFlags = kXcds + 1;
constexpr int kPool64 = 10;          // the pool: the last 10/64 of the list

struct RunTable {
    int32_t nruns;
    int32_t total;                          // candidates over all runs
    int32_t vstart[kMaxRuns + 1];           // prefix of run lengths
    int32_t s[kMaxRuns];                    // first slot of the run
    float sy[kMaxRuns], sz[kMaxRuns];       // dy * cell, dz * cell
    int32_t cb[kMaxRuns];                   // linear index of cell (cx, cy + dy, cz + dz)
    int32_t self_run;                       // run holding the target cell's own fluid particles
};

// ---------------------------------------------------------------------------
// wave reductions: DPP within rows of 16 lanes, then the four row results

template <int CTRL>
__device__ inline int dpp_i(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ inline float dpp_f(float v)
{
    return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}

__device__ inline float readlane_f(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E, row_half_mirror = 0x141,
// row_mirror = 0x140: after the four steps every lane holds its row's sum.
__device__ inline float wave_sum(float v)
{
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

__device__ inline unsigned wave_max_u(unsigned v)
{
    v = max(v, (unsigned)dpp_i<0xB1>((int)v));
    v = max(v, (unsigned)dpp_i<0x4E>((int)v));
    v = max(v, (unsigned)dpp_i<0x141>((int)v));
    v = max(v, (unsigned)dpp_i<0x140>((int)v));
    const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
    const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
    const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
    const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
    return max(max(a, b), max(c, d));
}

__device__ inline unsigned wave_sum_u(unsigned v)
{
    v += (unsigned)dpp_i<0xB1>((int)v);
    v += (unsigned)dpp_i<0x4E>((int)v);
    v += (unsigned)dpp_i<0x141>((int)v);
    v += (unsigned)dpp_i<0x140>((int)v);
    return (unsigned)__builtin_amdgcn_readlane((int)v, 0) +
           (unsigned)__builtin_amdgcn_readlane((int)v, 16) +
           (unsigned)__builtin_amdgcn_readlane((int)v, 32) +
           (unsigned)__builtin_amdgcn_readlane((int)v, 48);
}

// Inclusive prefix sum over the 64 lanes of a wave without LDS round trips:
// row_shr:1,2,4,8 (lanes without a source add the 0 of `old`) scan each row
// of 16 lanes, then every row adds the totals of the rows below it.
__device__ inline int32_t wave_scan_incl(int32_t v, int lane)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    const int32_t r0 = __builtin_amdgcn_readlane(v, 15);
    const int32_t r1 = __builtin_amdgcn_readlane(v, 31);
    const int32_t r2 = __builtin_amdgcn_readlane(v, 47);
    return v + (lane >= 16 ? r0 : 0) + (lane >= 32 ? r1 : 0) + (lane >= 48 ? r2 : 0);
}

// one exchange step of a transposed reduction: lanes with the bit clear keep lo
// and add the partner's lo, lanes with the bit set keep hi and add the
// partner's hi, so the number of live values halves while each covers twice
// the lanes
template <int CTRL>
__device__ inline float xchg(float lo, float hi, bool bit)
{
    return (bit ? hi : lo) + dpp_f<CTRL>(bit ? lo : hi);
}

// Cross-row steps use ds_bpermute with the byte addresses of lanes l ^ 16 and
// l ^ 32 (computed once per thread).
struct XorAddr {
    int x16, x32;
};

__device__ inline XorAddr xor_addr(int lane)
{
    return XorAddr{(lane ^ 16) << 2, (lane ^ 32) << 2};
}

__device__ inline float bperm_f(int addr, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}

// row_ror:4 = 0x124, row_ror:8 = 0x128 (rotations keep lane & 3)
// Sums of four per-lane values over the wave: lane l ends with the total of
// value (l & 3).
__device__ inline float wave_sum4(float v0, float v1, float v2, float v3, int lane, XorAddr xa)
{
    const bool b0 = lane & 1, b1 = lane & 2;
    const float x = xchg<0xB1>(v0, v1, b0);
    const float y = xchg<0xB1>(v2, v3, b0);
    float z = xchg<0x4E>(x, y, b1);
    z += dpp_f<0x124>(z);
    z += dpp_f<0x128>(z);
    z += bperm_f(xa.x16, z);
    z += bperm_f(xa.x32, z);
    return z;
}

// Sums of eight per-lane values: lane l ends with the total of value (l & 7).
// The third exchange pairs quads q and q + 1 (mod 4) of a row by rotation;
// with the row_ror:8 step after it every quad sum is counted once.
__device__ inline float wave_sum8(float v0, float v1, float v2, float v3, float v4, float v5,
                                  float v6, float v7, int lane, XorAddr xa)
{
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    const float x0 = xchg<0xB1>(v0, v1, b0), x1 = xchg<0xB1>(v2, v3, b0);
    const float x2 = xchg<0xB1>(v4, v5, b0), x3 = xchg<0xB1>(v6, v7, b0);
    const float y0 = xchg<0x4E>(x0, x1, b1), y1 = xchg<0x4E>(x2, x3, b1);
    float z = xchg<0x124>(y0, y1, b2);
    z += dpp_f<0x128>(z);
    z += bperm_f(xa.x16, z);
    z += bperm_f(xa.x32, z);
    return z;
}

// maximum of non-negative floats over the wave (their bit patterns order as
// unsigned integers), in every lane
__device__ inline float wave_max_nonneg(float f, XorAddr xa)
{
    unsigned v = __builtin_bit_cast(unsigned, f);
    v = max(v, (unsigned)dpp_i<0xB1>((int)v));
    v = max(v, (unsigned)dpp_i<0x4E>((int)v));
    v = max(v, (unsigned)dpp_i<0x124>((int)v));
    v = max(v, (unsigned)dpp_i<0x128>((int)v));
    v = max(v, (unsigned)__builtin_amdgcn_ds_bpermute(xa.x16, (int)v));
    v = max(v, (unsigned)__builtin_amdgcn_ds_bpermute(xa.x32, (int)v));
    return __builtin_bit_cast(float, v);
}

// LDS byte addressing
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f32x4 lds_f32x4;

__device__ inline float4 lds_load4(uint32_t addr)
{
    const f32x4 v = *(const lds_f32x4 *)(uintptr_t)addr;
    return make_float4(v.x, v.y, v.z, v.w);
}

// LDS byte address of a generic pointer into LDS: the low 32 bits of the
// generic address (the shared aperture's base is 4 GiB aligned).  Unlike an
// address-space cast this carries no null test, which the compiler would
// otherwise re-evaluate wherever it recomputes the address.
__device__ inline uint32_t lds_addr(const void *p)
{
    return (uint32_t)(uintptr_t)p;
}

// ---------------------------------------------------------------------------
// stencil runs of a target cell

// Build the run table of target cell c = (cx, cy, cz).  FLUID: candidates
// are boundary and fluid particles; otherwise fluid only.  With precomputed
// interaction ranges (rows != nullptr, Section 4.4 optimisation D) each run
// is read from the cell's row, otherwise from the starts of its first cell
// and of the cell after its last one.
template <bool FLUID>
__device__ void build_runs(const PairConsts &K, const int32_t *__restrict__ start,
                           const int2 *__restrict__ rows, int32_t c, int32_t cx, int32_t cy,
                           int32_t cz, RunTable &R)
{
    const int n = K.nsub;
    const int side = 2 * n + 1;
    const int nr = (FLUID ? 2 : 1) * side * side;
    const int32_t x0 = max(cx - n, 0);
    const int32_t x1 = min(cx + n, K.nc0 - 1);
    const int ncx = x1 - x0 + 1;
    int32_t len = 0;
    if ((int)threadIdx.x < nr) {
        const int r = threadIdx.x;
        const int type = FLUID ? r / (side * side) : 1;  // 0 boundary, 1 fluid
        const int rr = r % (side * side);
        const int dy = rr % side - n, dz = rr / side - n;
        const int32_t y = cy + dy, z = cz + dz;
        const bool ok = y >= 0 && y < K.nc1 && z >= 0 && z < K.nc2;
        int2 be;
        if (rows) {
            // row of cell c: (first, end) of type `type`, run rr
            be = rows[(int64_t)c * (2 * side * side) + type * side * side + rr];
        } else {
            // key of the run's first cell; key0 + ncx <= 2 ncell, and 0 + ncx
            // <= ncell for a run outside the grid, so both loads are in bounds
            const int32_t key0 = ok ? (type ? K.ncell : 0) + x0 + K.nc0 * (y + K.nc1 * z) : 0;
            be = make_int2(start[key0], start[key0 + ncx]);
        }
        const int32_t s0 = ok ? be.x : 0, se = ok ? be.y : 0;
        R.s[r] = s0;
        R.cb[r] = ok ? cx + K.nc0 * (y + K.nc1 * z) : 0;
        R.sy[r] = (float)dy * K.cellf;
        R.sz[r] = (float)dz * K.cellf;
        if (type == 1 && dy == 0 && dz == 0) R.self_run = r;
        len = ok ? se - s0 : 0;
    }
    // inclusive scan of the run lengths over the first wavefront (nr <= 50)
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        const int32_t v = wave_scan_incl(len, lane);
        if (lane < nr) R.vstart[lane + 1] = v;
        if (lane == 0) R.vstart[0] = 0;
        if (lane == nr - 1) {
            R.total = v;
            R.nruns = nr;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// pair kernel: forward (targets) and backward (gatherers) share the work
// queue, the stencil staging and the ballot compaction.

enum Kind { kFwdFluid = 0, kFwdBound = 1, kBwdFluid = 2, kBwdBound = 3, kFwdAll = 4, kBwdAll = 5 };

struct PairArgs {
    const int32_t *start, *items, *counts;
    const int32_t *items2, *counts2;  // fused launches: active boundary cells, their count
    const int2 *ranges;       // precomputed interaction ranges of the cells, or nullptr
    const int32_t *cell;      // cell of each slot (the frame shift of a staged candidate)
    const float4 *pos, *velrho;
    const double *pos64;      // SPH_POS_ABS64: FP64 absolute positions [3n]
    const int32_t *ids;
    float4 *ace;        // forward: out (a, drho/dt); backward: in (abar, Dbar)
    float *visc;        // forward: out max |mu|
    float4 *xbar;       // backward: pos_bar (+=)
    float4 *vbar;       // backward: velrho_bar (+=)
    float *alpha_part;  // backward: per-slot alpha adjoint of fluid targets
    int32_t *queue;     // kXcds counters of the first work list
    int32_t *queue2;    // fused launches: counter of the boundary work list
    unsigned long long *npairs;  // [2]: += fluid-target, boundary-target pairs
    int32_t *stats;
};

// A launch runs one work list (fluid target cells or active boundary cells),
// or both in turn (the fused kinds: fluid cells first, then boundary cells,
// so the short boundary items fill the tail of the launch).
template <int KIND, int POS = 0>
struct KindTraits {
    static constexpr bool fused = KIND == kFwdAll || KIND == kBwdAll;
    static constexpr bool bwd = KIND == kBwdFluid || KIND == kBwdBound || KIND == kBwdAll;
    static constexpr bool fluid = KIND == kFwdFluid || KIND == kBwdFluid || fused;  // first list
    // LDS per candidate: 32 B (forward), 48 B (backward), 56 B (forward with
    // FP64 positions)
    static constexpr int tile = bwd ? 1408 : (POS ? 1024 : kTile);
    static constexpr int first = fused ? (bwd ? kBwdFluid : kFwdFluid) : KIND;
    static constexpr int second = bwd ? kBwdBound : kFwdBound;
};

// LDS of one workgroup
template <int TILE, bool BWD, bool STATS, int POS = 0>
struct PairLds {
    static constexpr int STAGE = (TILE + kThreads - 1) / kThreads;
    static constexpr int DTILE = POS ? TILE + kPad : 1;
    double sDx[DTILE], sDy[DTILE], sDz[DTILE];  // SPH_POS_ABS64: x_b - centre of the
                                            //   target cell, FP64, + padding
    float4 sP[TILE + kPad];                 // (offset in target frame, P/rho^2) + padding
    float4 sV[TILE];                        // (v, rho - rho0)
    float4 sA[BWD ? TILE : 1];              // backward: (abar, Dbar), abar = 0 on boundary
    alignas(512) uint16_t sRing[kWaves][kRing];  // 512 bytes per wave
    uint16_t sTrash[kWaves][kWave];         // rejected candidates land here
    union {
        uint16_t sMap[TILE];                // fluid targets: staging index -> sorted slot
        float4 sTgt[TILE / 8];              // boundary targets: (pos, velrho) of the first
    };                                      //   TILE / 16 targets of the cell
    uint16_t sCnt[STAGE][kWaves][kBins];
    int32_t sBin[kBins + 1];                // first sorted slot of each x-bin
    int32_t sSlot[STATS ? TILE : 1];        // candidate slot (diagnostics only)
    RunTable R;
    int32_t sItem;
    int32_t sKind;                          // fused launches: 0 fluid item, 1 boundary item
};

// per-lane constants: LDS byte addresses of this wave's ring (512-aligned),
// the lane's first read entry and trash slot, the staged arrays
struct LaneCtx {
    int lane, wave;
    uint32_t rbase, rfirst, lane16, taddr, sPb, sVb, sAb, sTb;
    XorAddr xa;
};

// One work item: the targets of cell `key` (of the list kind KIND) against
// its stencil, staged tile by tile through the workgroup's LDS.
template <int KIND, bool STATS, int KER, bool TENS, int POS, class L>
__device__ __forceinline__ void pair_item(const PairConsts &K, const PairArgs &A, L &S,
                                          const LaneCtx &C, int32_t key,
                                          unsigned long long &pairs_acc)
{
    using T = KindTraits<KIND, POS>;
    constexpr bool FLUID = T::fluid;
    constexpr bool BWD = T::bwd;
    constexpr int TILE = T::tile;
    constexpr int STAGE = L::STAGE;
    auto &sP = S.sP;
    auto &sV = S.sV;
    auto &sA = S.sA;
    auto &sMap = S.sMap;
    auto &sCnt = S.sCnt;
    auto &sBin = S.sBin;
    auto &sSlot = S.sSlot;
    auto &R = S.R;
    const int lane = C.lane, wave = C.wave;
    const uint32_t rbase = C.rbase, rfirst = C.rfirst, lane16 = C.lane16, taddr = C.taddr;
    const uint32_t sPb = C.sPb, sVb = C.sVb, sAb = C.sAb;
    const XorAddr xa = C.xa;
    auto xbin = [&](float x) { return min(max((int)((x - K.xlo) * K.xscale), 0), kBins - 1); };

    const int32_t c = FLUID ? max(key - K.ncell, 0) : min(key, K.ncell - 1);
    const int32_t cx = c % K.nc0, cy = (c / K.nc0) % K.nc1, cz = c / (K.nc0 * K.nc1);
    // SPH_POS_ABS64: FP64 centre of the target cell; staged candidates and the
    // targets hold x - centre in FP64, and r_ab = fp32(x_a - x_b) from those
    double ctx = 0.0, cty = 0.0, ctz = 0.0;
    if (POS) {
        ctx = fma((double)cx + 0.5, K.cell64, K.org64[0]);
        cty = fma((double)cy + 0.5, K.cell64, K.org64[1]);
        ctz = fma((double)cz + 0.5, K.cell64, K.org64[2]);
    }
    const int32_t tbeg = __builtin_amdgcn_readfirstlane(min(max(A.start[key], 0), K.n));
    const int32_t tend = __builtin_amdgcn_readfirstlane(min(max(A.start[key + 1], tbeg), K.n));

    build_runs<FLUID>(K, A.start, A.ranges, c, cx, cy, cz, R);
    const int32_t total = __builtin_amdgcn_readfirstlane(R.total);
    const int nr = __builtin_amdgcn_readfirstlane(R.nruns);
    const int nbruns = FLUID ? nr / 2 : 0;  // runs [0, nbruns) hold boundary particles

    for (int32_t tb = 0; tb < max(total, 1); tb += TILE) {
        const int32_t tlen = max(min(TILE, total - tb), 0);
        // ---- stage candidates [tb, tb + tlen) into LDS, ordered by the x-bin of
        //      their position in the target frame (stable in staging order), so
        //      that each target scans one contiguous window |x_a - x_b| < 2h
        // locate staging index l: slot j of the sorted state and its run
        auto locate = [&](int32_t l, int32_t &j, int &run) {
            const int32_t v = tb + min(l, max(tlen - 1, 0));
            int lo = 0, hi = nr;  // find r with vstart[r] <= v < vstart[r+1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (R.vstart[mid] <= v) lo = mid;
                else hi = mid;
            }
            j = min(max(R.s[lo] + (v - R.vstart[lo]), 0), K.n - 1);
            run = lo;
        };
        // frame shift (k_b - k_a) cell along x, exact: the candidate's cell and
        // the run's centre cell differ by k_b - k_a in x
        auto shift_x = [&](int32_t j, int run) {
            return (float)(A.cell[j] - R.cb[run]) * K.cellf;
        };
        // Candidates farther than 2h from the target cell (box distance of
        // their staged position) interact with none of its targets: they are
        // neither ranked nor placed.  The margins (box half-side enlarged by
        // 2^-20, cutoff by 2^-10) exceed the FP32 rounding of the pair test,
        // so the kept candidates are exactly those that can pass it, in the
        // same order: results are bitwise those of staging everything.
        auto kept = [&](int u, const float4 p, float sx, int run) {
            if ((int32_t)(threadIdx.x + u * kThreads) >= tlen) return false;
            const float tx = fmaxf(fabsf(p.x + sx) - K.half, 0.f);
            const float ty = fmaxf(fabsf(p.y + R.sy[run]) - K.half, 0.f);
            const float tz = fmaxf(fabsf(p.z + R.sz[run]) - K.half, 0.f);
            return __builtin_fmaf(tz, tz, __builtin_fmaf(ty, ty, tx * tx)) < K.cull2;
        };
        // rank among the equal x-bins of this wave (stable in lane order)
        auto rank_round = [&](int u, int bin, bool valid) {
            unsigned long long peers = ballot(valid);
            for (int b = 0; b < kBinBits; ++b) {
                const bool bit = (bin >> b) & 1;
                const unsigned long long mb = ballot(bit);
                peers &= bit ? mb : ~mb;
            }
            const int rk = (int)lane_rank(peers);
            if (valid && rk == 0) sCnt[u][wave][bin] = (uint16_t)__popcll(peers);
            return rk;
        };
        static_assert(STAGE <= 4, "staging rounds");
        // boundary targets are not among the (fluid) candidates: stage the
        // cell's first kTgt targets with the candidates
        constexpr int32_t kTgt = TILE / 16;
        if (!FLUID && tb == 0 && (int32_t)threadIdx.x < min(tend - tbeg, kTgt)) {
            const float4 tp = A.pos[tbeg + threadIdx.x], tv = A.velrho[tbeg + threadIdx.x];
            S.sTgt[2 * threadIdx.x] = tp;
            S.sTgt[2 * threadIdx.x + 1] = tv;
        }
        for (int i = threadIdx.x; i < STAGE * kWaves * kBins; i += kThreads)
            (&sCnt[0][0][0])[i] = 0;
        // pass A: locate all of this thread's candidates, then one round of loads
        int32_t j0 = 0, j1 = 0, j2 = 0, j3 = 0;
        int q0 = 0, q1 = 0, q2 = 0, q3 = 0;
        locate(threadIdx.x, j0, q0);
        if (STAGE > 1) locate(threadIdx.x + kThreads, j1, q1);
        if (STAGE > 2) locate(threadIdx.x + 2 * kThreads, j2, q2);
        if (STAGE > 3) locate(threadIdx.x + 3 * kThreads, j3, q3);
        const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 p0 = A.pos[j0], p1 = STAGE > 1 ? A.pos[j1] : zero4,
                     p2 = STAGE > 2 ? A.pos[j2] : zero4, p3 = STAGE > 3 ? A.pos[j3] : zero4;
        const float sx0 = shift_x(j0, q0), sx1 = STAGE > 1 ? shift_x(j1, q1) : 0.f,
                    sx2 = STAGE > 2 ? shift_x(j2, q2) : 0.f, sx3 = STAGE > 3 ? shift_x(j3, q3) : 0.f;
        const int bn0 = xbin(p0.x + sx0);
        const int bn1 = STAGE > 1 ? xbin(p1.x + sx1) : 0;
        const int bn2 = STAGE > 2 ? xbin(p2.x + sx2) : 0;
        const int bn3 = STAGE > 3 ? xbin(p3.x + sx3) : 0;
        const bool kp0 = kept(0, p0, sx0, q0);
        const bool kp1 = STAGE > 1 ? kept(1, p1, sx1, q1) : false;
        const bool kp2 = STAGE > 2 ? kept(2, p2, sx2, q2) : false;
        const bool kp3 = STAGE > 3 ? kept(3, p3, sx3, q3) : false;
        __syncthreads();
        const int rk0 = rank_round(0, bn0, kp0);
        const int rk1 = STAGE > 1 ? rank_round(1, bn1, kp1) : 0;
        const int rk2 = STAGE > 2 ? rank_round(2, bn2, kp2) : 0;
        const int rk3 = STAGE > 3 ? rank_round(3, bn3, kp3) : 0;
        __syncthreads();
        // per-bin offsets over (round, wave), then the bin starts (exclusive
        // scan of the bin totals), both in the first wavefront; the counts are
        // read eight at a time ahead of their running sums (four LDS round
        // trips per bin instead of one per count)
        static_assert(kBins <= kWave, "one lane per x-bin");
        if (threadIdx.x < kWave) {
            const int b = threadIdx.x;
            int32_t run = 0;
            if (b < kBins) {
                uint16_t *const cnt = &sCnt[0][0][0];
#pragma unroll
                for (int k0 = 0; k0 < STAGE * kWaves; k0 += 8) {
                    uint16_t cc[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) cc[k] = cnt[(k0 + k) * kBins + b];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        cnt[(k0 + k) * kBins + b] = (uint16_t)run;
                        run += cc[k];
                    }
                }
            }
            const int32_t v = wave_scan_incl(run, b);
            if (b < kBins) sBin[b + 1] = v;
            if (b == 0) sBin[0] = 0;
        }
        __syncthreads();
        // pass B: write each candidate to its sorted slot
        // pass B reads the candidate's cell again, except in the tensile kinds,
        // where keeping the shift of pass A leaves their 128-VGPR budget more
        // room (1.8% faster there, 0.2% slower in the default kind)
        auto place = [&](int u, int32_t j, int run, int bin, int rk, float sx, bool keep) {
            const int32_t l = threadIdx.x + u * kThreads;
            if (!keep) return;
            const int slot = sBin[bin] + sCnt[u][wave][bin] + rk;
            float4 pp = A.pos[j];
            if (POS) {
                const double dx = A.pos64[3 * (int64_t)j] - ctx;
                const double dy = A.pos64[3 * (int64_t)j + 1] - cty;
                const double dz = A.pos64[3 * (int64_t)j + 2] - ctz;
                S.sDx[slot] = dx;
                S.sDy[slot] = dy;
                S.sDz[slot] = dz;
                pp.x = (float)dx;
                pp.y = (float)dy;
                pp.z = (float)dz;
            } else {
                pp.x += TENS ? sx : shift_x(j, run);
                pp.y += R.sy[run];
                pp.z += R.sz[run];
            }
            sP[slot] = pp;
            sV[slot] = A.velrho[j];
            if (BWD) {
                float4 ab = A.ace[j];
                if (run < nbruns) ab.x = ab.y = ab.z = 0.f;
                sA[slot] = ab;
            }
            if (STATS) sSlot[slot] = j;
            if (FLUID) sMap[l] = (uint16_t)slot;
        };
        place(0, j0, q0, bn0, rk0, sx0, kp0);
        if (STAGE > 1) place(1, j1, q1, bn1, rk1, sx1, kp1);
        if (STAGE > 2) place(2, j2, q2, bn2, rk2, sx2, kp2);
        if (STAGE > 3) place(3, j3, q3, bn3, rk3, sx3, kp3);
        // padding after the placed candidates: the chunks of a window end
        // before sBin[kBins] + kPad
        const int32_t nplaced = sBin[kBins];
        if (threadIdx.x < kPad) {
            sP[nplaced + threadIdx.x] = make_float4(kFar, kFar, kFar, 0.f);
            if (POS) {
                S.sDx[nplaced + threadIdx.x] = (double)kFar;
                S.sDy[nplaced + threadIdx.x] = (double)kFar;
                S.sDz[nplaced + threadIdx.x] = (double)kFar;
            }
        }
        __syncthreads();

        // ---- one wavefront per target
        const int32_t selfbase =
            FLUID ? __builtin_amdgcn_readfirstlane(R.vstart[R.self_run] - R.s[R.self_run]) - tb
                  : 0;
        // LDS slot of a target staged in this tile (its staging index is
        // selfbase + a; targets are never dropped by the staging's box
        // test), or -1; read one target ahead, before the current target's
        // candidate scan, to take an LDS round trip off each target's start
        auto slot_of = [&](int32_t a) -> int32_t {
            const int32_t v = selfbase + a;
            return (FLUID && v >= 0 && v < tlen) ? (int32_t)sMap[v] : -1;
        };
        int32_t next_l = slot_of(tbeg + wave);
        for (int32_t a = tbeg + wave; a < tend; a += kWaves) {
            const bool self_here = FLUID && next_l >= 0;
            const int32_t self_l = max(next_l, 0);
            // LDS reads through LDS addresses, global reads through global
            // pointers, in separate (wave-uniform) branches: a select between
            // the two pointers would turn every one of them into a flat load
            float4 pa, va, aa = make_float4(0.f, 0.f, 0.f, 0.f);
            if (self_here) {
                const uint32_t off = (uint32_t)self_l << 4;
                pa = lds_load4(sPb + off);
                va = lds_load4(sVb + off);
                if (BWD) aa = lds_load4(sAb + off);
            } else if (!FLUID && a - tbeg < kTgt) {
                const uint32_t off = (uint32_t)(a - tbeg) << 5;
                pa = lds_load4(C.sTb + off);
                va = lds_load4(C.sTb + off + 16);
            } else {
                pa = A.pos[a];
                va = A.velrho[a];
                if (BWD && FLUID) aa = A.ace[a];
            }
            double pax = 0.0, pay = 0.0, paz = 0.0;  // SPH_POS_ABS64 target position
            if (POS) {
                if (self_here) {
                    pax = S.sDx[self_l];
                    pay = S.sDy[self_l];
                    paz = S.sDz[self_l];
                } else {
                    pax = A.pos64[3 * (int64_t)a] - ctx;
                    pay = A.pos64[3 * (int64_t)a + 1] - cty;
                    paz = A.pos64[3 * (int64_t)a + 2] - ctz;
                }
                pa.x = (float)pax;
                pa.y = (float)pay;
                pa.z = (float)paz;
            }
            // t = rho / rho0; the Monaghan factor cbar / rhobar for c = c0 t^3 is
            // (c0 / rho0) (ta^3 + tb^3) / (ta + tb) = (c0 / rho0) (ta^2 - ta tb + tb^2)
            const float ta = __builtin_fmaf(va.w, K.inv_rho0, 1.0f);
            const float ta2 = ta * ta;
            // forward: Pi_ab = kh (ta^2 - ta tb + tb^2) min(u, 0), u = v.r / (r^2 + eta2),
            // evaluated as tb (kh tb - kh ta) + kh ta^2
            const float kta = -K.kh * ta, kta2 = K.kh * ta2;
            // backward: d(P/rho^2)/drho = c^2 / rho^2 - 2 (P/rho^2) / rho, c = c0 ta^3
            float dpa = 0.f;
            if (BWD) {
                const float inv_ra = __builtin_amdgcn_rcpf(K.rho0 * ta);
                const float ca = K.c0 * ta2 * ta;
                dpa = (ca * inv_ra) * (ca * inv_ra) - 2.f * pa.w * inv_ra;
            }
            // tensile correction: R_a = eps_a P_a/rho_a^2, eps = 0.01 (P > 0) or
            // -0.2 (P < 0); backward: dR_a/drho_a = eps_a d(P/rho^2)/drho
            const float eps_a = pa.w > 0.f ? 0.01f : -0.2f;
            const float ra_t = TENS ? eps_a * pa.w : 0.f;
            const float eda = TENS ? eps_a * dpa : 0.f;
            // accumulators: forward (s0..s3 = sums for a.xyz and drho in units of
            // gs, vmf = max |u|); backward (s0..s2 = xbar, s3 = rhobar, s4..s6 = vbar,
            // s7 = alphabar)
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f, s6 = 0.f,
                  s7 = 0.f, vmf = 0.f;
            unsigned hs = 0;
            int wp = 0, rp = 0;          // ring write / read counters (wave-uniform)
            uint32_t raddr = rfirst;     // this lane's ring entry of the next batch

            // one batch: every lane evaluates the pair with the staged entry at
            // byte offset off
            auto pair = [&](uint32_t off) {
                const float4 pb = lds_load4(sPb + off);
                const float4 vb = lds_load4(sVb + off);
                float rx, ry, rz;
                if (POS) {
                    const int ix = (int)(off >> 4);
                    rx = (float)(pax - S.sDx[ix]);
                    ry = (float)(pay - S.sDy[ix]);
                    rz = (float)(paz - S.sDz[ix]);
                } else {
                    rx = pa.x - pb.x;
                    ry = pa.y - pb.y;
                    rz = pa.z - pb.z;
                }
                const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
                // the adjoint needs 1/r too: one reciprocal square root instead of
                // a square root and a reciprocal (r = 0 only for the target itself)
                float r, ir = 0.f;
                if (BWD) {
                    ir = __builtin_amdgcn_rsqf(r2);
                    r = r2 > 0.f ? r2 * ir : 0.f;
                } else {
                    r = __builtin_amdgcn_sqrtf(r2);
                }
                // kernel gradient factor in units of gs: F = gs G (grad_a W = F r_ab)
                float G, wq = 0.f, qq = 0.f;
                if (KER == SPH_WENDLAND5) {
                    wq = __builtin_fmaf(-0.5f * K.inv_h, r, 1.0f);
                    G = wq * wq * wq;
                } else {
                    qq = r * K.inv_h;
                    const float t = 2.f - qq;
                    G = qq < 1.f ? __builtin_fmaf(2.25f, qq, -3.f)
                                 : K.kco * (t * t) * __builtin_amdgcn_rcpf(r);
                }
                // tensile correction: f = Wn(r) / Wn(dp), R_ab = R_a + R_b
                float f4 = 0.f, f3 = 0.f, rab = 0.f;
                if (TENS && (FLUID || BWD)) {
                    float wn;
                    if (KER == SPH_WENDLAND5) {
                        const float wq2 = wq * wq;
                        wn = (wq2 * wq2) * __builtin_fmaf(2.f * K.inv_h, r, 1.f);
                    } else {
                        const float t = 2.f - qq;
                        wn = qq < 1.f ? __builtin_fmaf(qq * qq, __builtin_fmaf(0.75f, qq, -1.5f), 1.f)
                                      : 0.25f * (t * t) * t;
                    }
                    const float f = wn * K.inv_wndp;
                    const float f2 = f * f;
                    f3 = f2 * f;
                    f4 = f2 * f2;
                    rab = __builtin_fmaf(pb.w, pb.w > 0.f ? 0.01f : -0.2f, ra_t);
                }
                const float vx = va.x - vb.x, vy = va.y - vb.y, vz = va.z - vb.z;
                const float vdr = __builtin_fmaf(vz, rz, __builtin_fmaf(vy, ry, vx * rx));
                if (!BWD) {
                    s3 = __builtin_fmaf(vdr, G, s3);
                    if (FLUID) {
                        const float u = vdr * __builtin_amdgcn_rcpf(r2 + K.eta2);
                        vmf = fmaxf(vmf, fabsf(u));
                        const float tb = __builtin_fmaf(vb.w, K.inv_rho0, 1.0f);
                        const float crk = __builtin_fmaf(tb, __builtin_fmaf(tb, K.kh, kta), kta2);
                        // P_a/rho_a^2 + P_b/rho_b^2 + Pi_ab [+ R_ab f^4]
                        float sm = __builtin_fmaf(crk, fminf(u, 0.f), pa.w + pb.w);
                        if (TENS) sm = __builtin_fmaf(rab, f4, sm);
                        const float coef = sm * G;
                        s0 = __builtin_fmaf(coef, rx, s0);
                        s1 = __builtin_fmaf(coef, ry, s1);
                        s2 = __builtin_fmaf(coef, rz, s2);
                    }
                    if (STATS) hs += (uint32_t)A.ids[sSlot[off >> 4]] * 2654435761u;
                } else {
                    const float F = K.gs * G;
                    // Pair contribution to the loss, symmetric in (a, b):
                    //   (abar_a - abar_b) . T_ab + (Dbar_a + Dbar_b) S_ab,
                    //   T_ab = -m s F r_ab, s = P_a/rho_a^2 + P_b/rho_b^2 + Pi_ab [+ R_ab f^4],
                    //   S_ab = m (v_ab . r_ab) F;  its derivatives w.r.t. the gatherer a.
                    const float4 ab = lds_load4(sAb + off);
                    const float dax = aa.x - ab.x, day = aa.y - ab.y, daz = aa.z - ab.z;
                    const float Q = __builtin_fmaf(daz, rz, __builtin_fmaf(day, ry, dax * rx));
                    const float tb = __builtin_fmaf(vb.w, K.inv_rho0, 1.0f);
                    const float cr = __builtin_fmaf(tb, tb - ta, ta2);
                    const float invden = __builtin_amdgcn_rcpf(r2 + K.eta2);
                    const float mu = K.h * vdr * invden;
                    const float mneg = fminf(mu, 0.f);
                    // d/drho_a of s: d(P/rho^2)/drho + dPi/drho_a
                    const float dpi_dra = K.kpi * K.inv_rho0 * __builtin_fmaf(2.f, ta, -tb) * mneg;
                    // (+ the tensile term's dR_a/drho_a f^4)
                    float drs = dpa + dpi_dra;
                    if (TENS) drs = __builtin_fmaf(eda, f4, drs);
                    s3 = __builtin_fmaf(-F * Q, drs, s3);
                    if (FLUID) {
                        // (dF/dr) / r; 0 for the self pair
                        float Fr;
                        if (KER == SPH_WENDLAND5) {
                            Fr = K.kfr * wq * wq * ir;
                        } else {
                            Fr = qq < 1.f ? K.kcr_in * ir
                                          : K.kcr_out * __builtin_fmaf(-qq, qq, 4.f) * (ir * ir * ir);
                        }
                        Fr = r2 > 0.f ? Fr : 0.f;
                        // continuity
                        const float sD = aa.w + ab.w;
                        const float c1 = sD * F, c2 = sD * vdr * Fr;
                        // momentum
                        const float pi = K.kpi * cr * mneg;
                        float sm = pa.w + pb.w + pi;
                        if (TENS) sm = __builtin_fmaf(rab, f4, sm);
                        const float dpi_dmu = mu < 0.f ? K.kpi * cr : 0.f;
                        const float e1 = F * Q * dpi_dmu;
                        const float e1i = e1 * invden;
                        const float e1h = e1i * K.h;
                        float e2 = __builtin_fmaf(-2.f * e1i, mu, sm * Q * Fr);
                        // tensile: d(R_ab f^4)/dx_a = R_ab 4 f^3 (F / W(dp)) r_ab
                        if (TENS) e2 = __builtin_fmaf(4.f * rab * f3 * K.inv_wdp, F * F * Q, e2);
                        const float e3 = sm * F;
                        // c1 v + c2 r - (e1h v + e2 r + e3 da), grouped by vector
                        const float g = c1 - e1h, hr = c2 - e2;
                        s0 = __builtin_fmaf(g, vx, __builtin_fmaf(hr, rx, __builtin_fmaf(-e3, dax, s0)));
                        s1 = __builtin_fmaf(g, vy, __builtin_fmaf(hr, ry, __builtin_fmaf(-e3, day, s1)));
                        s2 = __builtin_fmaf(g, vz, __builtin_fmaf(hr, rz, __builtin_fmaf(-e3, daz, s2)));
                        s4 = __builtin_fmaf(g, rx, s4);
                        s5 = __builtin_fmaf(g, ry, s5);
                        s6 = __builtin_fmaf(g, rz, s6);
                        // alpha: own target term abar_a . dA_a/dalpha, dPi/dalpha = Pi/alpha
                        const float qa = __builtin_fmaf(aa.z, rz, __builtin_fmaf(aa.y, ry, aa.x * rx));
                        s7 = __builtin_fmaf(-F * qa, K.kpa * cr * mneg, s7);
                    }
                }
            };

            // test one chunk of 64 staged candidates; survivors go to the ring as
            // byte offsets of their staged entries, and full batches of 64 are
            // evaluated after every two chunks (drain below; checking after
            // every chunk cost 1.6% of the fused stage in scalar instructions
            // and branches).  The ring holds kRing entries in 512 bytes, so
            // slot k sits at rbase | (2 k mod 512).
            auto chunk = [&](float rx, float ry, float rz, int32_t cb0) {
                const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
                const bool pass = r2 < K.rc2;
                const unsigned long long m = ballot(pass);
                // rank in every lane (no exec-mask switch); rejected lanes write
                // their own trash slot
                int rk = (int)lane_rank(m);
                asm volatile("" : "+v"(rk));
                const uint32_t w = ((uint32_t)(2 * (wp + rk)) & 0x1FEu) | rbase;
                *(lds_u16 *)(uintptr_t)(pass ? w : taddr) = (uint16_t)(lane16 + ((uint32_t)cb0 << 4));
                wp += __popcll(m);
            };
            // evaluate every full batch of 64 in the ring (at most two after
            // two chunks: fewer than 64 + 128 entries pending)
            auto drain = [&]() {
                while (wp - rp >= kWave) {
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    pair(*(const lds_u16 *)(uintptr_t)raddr);
                    raddr = ((raddr + 2u * kWave) & 0x1FFu) | rbase;
                    rp += kWave;
                }
            };
            // the window of x-bins within 2h of the target (conservative: bins
            // are monotone in x), rounded up to whole chunks of 64; entries past
            // the window are real candidates or padding and are tested as usual.
            // Two chunks per iteration, both loaded up front: the second read
            // ends before sBin[kBins] + 2 * kWave, inside the padding (four
            // for boundary targets, whose reads end before sBin[kBins] + kPad).
            // (wave-uniform: every lane holds the same target)
            // both bin starts are read before either is used (one LDS round trip)
            const int32_t sb0 = sBin[xbin(pa.x - K.xwin)];
            const int32_t sb1 = sBin[xbin(pa.x + K.xwin) + 1];
            const int32_t w0 = __builtin_amdgcn_readfirstlane(sb0);
            const int32_t w1 = __builtin_amdgcn_readfirstlane(sb1);
            next_l = slot_of(a + kWaves);  // returns during the scan below
            const int32_t wend = w0 + ((w1 - w0 + kWave - 1) & ~(kWave - 1));
            if (!FLUID && !POS) {
                // boundary targets (few per wave, latency-bound): four chunks
                // per iteration, the last two loaded only inside the window
                // (their reads end inside the padding)
                for (int32_t cb0 = w0; cb0 < wend; cb0 += 4 * kWave) {
                    const float4 c0 = sP[cb0 + lane];
                    const float4 c1 = sP[cb0 + kWave + lane];
                    const bool more = cb0 + 2 * kWave < wend;
                    float4 c2 = c0, c3 = c0;
                    if (more) {
                        c2 = sP[cb0 + 2 * kWave + lane];
                        c3 = sP[cb0 + 3 * kWave + lane];
                    }
                    chunk(pa.x - c0.x, pa.y - c0.y, pa.z - c0.z, cb0);
                    if (cb0 + kWave < wend)
                        chunk(pa.x - c1.x, pa.y - c1.y, pa.z - c1.z, cb0 + kWave);
                    drain();
                    if (more) {
                        chunk(pa.x - c2.x, pa.y - c2.y, pa.z - c2.z, cb0 + 2 * kWave);
                        if (cb0 + 3 * kWave < wend)
                            chunk(pa.x - c3.x, pa.y - c3.y, pa.z - c3.z, cb0 + 3 * kWave);
                        drain();
                    }
                }
            } else
            for (int32_t cb0 = w0; cb0 < wend; cb0 += 2 * kWave) {
                if (POS) {
                    const int i0 = cb0 + lane, i1 = cb0 + kWave + lane;
                    const double x0 = S.sDx[i0], y0 = S.sDy[i0], z0 = S.sDz[i0];
                    const double x1 = S.sDx[i1], y1 = S.sDy[i1], z1 = S.sDz[i1];
                    chunk((float)(pax - x0), (float)(pay - y0), (float)(paz - z0), cb0);
                    if (cb0 + kWave < wend)
                        chunk((float)(pax - x1), (float)(pay - y1), (float)(paz - z1), cb0 + kWave);
                } else {
                    const float4 c0 = sP[cb0 + lane];
                    const float4 c1 = sP[cb0 + kWave + lane];
                    chunk(pa.x - c0.x, pa.y - c0.y, pa.z - c0.z, cb0);
                    if (cb0 + kWave < wend)
                        chunk(pa.x - c1.x, pa.y - c1.y, pa.z - c1.z, cb0 + kWave);
                }
                drain();
            }
            if (wp > rp) {
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (lane < wp - rp) pair(*(const lds_u16 *)(uintptr_t)raddr);
            }
            const int cnt = wp - (self_here ? 1 : 0);
            pairs_acc += (unsigned long long)cnt;

            // ---- reduce over the wave, write (first tile) or accumulate
            if (!BWD && FLUID) {
                // lane l < 4 ends with component l: a.x, a.y, a.z (in units of
                // -m gs), drho/dt (in units of m gs)
                const float t = wave_sum4(s0, s1, s2, s3, lane, xa);
                const float tvm = wave_max_nonneg(vmf, xa) * K.h;
                unsigned ths = 0;
                if (STATS) {
                    ths = wave_sum_u(hs);
                    if (self_here) ths -= (uint32_t)A.ids[a] * 2654435761u;
                }
                // the scale and gravity of lane l's component are selected on
                // lane bits, outside the store's branch: written as a chain of
                // lane tests they became a nest of divergent branches per target
                // (2.7% of the fused stage at 1.65M particles)
                const float scale = lane < 3 ? -K.mgs : K.mgs;
                const float g01 = (lane & 1) ? K.gy : K.gx;
                const float g23 = (lane & 1) ? 0.f : K.gz;
                const float g = (lane & 2) ? g23 : g01;
                if (lane < 4) {
                    float *o = (float *)A.ace + 4 * (int64_t)a + lane;
                    *o = __builtin_fmaf(scale, t, tb == 0 ? g : *o);
                }
                if (lane == 0) {
                    A.visc[a] = tb == 0 ? tvm : fmaxf(A.visc[a], tvm);
                    if (STATS) {
                        if (tb == 0) {
                            A.stats[2 * a] = cnt;
                            A.stats[2 * a + 1] = (int32_t)ths;
                        } else {
                            A.stats[2 * a] += cnt;
                            A.stats[2 * a + 1] = (int32_t)((uint32_t)A.stats[2 * a + 1] + ths);
                        }
                    }
                }
            } else if (!BWD) {
                const float tsd = wave_sum(s3);
                unsigned ths = 0;
                if (STATS) ths = wave_sum_u(hs);
                if (lane == 0) {
                    const float d = K.mgs * tsd;
                    if (tb == 0) {
                        A.ace[a] = make_float4(0.f, 0.f, 0.f, d);
                        A.visc[a] = 0.f;
                        if (STATS) { A.stats[2 * a] = cnt; A.stats[2 * a + 1] = (int32_t)ths; }
                    } else {
                        A.ace[a].w += d;
                        if (STATS) {
                            A.stats[2 * a] += cnt;
                            A.stats[2 * a + 1] = (int32_t)((uint32_t)A.stats[2 * a + 1] + ths);
                        }
                    }
                }
            } else if (FLUID) {
                // lane l < 8 ends with s_l: xbar.xyz, rhobar, vbar.xyz, alphabar
                const float t = wave_sum8(s0, s1, s2, s3, s4, s5, s6, s7, lane, xa);
                // lane l < 8 adds s_l to its slot (xbar components, rhobar, vbar
                // components, the per-slot alpha adjoint, which the first tile
                // overwrites), slot chosen without branches (-5% on the pair VJP
                // at 1.65M particles against a branch per slot kind)
                float *const base =
                    lane < 3 ? (float *)A.xbar : (lane < 7 ? (float *)A.vbar : A.alpha_part);
                const int comp = lane < 3 ? lane : (lane == 3 ? 3 : lane - 4);
                const int64_t idx = lane < 7 ? 4 * (int64_t)a + comp : (int64_t)a;
                if (lane < 8) {
                    float *o = base + idx;
                    const float old = *o;
                    *o = __builtin_fmaf(K.mass, t, lane == 7 && tb == 0 ? 0.f : old);
                }
            } else {
                const float tr = wave_sum(s3);
                if (lane == 0) A.vbar[a].w += K.mass * tr;
            }
        }
        __syncthreads();
    }
}

// Four waves per SIMD (two workgroups per CU) is what the LDS allows, and the
// kernel needs them to hide its LDS and memory latency; at 129+ VGPRs only
// three fit (about 1.6x the time).  Every kind without per-pair statistics is
// held to 128 VGPRs (none spills); with statistics the LDS allows two waves
// per SIMD only.
template <int KIND, bool STATS, int KER, bool TENS, int POS>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(!STATS ? 4 : 1, 4))) void k_interact(
    PairConsts K, PairArgs A)
{
    using T = KindTraits<KIND, POS>;
    __shared__ PairLds<T::tile, T::bwd, STATS, POS> S;
    LaneCtx C;
    C.lane = threadIdx.x & (kWave - 1);
    C.wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint32_t rbase = lds_addr(&S.sRing[C.wave][0]);
    C.rfirst = rbase | (2u * C.lane);
    asm volatile("" : "+v"(rbase));  // per-lane copy: one and-or per ring slot
    C.rbase = rbase;
    C.xa = xor_addr(C.lane);
    uint32_t lane16 = (uint32_t)C.lane << 4;  // byte offset of this lane's entry in a chunk
    asm volatile("" : "+v"(lane16));
    C.lane16 = lane16;
    C.taddr = lds_addr(&S.sTrash[C.wave][C.lane]);
    C.sPb = lds_addr(S.sP);
    C.sVb = lds_addr(S.sV);
    C.sAb = lds_addr(S.sA);
    C.sTb = lds_addr(S.sTgt);

    // First list: fluid cells are list[info[0] .. info[0] + info[1]); boundary
    // cells with fluid in reach are active[0 .. nactive).  Counts are clamped
    // so that inconsistent inputs can never index outside [0, n).
    int32_t ibase, nitems;
    if (T::fluid) {
        ibase = min(max(A.counts[0], 0), K.n);
        nitems = min(max(A.counts[1], 0), K.n - ibase);
    } else {
        ibase = 0;
        nitems = min(max(A.counts[0], 0), K.n);
    }
    unsigned long long p1 = 0, p2 = 0;  // wave-uniform pair counts of the two lists
    // XCD-aware dynamic schedule of the first list, in three phases:
    //  * home: its first (64 - kPool64)/64 is cut into kXcds contiguous chunks
    //    with one counter each, and workgroup b (dealt to XCD b mod kXcds)
    //    draws from chunk b mod kXcds, so cells with common stencil neighbours
    //    run on the XCD whose L2 holds them;
    //  * pool: the rest of the list behind one counter of all workgroups, so
    //    the XCDs whose chunk ends early take more of it;
    //  * steal: then from the chunks that still hold more than four items per
    //    workgroup of their own (flag word: bit x is set by the draw that
    //    leaves that many in chunk x), which only happens when the chunks'
    //    work differs widely (clustered layouts).
    // No workgroup walks through exhausted chunks with atomics: at the end of
    // a launch every workgroup would do so at once.  Fused launches interleave
    // the second list (one counter): after every `mix` items of the first
    // list a workgroup takes one of the second, so its short, latency-bound
    // items overlap with the compute-bound ones instead of forming the tail;
    // once the first list is exhausted the second is drained.  The counters
    // only grow, so every workgroup leaves once both lists are exhausted: each
    // chunk is drained by the workgroups of its own XCD at least.
    const int32_t n2 = T::fused ? min(max(A.counts2[0], 0), K.n) : 0;
    const int32_t mix = nitems / (n2 + 1);
    const int home = blockIdx.x % kXcds;
    const int32_t plen = (int32_t)(((int64_t)nitems * kPool64) / 64);
    const int32_t m = nitems - plen;  // chunks cover [0, m), the pool [m, nitems)
    const int32_t lo = (int32_t)(((int64_t)m * home) / kXcds);
    const int32_t hi = (int32_t)(((int64_t)m * (home + 1)) / kXcds);
    int32_t *const flags = A.queue + kQFlags * kCounterStride;
    const int32_t near = max(4 * (int32_t)gridDim.x / kXcds, 1);
    // thread 0 only: schedule state
    bool home_done = false, pool_done = false, ex_read = false;
    int steal = 1;       // next chunk to steal from: home + steal
    unsigned ex = 0;     // chunks known to hold at most `near` unclaimed items
    int32_t since = 0;   // first-list items since the last second-list item
    bool done2 = !T::fused;
    for (;;) {
        if (threadIdx.x == 0) {
            int32_t it = -1;
            int kind = 0;
            if (!done2 && since >= mix) {
                const int32_t k = atomicAdd(A.queue2, 1);
                if (k < n2) {
                    it = k;
                    kind = 1;
                    since = 0;
                } else {
                    done2 = true;
                }
            }
            if (it < 0 && !home_done) {
                const int32_t k = atomicAdd(A.queue + home * kCounterStride, 1);
                if (k < hi - lo) {
                    it = lo + k;
                    ++since;
                    if (k == max(hi - lo - 1 - near, 0)) atomicOr(flags, 1 << home);
                } else {
                    home_done = true;
                }
            }
            if (it < 0 && !pool_done) {
                const int32_t k = atomicAdd(A.queue + kQPool * kCounterStride, 1);
                if (k < plen) {
                    it = m + k;
                    ++since;
                } else {
                    pool_done = true;
                }
            }
            if (it < 0 && steal < kXcds) {
                if (!ex_read) {
                    ex_read = true;
                    ex = (unsigned)__hip_atomic_load(flags, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                }
                while (steal < kXcds) {
                    const int x = (home + steal) % kXcds;
                    if (!((ex >> x) & 1u)) {
                        const int32_t xlo = (int32_t)(((int64_t)m * x) / kXcds);
                        const int32_t xhi = (int32_t)(((int64_t)m * (x + 1)) / kXcds);
                        const unsigned f = (unsigned)__hip_atomic_load(
                            flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const int32_t k = atomicAdd(A.queue + x * kCounterStride, 1);
                        ex |= f;
                        if (k < xhi - xlo) {
                            it = xlo + k;
                            ++since;
                            if (k == max(xhi - xlo - 1 - near, 0)) atomicOr(flags, 1 << x);
                            break;
                        }
                        ex |= 1u << x;
                    }
                    ++steal;
                }
            }
            if (it < 0 && !done2) {
                const int32_t k = atomicAdd(A.queue2, 1);
                if (k < n2) {
                    it = k;
                    kind = 1;
                } else {
                    done2 = true;
                }
            }
            S.sItem = it;
            S.sKind = kind;
        }
        __syncthreads();
        const int32_t item = __builtin_amdgcn_readfirstlane(S.sItem);
        const int kind = __builtin_amdgcn_readfirstlane(S.sKind);
        if (item < 0) break;
        if (!T::fused || kind == 0) {
            const int32_t key = __builtin_amdgcn_readfirstlane(
                min(max(A.items[ibase + item], 0), 2 * K.ncell - 1));
            pair_item<T::first, STATS, KER, TENS, POS>(K, A, S, C, key, p1);
        } else {
            const int32_t key =
                __builtin_amdgcn_readfirstlane(min(max(A.items2[item], 0), 2 * K.ncell - 1));
            pair_item<T::second, STATS, KER, TENS, POS>(K, A, S, C, key, p2);
        }
    }
    if (A.npairs) {
        // one atomic per workgroup and list: the waves' counts are summed in
        // LDS (the rings are free once the item loop has ended); one per wave
        // on the same address lengthened the fused launch by 5%
        unsigned long long *sp = (unsigned long long *)&S.sRing[0][0];
        if (C.lane == 0) {
            sp[C.wave] = p1;
            sp[kWaves + C.wave] = p2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t1 = 0, t2 = 0;
            for (int w = 0; w < kWaves; ++w) {
                t1 += sp[w];
                t2 += sp[kWaves + w];
            }
            if (t1) atomicAdd(A.npairs + (T::fluid ? 0 : 1), t1);
            if (t2) atomicAdd(A.npairs + 1, t2);
        }
    }
}

// Boundary cells: those with fluid particles in their stencil go to the work
// list of the B-F pass.  Forward only (ace != NULL): every boundary slot and
// every excluded slot first gets zero outputs (coalesced, one thread per
// slot); the boundary items of the pair kernel, which run after this kernel
// on the same stream, overwrite the targets of the active cells.
template <int NSUB>
__device__ inline int32_t fluid_in_reach(const PairConsts &K, const int32_t *__restrict__ start,
                                         int32_t key)
{
    const int32_t cx = key % K.nc0, cy = (key / K.nc0) % K.nc1, cz = key / (K.nc0 * K.nc1);
    const int32_t x0 = max(cx - NSUB, 0), x1 = min(cx + NSUB, K.nc0 - 1);
    int32_t total = 0;
#pragma unroll
    for (int dz = -NSUB; dz <= NSUB; ++dz)
#pragma unroll
        for (int dy = -NSUB; dy <= NSUB; ++dy) {
            const int32_t y = cy + dy, z = cz + dz;
            const bool ok = y >= 0 && y < K.nc1 && z >= 0 && z < K.nc2;
            // an out-of-grid run reads start[0] twice (in bounds, difference 0)
            const int32_t k0 = ok ? K.ncell + x0 + K.nc0 * (y + K.nc1 * z) : 0;
            const int32_t len = ok ? x1 - x0 + 1 : 0;
            total += start[k0 + len] - start[k0];
        }
    return total;
}

__global__ void k_bound_filter(PairConsts K, const int32_t *__restrict__ start,
                               const int32_t *__restrict__ list, const int32_t *__restrict__ info,
                               int32_t *__restrict__ active, int32_t *__restrict__ nactive,
                               float4 *__restrict__ ace, float *__restrict__ visc,
                               int32_t *__restrict__ stats)
{
    const int32_t stride = gridDim.x * blockDim.x;
    const int32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (ace) {
        // slots [0, start[ncell]) hold the boundary particles inside the grid,
        // the last info[2] slots the excluded particles
        const int32_t nbs = min(max(start[K.ncell], 0), K.n);
        const int32_t nex = min(max(info[2], 0), K.n - nbs);
        for (int32_t i = gid; i < nbs + nex; i += stride) {
            const int32_t a = i < nbs ? i : K.n - nex + (i - nbs);
            ace[a] = make_float4(0.f, 0.f, 0.f, 0.f);
            visc[a] = 0.f;
            if (stats) {
                stats[2 * a] = 0;
                stats[2 * a + 1] = 0;
            }
        }
    }
    // one atomic per wavefront: the first live lane reserves the wave's slots
    const int32_t nbc = min(max(info[0], 0), K.n);
    const int lane = lane_id();
    for (int32_t i = gid; i < nbc; i += stride) {
        const int32_t key = min(max(list[i], 0), K.ncell - 1);
        const int32_t total = K.nsub == 1 ? fluid_in_reach<1>(K, start, key)
                                          : fluid_in_reach<2>(K, start, key);
        const unsigned long long live = ballot(true);
        const unsigned long long m = ballot(total > 0);
        if (m) {
            const int leader = __ffsll((long long)live) - 1;
            int32_t base = 0;
            if (lane == leader) base = atomicAdd(nactive, __popcll(m));
            base = __shfl(base, leader, kWave);
            if (total > 0) active[base + (int32_t)lane_rank(m)] = key;
        }
    }
}

// clears counter slots [0, count) (count <= 64), kCounterStride ints apart
__global__ void k_zero_counters(int32_t *q, int count)
{
    if ((int)threadIdx.x < count) q[threadIdx.x * kCounterStride] = 0;
}


static PairConsts pair_consts(const sph_grid *g, const sph_params *p, int32_t n)
{
    PairConsts K;
    const double pi = 3.14159265358979323846;
    const double h = p->h;
    const double ad = 21.0 / (16.0 * pi * h * h * h);
    K.cellf = (float)g->cell;
    K.rc2 = (float)(4.0 * h * h);
    K.h = (float)h;
    K.inv_h = (float)(1.0 / h);
    K.kf = (float)(-5.0 * ad / (h * h));
    K.eta2 = (float)p->eta2;
    K.kpi = (float)(-p->alpha * p->c0 / p->rho0);
    K.kpa = (float)(-p->c0 / p->rho0);
    K.kfr = (float)(1.5 * 5.0 * ad / (h * h * h));
    const double ac = 1.0 / (pi * h * h * h);
    K.kc_in = (float)(ac / (h * h));
    K.kc_out = (float)(-0.75 * ac / h);
    K.kcr_in = (float)(2.25 * ac / (h * h * h));
    K.kcr_out = (float)(0.75 * ac / h);
    K.kernel = p->kernel;
    K.kh = (float)(-p->alpha * p->c0 / p->rho0 * h);
    if (p->kernel == SPH_CUBIC_SPLINE) {
        K.gs = K.kc_in;
        K.kco = (float)(-0.75 * h);  // kc_out / kc_in
    } else {
        K.gs = K.kf;
        K.kco = 0.f;
    }
    K.mgs = (float)(p->mass * (double)K.gs);
    // tensile correction: kernel shape Wn = W / aD at the particle spacing
    K.tensile = p->tensile_dp > 0.0 ? 1 : 0;
    K.inv_wndp = 0.f;
    K.inv_wdp = 0.f;
    if (K.tensile) {
        const double q = p->tensile_dp / h;
        double wn, adk;
        if (p->kernel == SPH_CUBIC_SPLINE) {
            wn = q < 1.0 ? 1.0 - 1.5 * q * q + 0.75 * q * q * q : 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
            adk = ac;
        } else {
            const double t = 1.0 - 0.5 * q;
            wn = t * t * t * t * (2.0 * q + 1.0);
            adk = ad;
        }
        K.inv_wndp = (float)(1.0 / wn);
        K.inv_wdp = (float)(1.0 / (adk * wn));
    }
    K.c0 = (float)p->c0;
    K.rho0 = (float)p->rho0;
    K.inv_rho0 = (float)(1.0 / p->rho0);
    K.gx = (float)p->g[0];
    K.gy = (float)p->g[1];
    K.gz = (float)p->g[2];
    K.mass = (float)p->mass;
    K.nsub = g->nsub;
    K.nc0 = g->nc[0];
    K.nc1 = g->nc[1];
    K.nc2 = g->nc[2];
    K.ncell = (int32_t)ncell_of(g);
    K.n = n;
    // x-bins over the staged extent [-(n + 1/2) cell, (n + 1/2) cell] of the target frame
    K.xlo = (float)(-(g->nsub + 0.5) * g->cell);
    K.xscale = (float)(kBins / ((2 * g->nsub + 1) * g->cell));
    K.xwin = (float)(2.0 * h * (1.0 + 1.0 / 1024.0));
    K.half = (float)(0.5 * g->cell * (1.0 + ldexp(1.0, -20)));
    K.cull2 = (float)(4.0 * h * h * (1.0 + 1.0 / 1024.0));
    K.pos_policy = p->pos_policy;
    for (int d = 0; d < 3; ++d) K.org64[d] = g->origin[d];
    K.cell64 = g->cell;
    return K;
}

template <int KIND, bool STATS, int KER, bool TENS, int POS = 0>
static hipError_t launch_one(const PairConsts &K, const PairArgs &A, hipStream_t s)
{
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_interact<KIND, STATS, KER, TENS, POS>,
                                                     kThreads, 0);
    if (e != hipSuccess) return e;
    if (cus <= 0) cus = 1;
    if (occ <= 0) occ = 1;
    // every chunk of the work queue needs a workgroup of its own XCD
    const int grid = cus * occ < kXcds ? kXcds : cus * occ;
    k_interact<KIND, STATS, KER, TENS, POS><<<grid, kThreads, 0, s>>>(K, A);
    return hipGetLastError();
}

// instantiation for the kernel shape; per-pair statistics only in the forward
template <int KIND>
static hipError_t launch_kind(const PairConsts &K, const PairArgs &A, bool stats, hipStream_t s)
{
    constexpr bool fwd = KIND == kFwdFluid || KIND == kFwdBound || KIND == kFwdAll;
    const bool st = fwd && stats;
    // FP64 absolute positions (a measurement variant of the default kernel
    // shape; the entry points refuse it with statistics, another kernel shape,
    // the tensile correction or the adjoint)
    if constexpr (fwd) {
        if (K.pos_policy == SPH_POS_ABS64) return launch_one<KIND, false, SPH_WENDLAND5, false, 1>(K, A, s);
    }
    if (K.kernel == SPH_CUBIC_SPLINE) {
        if (K.tensile)
            return st ? launch_one<KIND, fwd, SPH_CUBIC_SPLINE, true>(K, A, s)
                      : launch_one<KIND, false, SPH_CUBIC_SPLINE, true>(K, A, s);
        return st ? launch_one<KIND, fwd, SPH_CUBIC_SPLINE, false>(K, A, s)
                  : launch_one<KIND, false, SPH_CUBIC_SPLINE, false>(K, A, s);
    }
    if (K.tensile)
        return st ? launch_one<KIND, fwd, SPH_WENDLAND5, true>(K, A, s)
                  : launch_one<KIND, false, SPH_WENDLAND5, true>(K, A, s);
    return st ? launch_one<KIND, fwd, SPH_WENDLAND5, false>(K, A, s)
              : launch_one<KIND, false, SPH_WENDLAND5, false>(K, A, s);
}

static PairArgs base_args(const sph_state *st, const sph_cells *cells)
{
    PairArgs A;
    A.start = cells->start;
    A.items = cells->list;
    A.counts = cells->info;
    A.ranges = (const int2 *)cells->ranges;
    A.cell = st->cell;
    A.pos = (const float4 *)st->pos;
    A.velrho = (const float4 *)st->velrho;
    A.pos64 = st->pos64;
    A.ids = st->id;
    A.ace = nullptr;
    A.visc = nullptr;
    A.xbar = nullptr;
    A.vbar = nullptr;
    A.alpha_part = nullptr;
    A.queue = nullptr;
    A.items2 = nullptr;
    A.counts2 = nullptr;
    A.queue2 = nullptr;
    A.npairs = nullptr;
    A.stats = nullptr;
    return A;
}

hipError_t launch_interact(const sph_grid *g, const sph_params *p, const sph_state *st,
                           const sph_cells *cells, unsigned parts, float *ace, float *visc,
                           unsigned long long *npairs, int32_t *nbr_stats, const Workspace &w,
                           hipStream_t s)
{
    if (st->n == 0) return hipSuccess;
    const PairConsts K = pair_consts(g, p, st->n);
    PairArgs A = base_args(st, cells);
    A.ace = (float4 *)ace;
    A.visc = visc;
    A.npairs = npairs;
    A.stats = nbr_stats;
    // counter slots: [0, 10) the first list's queue (chunks, pool, flags),
    // [16, 26) the queue of a separate boundary launch or [16] the boundary
    // counter of the fused launch, [32] active boundary cells
    const bool stats = nbr_stats != nullptr;
    int32_t *const q = w.counters;
    constexpr int S = kCounterStride;
    k_zero_counters<<<1, 64, 0, s>>>(q, 33);
    if (parts & SPH_PI_BOUNDARY)
        k_bound_filter<<<256, 256, 0, s>>>(K, cells->start, cells->list, cells->info, w.active,
                                           q + 32 * S, (float4 *)ace, visc, nbr_stats);
    if (parts == SPH_PI_ALL) {
        A.queue = q;
        A.items2 = w.active;
        A.counts2 = q + 32 * S;
        A.queue2 = q + 16 * S;
        return launch_kind<kFwdAll>(K, A, stats, s);
    }
    hipError_t e = hipSuccess;
    if (parts & SPH_PI_FLUID) {
        A.queue = q;
        e = launch_kind<kFwdFluid>(K, A, stats, s);
        if (e != hipSuccess) return e;
    }
    if (parts & SPH_PI_BOUNDARY) {
        A.items = w.active;
        A.counts = q + 32 * S;
        A.queue = q + 16 * S;
        e = launch_kind<kFwdBound>(K, A, stats, s);
    }
    return e;
}

// Deterministic FP64 sum of the per-slot alpha adjoints of the fluid slots
// [nb, n - excluded): fixed-order block partials, then one block.
__global__ __launch_bounds__(kReduceThreads) void k_alpha_partial(int32_t n, int32_t nb,
                                                                  const int32_t *__restrict__ info,
                                                                  const float *__restrict__ part,
                                                                  double *__restrict__ out)
{
    __shared__ double sh[kReduceThreads];
    const int32_t hi = n - min(max(info[2], 0), n);
    double acc = 0.0;
    for (int32_t i = nb + blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += gridDim.x * blockDim.x)
        acc += (double)part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kReduceThreads) void k_alpha_final(int nblk, const double *__restrict__ in,
                                                                double *__restrict__ alpha_bar)
{
    __shared__ double sh[kReduceThreads];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kReduceThreads) acc += in[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) alpha_bar[0] += sh[0];
}

hipError_t launch_interact_backward(const sph_grid *g, const sph_params *p, const sph_state *st,
                                    const sph_cells *cells, const float *ace_bar, float *pos_bar,
                                    float *velrho_bar, double *alpha_bar, const Workspace &w,
                                    hipStream_t s)
{
    if (st->n == 0) return hipSuccess;
    const PairConsts K = pair_consts(g, p, st->n);
    PairArgs A = base_args(st, cells);
    A.ace = (float4 *)ace_bar;
    A.xbar = (float4 *)pos_bar;
    A.vbar = (float4 *)velrho_bar;
    A.alpha_part = w.alpha_part;
    // counter slots: [40, 50) the fluid list's queue, [56] boundary counter,
    // [60] active cells
    int32_t *const q = w.counters;
    constexpr int S = kCounterStride;
    k_zero_counters<<<1, 64, 0, s>>>(q + 40 * S, 21);
    // boundary gatherers: only cells with fluid in reach have non-zero terms
    k_bound_filter<<<256, 256, 0, s>>>(K, cells->start, cells->list, cells->info, w.active,
                                       q + 60 * S, nullptr, nullptr, nullptr);
    A.queue = q + 40 * S;
    A.items2 = w.active;
    A.counts2 = q + 60 * S;
    A.queue2 = q + 56 * S;
    hipError_t e = launch_kind<kBwdAll>(K, A, false, s);
    if (e != hipSuccess) return e;
    int nblk = (int)(((int64_t)st->n + kReduceThreads - 1) / kReduceThreads);
    if (nblk > kReduceBlocksMax) nblk = kReduceBlocksMax;
    if (nblk < 1) nblk = 1;
    k_alpha_partial<<<nblk, kReduceThreads, 0, s>>>(st->n, st->nb, cells->info, w.alpha_part,
                                                    w.reduce);
    k_alpha_final<<<1, kReduceThreads, 0, s>>>(nblk, w.reduce, alpha_bar);
    return hipGetLastError();
}

}  // namespace sph
