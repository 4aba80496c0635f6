// interact.hip -- particle-interaction stage (Section 2 "PI"): fluid targets
// (F-F and F-B fused in one kernel, Section 4.5) and boundary targets (B-F).
//
// Work decomposition (gfx950, wave64):
//   * one workgroup per non-empty target cell, taken from a device work queue
//     (dynamic scheduling, like the OpenMP dynamic scheduler of Section 3.4);
//   * the (2n+1)^2 X-runs of the stencil (Section 4.4: three consecutive
//     cells along X are one contiguous range of the sorted arrays) are staged
//     into LDS in the frame of the target cell: each candidate's offset gets
//     (k_b - k_a) * cell added once, in FP32;
//   * one wavefront per target: 64 candidates per step are tested for
//     r^2 < (2h)^2, survivors are compacted with a ballot into a per-wave ring
//     in LDS, and every full batch of 64 survivors is evaluated with all lanes
//     busy.  This removes the divergence of a thread-per-target loop (the
//     "code divergence" problem of Section 4) without any neighbour list in
//     HBM;
//   * per-lane partial sums are reduced across the wave once per target and
//     written once (Section 4.5: accumulate in registers, write at the end).
#include "sph_internal.h"

namespace sph {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / kWave;
constexpr int kTile = 2048;          // candidates staged per pass
constexpr int kRing = 128;           // per-wave ring of compacted candidates
constexpr int kMaxRuns = 2 * 25;     // types x (2n+1)^2, n <= 2
constexpr int kMaxRunCells = 5;      // 2n+1

struct RunTable {
    int32_t nruns;
    int32_t total;                      // candidates over all runs
    int32_t vstart[kMaxRuns + 1];       // prefix of run lengths
    int32_t s[kMaxRuns][kMaxRunCells + 1];  // slot starts of the run's cells, last = end
    int32_t ncx[kMaxRuns];
    int32_t dx0[kMaxRuns];              // x0 - cx
    float sy[kMaxRuns], sz[kMaxRuns];   // dy * cell, dz * cell
    int32_t self_run;                   // run holding the target cell's own fluid particles
};

__device__ inline float wave_sum(float v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

__device__ inline unsigned wave_sum_u(unsigned v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Build the run table of target cell c (coordinates cx, cy, cz).  FLUID:
// candidates are boundary and fluid particles; otherwise fluid only.
template <bool FLUID>
__device__ void build_runs(const PairConsts &K, const int32_t *__restrict__ start, int32_t cx,
                           int32_t cy, int32_t cz, RunTable &R)
{
    const int n = K.nsub;
    const int side = 2 * n + 1;
    const int ntypes = FLUID ? 2 : 1;
    const int nr = ntypes * side * side;
    const int32_t x0 = max(cx - n, 0);
    const int32_t x1 = min(cx + n, K.nc0 - 1);
    const int ncx = x1 - x0 + 1;
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
        const int type = FLUID ? r / (side * side) : 1;  // 0 boundary, 1 fluid
        const int rr = r % (side * side);
        const int dy = rr % side - n, dz = rr / side - n;
        const int32_t y = cy + dy, z = cz + dz;
        const bool ok = y >= 0 && y < K.nc1 && z >= 0 && z < K.nc2;
        int32_t key0 = 0;
        if (ok) key0 = (type ? K.ncell : 0) + x0 + K.nc0 * (y + K.nc1 * z);
        for (int i = 0; i <= kMaxRunCells; ++i) {
            int32_t v = 0;
            if (ok) v = start[key0 + min(i, ncx)];
            R.s[r][i] = v;
        }
        R.ncx[r] = ok ? ncx : 0;
        R.dx0[r] = x0 - cx;
        R.sy[r] = (float)dy * K.cellf;
        R.sz[r] = (float)dz * K.cellf;
        if (type == 1 && dy == 0 && dz == 0) R.self_run = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int r = 0; r < nr; ++r) {
            R.vstart[r] = acc;
            acc += R.ncx[r] ? R.s[r][R.ncx[r]] - R.s[r][0] : 0;
        }
        R.vstart[nr] = acc;
        R.total = acc;
        R.nruns = nr;
    }
    __syncthreads();
}

template <bool FLUID, bool STATS>
__global__ __launch_bounds__(kThreads) void k_interact(
    PairConsts K, const int32_t *__restrict__ start, const int32_t *__restrict__ list,
    const int32_t *__restrict__ info, const float4 *__restrict__ pos,
    const float4 *__restrict__ velrho, const int32_t *__restrict__ ids, float4 *__restrict__ ace,
    float *__restrict__ visc, int32_t *__restrict__ queue, unsigned long long *__restrict__ npairs,
    int32_t *__restrict__ stats)
{
    __shared__ float4 sP[kTile];                  // (offset in target frame, P/rho^2)
    __shared__ float4 sV[kTile];                  // (v, rho - rho0)
    __shared__ uint16_t sRing[kWaves][kRing];
    __shared__ int32_t sSlot[STATS ? kTile : 1];  // candidate slot (diagnostics only)
    __shared__ RunTable R;
    __shared__ int32_t sItem;

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    // counts come from sph_build_cells on the same stream; clamp them so that
    // inconsistent inputs can never index outside [0, n)
    const int32_t nbc = min(max(info[0], 0), K.n);
    const int32_t ibase = FLUID ? nbc : 0;
    const int32_t nitems = FLUID ? min(max(info[1], 0), K.n - nbc) : nbc;
    unsigned long long pairs_acc = 0;  // wave-uniform

    for (;;) {
        if (threadIdx.x == 0) sItem = atomicAdd(queue, 1);
        __syncthreads();
        const int32_t item = sItem;
        if (item >= nitems) break;
        const int32_t key = min(max(list[ibase + item], 0), 2 * K.ncell - 1);
        const int32_t c = FLUID ? max(key - K.ncell, 0) : min(key, K.ncell - 1);
        const int32_t cx = c % K.nc0, cy = (c / K.nc0) % K.nc1, cz = c / (K.nc0 * K.nc1);
        const int32_t tbeg = min(max(start[key], 0), K.n);
        const int32_t tend = min(max(start[key + 1], tbeg), K.n);

        build_runs<FLUID>(K, start, cx, cy, cz, R);
        const int32_t total = R.total;
        const int nr = R.nruns;

        if (!FLUID && total == 0) {
            // boundary cell with no fluid in reach
            for (int32_t a = tbeg + threadIdx.x; a < tend; a += blockDim.x) {
                ace[a] = make_float4(0.f, 0.f, 0.f, 0.f);
                visc[a] = 0.f;
                if (STATS) { stats[2 * a] = 0; stats[2 * a + 1] = 0; }
            }
            __syncthreads();
            continue;
        }

        for (int32_t tb = 0; tb < max(total, 1); tb += kTile) {
            const int32_t tlen = min(kTile, total - tb);
            // ---- stage candidates [tb, tb + tlen) into LDS
            for (int32_t l = threadIdx.x; l < tlen; l += blockDim.x) {
                const int32_t v = tb + l;
                int lo = 0, hi = nr;  // find r with vstart[r] <= v < vstart[r+1]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (R.vstart[mid] <= v) lo = mid;
                    else hi = mid;
                }
                const int r = lo;
                const int32_t j = min(max(R.s[r][0] + (v - R.vstart[r]), 0), K.n - 1);
                int ci = 0;
                for (int i = 1; i < R.ncx[r]; ++i) ci += R.s[r][i] <= j ? 1 : 0;
                const float4 p = pos[j];
                const float sx = (float)(R.dx0[r] + ci) * K.cellf;  // (k_b - k_a) cell, exact
                sP[l] = make_float4(p.x + sx, p.y + R.sy[r], p.z + R.sz[r], p.w);
                sV[l] = velrho[j];
                if (STATS) sSlot[l] = j;
            }
            __syncthreads();

            // ---- one wavefront per target
            const int32_t selfbase = FLUID ? R.vstart[R.self_run] - R.s[R.self_run][0] - tb : 0;
            for (int32_t a = tbeg + wave; a < tend; a += kWaves) {
                const float4 pa = pos[a];
                const float4 va = velrho[a];
                const int32_t self_l = FLUID ? selfbase + a : -1;
                const float rhoa = K.rho0 + va.w;
                const float ta = rhoa * K.inv_rho0;
                const float ca = K.c0 * ta * ta * ta;
                float sx = 0.f, sy = 0.f, sz = 0.f, sd = 0.f, vm = 0.f;
                unsigned hs = 0;
                int wp = 0, rp = 0;

                auto pair = [&](int idx) {
                    const float4 pb = sP[idx];
                    const float4 vb = sV[idx];
                    const float rx = pa.x - pb.x, ry = pa.y - pb.y, rz = pa.z - pb.z;
                    const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
                    const float r = __builtin_amdgcn_sqrtf(r2);
                    const float wq = __builtin_fmaf(-0.5f * K.inv_h, r, 1.0f);
                    const float F = K.kf * (wq * wq * wq);
                    const float vx = va.x - vb.x, vy = va.y - vb.y, vz = va.z - vb.z;
                    const float vdr = __builtin_fmaf(vz, rz, __builtin_fmaf(vy, ry, vx * rx));
                    sd = __builtin_fmaf(vdr, F, sd);
                    if (FLUID) {
                        const float rhob = K.rho0 + vb.w;
                        const float mu = K.h * vdr * __builtin_amdgcn_rcpf(r2 + K.eta2);
                        vm = fmaxf(vm, fabsf(mu));
                        const float tb3 = rhob * K.inv_rho0;
                        const float cb = K.c0 * tb3 * tb3 * tb3;
                        const float pi = vdr < 0.f
                                             ? -K.alpha * (ca + cb) * mu * __builtin_amdgcn_rcpf(rhoa + rhob)
                                             : 0.f;
                        const float coef = (pa.w + pb.w + pi) * F;
                        sx = __builtin_fmaf(coef, rx, sx);
                        sy = __builtin_fmaf(coef, ry, sy);
                        sz = __builtin_fmaf(coef, rz, sz);
                    }
                    if (STATS) hs += (uint32_t)ids[sSlot[idx]] * 2654435761u;
                };

                for (int32_t cb0 = 0; cb0 < tlen; cb0 += kWave) {
                    const int32_t j = cb0 + lane;
                    bool pass = false;
                    if (j < tlen) {
                        const float4 pb = sP[j];
                        const float rx = pa.x - pb.x, ry = pa.y - pb.y, rz = pa.z - pb.z;
                        const float r2 = __builtin_fmaf(rz, rz, __builtin_fmaf(ry, ry, rx * rx));
                        pass = r2 < K.rc2 && j != self_l;
                    }
                    const unsigned long long m = ballot(pass);
                    if (pass) sRing[wave][(wp + (int)lane_rank(m)) & (kRing - 1)] = (uint16_t)j;
                    wp += __popcll(m);
                    if (wp - rp >= kWave) {
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        pair(sRing[wave][(rp + lane) & (kRing - 1)]);
                        rp += kWave;
                    }
                }
                if (wp > rp) {
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    if (lane < wp - rp) pair(sRing[wave][(rp + lane) & (kRing - 1)]);
                }
                pairs_acc += (unsigned long long)wp;

                // ---- reduce over the wave, write (first tile) or accumulate
                const float tsd = wave_sum(sd);
                float tsx = 0.f, tsy = 0.f, tsz = 0.f, tvm = 0.f;
                if (FLUID) {
                    tsx = wave_sum(sx);
                    tsy = wave_sum(sy);
                    tsz = wave_sum(sz);
                    tvm = wave_max(vm);
                }
                unsigned ths = 0;
                if (STATS) ths = wave_sum_u(hs);
                if (lane == 0) {
                    float4 o;
                    if (FLUID)
                        o = make_float4(-K.mass * tsx, -K.mass * tsy, -K.mass * tsz, K.mass * tsd);
                    else
                        o = make_float4(0.f, 0.f, 0.f, K.mass * tsd);
                    if (tb == 0) {
                        if (FLUID) { o.x += K.gx; o.y += K.gy; o.z += K.gz; }
                        ace[a] = o;
                        visc[a] = tvm;
                        if (STATS) { stats[2 * a] = wp; stats[2 * a + 1] = (int32_t)ths; }
                    } else {
                        float4 p0 = ace[a];
                        p0.x += o.x; p0.y += o.y; p0.z += o.z; p0.w += o.w;
                        ace[a] = p0;
                        visc[a] = fmaxf(visc[a], tvm);
                        if (STATS) {
                            stats[2 * a] += wp;
                            stats[2 * a + 1] = (int32_t)((uint32_t)stats[2 * a + 1] + ths);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    if (npairs && lane == 0 && pairs_acc) atomicAdd(npairs, pairs_acc);
}

__global__ void k_zero_queue(int32_t *q)
{
    if (threadIdx.x == 0) q[0] = 0;
}

// Excluded particles (the tail of the sorted state) get zero outputs.
__global__ void k_zero_excluded(int32_t n, const int32_t *__restrict__ info, float4 *__restrict__ ace,
                                float *__restrict__ visc, int32_t *__restrict__ stats)
{
    const int32_t nex = info[2];
    for (int32_t i = n - nex + blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x) {
        ace[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        visc[i] = 0.f;
        if (stats) { stats[2 * i] = 0; stats[2 * i + 1] = 0; }
    }
}

static PairConsts pair_consts(const sph_grid *g, const sph_params *p)
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
    K.alpha = (float)p->alpha;
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
    K.n = 0;
    return K;
}

template <bool FLUID, bool STATS>
static hipError_t launch_one(const PairConsts &K, const sph_state *st, const sph_cells *cells,
                             float *ace, float *visc, unsigned long long *npairs, int32_t *stats,
                             int32_t *queue, hipStream_t s)
{
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_interact<FLUID, STATS>, kThreads, 0);
    if (e != hipSuccess) return e;
    if (cus <= 0) cus = 1;
    if (occ <= 0) occ = 1;
    const int grid = cus * occ;
    k_interact<FLUID, STATS><<<grid, kThreads, 0, s>>>(
        K, cells->start, cells->list, cells->info, (const float4 *)st->pos,
        (const float4 *)st->velrho, st->id, (float4 *)ace, visc, queue, npairs, stats);
    return hipGetLastError();
}

hipError_t launch_interact(const sph_grid *g, const sph_params *p, const sph_state *st,
                           const sph_cells *cells, unsigned parts, float *ace, float *visc,
                           unsigned long long *npairs, int32_t *nbr_stats, const Workspace &w,
                           hipStream_t s)
{
    if (st->n == 0) return hipSuccess;
    PairConsts K = pair_consts(g, p);
    K.n = st->n;
    hipError_t e = hipSuccess;
    if (parts & SPH_PI_FLUID) {
        k_zero_queue<<<1, 64, 0, s>>>(w.counters + 0);
        e = nbr_stats ? launch_one<true, true>(K, st, cells, ace, visc, npairs, nbr_stats,
                                               w.counters + 0, s)
                      : launch_one<true, false>(K, st, cells, ace, visc, npairs, nullptr,
                                                w.counters + 0, s);
        if (e != hipSuccess) return e;
    }
    if (parts & SPH_PI_BOUNDARY) {
        k_zero_queue<<<1, 64, 0, s>>>(w.counters + 1);
        k_zero_excluded<<<64, 256, 0, s>>>(st->n, cells->info, (float4 *)ace, visc, nbr_stats);
        e = nbr_stats ? launch_one<false, true>(K, st, cells, ace, visc, npairs, nbr_stats,
                                                w.counters + 1, s)
                      : launch_one<false, false>(K, st, cells, ace, visc, npairs, nullptr,
                                                 w.counters + 1, s);
    }
    return e;
}

}  // namespace sph
