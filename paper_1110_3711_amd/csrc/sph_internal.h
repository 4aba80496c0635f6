// sph_internal.h -- shared declarations of the gfx950 kernels and host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph.h"

namespace sph {

constexpr int kWave = 64;            // CDNA4 wavefront
constexpr int kSortThreads = 512;    // radix sort block (8 wavefronts)
constexpr int kSortItems = 8;        // keys per thread per block
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBitsMax = 11;    // digit width of a pass: at most 11 bits
constexpr int kRadixMax = 1 << kRadixBitsMax;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kReduceThreads = 256;
constexpr int kReduceBlocksMax = 1024;
constexpr int kConsSums = 16;        // conservation sums (sph_conservation)
// work-queue counters of the pair kernels: kCounterSlots counters, each on a
// 128-byte line of its own (atomics of many workgroups on one line queue
// behind each other)
constexpr int kCounterStride = 32;
constexpr int kCounterSlots = 64;

inline int64_t ncell_of(const sph_grid *g)
{
    return (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace layout, shared by every entry point of one simulation.
struct Workspace {
    uint32_t *keys0, *vals0, *keys1, *vals1;  // radix ping-pong [n] each
    uint32_t *hist;                           // [kRadixMax * nblk_sort] digit-major
    uint32_t *hist2;                          // the same, second pass (filled by the first)
    unsigned long long *partials;             // scan partial sums
    unsigned long long *keyscan;              // [nkeys + 1] packed (count << 32 | nonempty)
    int32_t *counters;                        // [kCounterSlots * kCounterStride] work queues
    int32_t *active;                          // [n] boundary cells with fluid in reach
    float *alpha_part;                        // [n] per-slot alpha adjoint
    double *reduce;                           // [kConsSums * kReduceBlocksMax] block partials
                                              //   (CFL maxima, conservation sums)
    size_t bytes;
};

inline int nblk_sort(int64_t n) { return (int)((n + kSortTile - 1) / kSortTile); }

inline size_t scan_partials_needed(int64_t len) { return (size_t)((len + kScanTile - 1) / kScanTile) + 1; }

inline bool layout_workspace(const sph_grid *g, int64_t n, void *base, Workspace *w)
{
    const int64_t ncell = ncell_of(g);
    const int64_t nkeys = 2 * ncell + 1;
    const int64_t nb = nblk_sort(n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t o_k0 = take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    const size_t o_v0 = take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    const size_t o_k1 = take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    const size_t o_v1 = take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    const size_t o_h = take(sizeof(uint32_t) * (size_t)kRadixMax * (size_t)(nb > 0 ? nb : 1));
    const size_t o_h2 = take(sizeof(uint32_t) * (size_t)kRadixMax * (size_t)(nb > 0 ? nb : 1));
    size_t np = scan_partials_needed((int64_t)kRadixMax * nb);
    const size_t np2 = scan_partials_needed(nkeys + 1);
    if (np2 > np) np = np2;
    const size_t o_p = take(sizeof(unsigned long long) * np);
    const size_t o_ks = take(sizeof(unsigned long long) * (size_t)(nkeys + 1));
    const size_t o_c = take(sizeof(int32_t) * kCounterSlots * kCounterStride);
    const size_t o_a = take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    const size_t o_ap = take(sizeof(float) * (size_t)(n > 0 ? n : 1));
    const size_t o_r = take(sizeof(double) * kConsSums * kReduceBlocksMax);
    w->bytes = off;
    if (base) {
        char *b = (char *)base;
        w->keys0 = (uint32_t *)(b + o_k0);
        w->vals0 = (uint32_t *)(b + o_v0);
        w->keys1 = (uint32_t *)(b + o_k1);
        w->vals1 = (uint32_t *)(b + o_v1);
        w->hist = (uint32_t *)(b + o_h);
        w->hist2 = (uint32_t *)(b + o_h2);
        w->partials = (unsigned long long *)(b + o_p);
        w->keyscan = (unsigned long long *)(b + o_ks);
        w->counters = (int32_t *)(b + o_c);
        w->active = (int32_t *)(b + o_a);
        w->alpha_part = (float *)(b + o_ap);
        w->reduce = (double *)(b + o_r);
    }
    return true;
}

// FP32 constants of the pair kernels, derived once on the host in FP64.
struct PairConsts {
    float cellf;     // cell side
    float rc2;       // (2h)^2
    float h;         // smoothing length
    float inv_h;     // 1/h
    float kf;        // F = kf (1 - q/2)^3, kf = -5 aD / h^2, aD = 21 / (16 pi h^3)
    float eta2;
    float kpi;       // -alpha c0 / rho0
    float kpa;       // -c0 / rho0 (d Pi / d alpha per unit cr min(mu, 0))
    float kfr;       // (dF/dr)/r = kfr (1 - q/2)^2 / r, kfr = -3 kf / (2h)
    // cubic spline, aD = 1 / (pi h^3):
    //   q < 1:  F = kc_in (9q/4 - 3),      (dF/dr)/r = kcr_in / r
    //   q >= 1: F = kc_out (2 - q)^2 / r,  (dF/dr)/r = kcr_out (4 - q^2) / r^3
    float kc_in;     // aD / h^2
    float kc_out;    // -3 aD / (4h)
    float kcr_in;    // 9 aD / (4 h^3)
    float kcr_out;   // 3 aD / (4h)
    int32_t kernel;  // SPH_WENDLAND5 or SPH_CUBIC_SPLINE (selects the instantiation)
    // forward pair sums carry G = F / gs (Wendland: G = (1 - q/2)^3, gs = kf;
    // cubic: G = 9q/4 - 3 or kco (2 - q)^2 / r, gs = kc_in)
    float gs;
    float kco;       // cubic: kc_out / kc_in = -3h/4
    float mgs;       // mass * gs
    float kh;        // -alpha h c0 / rho0: Pi_ab = kh cr min(u, 0), mu = h u
    // tensile correction (tensile != 0): f = Wn(r) / Wn(dp) with the kernel
    // shape Wn = W / aD; inv_wdp = 1 / W(dp) with aD (for dT/dr = R 4 f^3 F / W(dp))
    int32_t tensile;
    float inv_wndp;  // 1 / Wn(dp)
    float inv_wdp;   // 1 / W(dp)
    float c0;
    float rho0;
    float inv_rho0;
    float gx, gy, gz;
    float mass;
    int32_t nsub;
    int32_t nc0, nc1, nc2;
    int32_t ncell;
    int32_t n;       // particles in the state
    float xlo, xscale, xwin;  // x-bins of the staged candidates; window half-width
    float half, cull2;        // target-cell half side and squared cutoff of the staging
                              //   box test, both enlarged to cover FP32 rounding
    // position-load policy SPH_POS_ABS64: pair vectors from FP64 absolute
    // positions, relative to the target cell's centre org64 + (k + 1/2) cell64
    int32_t pos_policy;
    double org64[3];
    double cell64;
};

// Host launchers (one per source file).
hipError_t launch_encode(const sph_grid *g, const sph_params *p, const double *x, const double *v,
                         const double *rho, sph_state *st, int32_t *dev_status, hipStream_t s);
hipError_t launch_decode(const sph_grid *g, const sph_params *p, const sph_state *st, double *x,
                         double *v, double *rho, hipStream_t s);
hipError_t launch_build_cells(const sph_grid *g, const sph_state *src, sph_state *dst,
                              sph_cells *cells, int32_t *perm, const Workspace &w,
                              int32_t *dev_status, hipStream_t s);
hipError_t launch_interact(const sph_grid *g, const sph_params *p, const sph_state *st,
                           const sph_cells *cells, unsigned parts, float *ace, float *visc,
                           unsigned long long *npairs, int32_t *nbr_stats, const Workspace &w,
                           hipStream_t s);
hipError_t launch_interact_backward(const sph_grid *g, const sph_params *p, const sph_state *st,
                                    const sph_cells *cells, const float *ace_bar, float *pos_bar,
                                    float *velrho_bar, double *alpha_bar, const Workspace &w,
                                    hipStream_t s);
hipError_t launch_conservation(const sph_grid *g, const sph_params *p, const sph_state *st,
                               const float *ace, double *out, const Workspace &w, hipStream_t s);
hipError_t launch_unsort_adjoint(const int32_t *perm, int32_t n, const sph_adjoint *dst_bar,
                                 sph_adjoint *src_bar, hipStream_t s);
hipError_t launch_step(const sph_grid *g, const sph_params *p, sph_state *st, const float *ace,
                       const float *visc, double *dt, long long step, unsigned flags,
                       sph_adjoint *adj, const Workspace &w, int32_t *dev_status, hipStream_t s);

// ---------------------------------------------------------------------------
// Device helpers

// Tait pressure over rho^2 for gamma = 7, FP64:  B ((1+d)^7 - 1) / rho^2 with
// (1+d)^7 - 1 = d * sum_{k<7} (1+d)^k (no cancellation near rho0).
__device__ inline double p_over_rho2(double w, double rho0, double B)
{
    const double d = w / rho0;
    const double u = 1.0 + d;
    double s = 1.0;
    for (int k = 0; k < 6; ++k) s = fma(s, u, 1.0);
    const double rho = rho0 + w;
    return B * d * s / (rho * rho);
}

__device__ inline unsigned long long ballot(bool pred)
{
    return __builtin_amdgcn_ballot_w64(pred);
}

// number of set bits of m in lanes below this lane
__device__ inline unsigned lane_rank(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ inline int lane_id() { return (int)lane_rank(~0ull); }

}  // namespace sph
