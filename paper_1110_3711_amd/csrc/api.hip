// api.hip -- the extern "C" entry points: host-side validation, workspace
// layout and the calls into the per-stage launchers.
#include <math.h>

#include <atomic>
#include <mutex>

#include "sph_internal.h"

using namespace sph;

namespace {

bool grid_ok(const sph_grid *g)
{
    if (!g) return false;
    if (g->nsub != 1 && g->nsub != 2) return false;
    if (!(g->cell > 0.0) || !isfinite(g->cell)) return false;
    for (int d = 0; d < 3; ++d) {
        if (g->nc[d] <= 0) return false;
        if (!isfinite(g->origin[d]) || !isfinite(g->hi[d]) || !(g->hi[d] > g->origin[d]))
            return false;
        // the grid must cover the domain
        if ((double)g->nc[d] * g->cell < g->hi[d] - g->origin[d]) return false;
    }
    const int64_t ncell = ncell_of(g);
    return ncell > 0 && ncell < (1 << 30) - 1;
}

bool params_ok(const sph_grid *g, const sph_params *p)
{
    if (!p) return false;
    if (!(p->h > 0.0) || !(p->rho0 > 0.0) || !(p->c0 > 0.0) || !(p->mass > 0.0)) return false;
    if (p->gamma != 7.0) return false;
    if (p->kernel != SPH_WENDLAND5 && p->kernel != SPH_CUBIC_SPLINE) return false;
    if (p->verlet_ns < 1) return false;
    if (p->pos_policy != SPH_POS_OFFSET32 && p->pos_policy != SPH_POS_ABS64) return false;
    if (!(p->eta2 > 0.0) || !(p->alpha >= 0.0) || !(p->cfl > 0.0)) return false;
    // tensile correction: off (0) or a spacing inside the support
    if (!(p->tensile_dp >= 0.0) || !(p->tensile_dp < 2.0 * p->h)) return false;
    // the (2 nsub + 1)^3 stencil must cover the support 2h, with margin for
    // FP32 rounding of the offsets
    if (g->nsub * g->cell < 2.0 * p->h * (1.0 + ldexp(1.0, -21))) return false;
    return true;
}

bool state_ok(const sph_state *st, bool with_arrays = true)
{
    if (!st) return false;
    if (st->n < 0 || st->nb < 0 || st->nb > st->n) return false;
    if (with_arrays && st->n > 0 &&
        (!st->cell || !st->pos || !st->velrho || !st->velrho_prev || !st->id))
        return false;
    return true;
}

bool cells_ok(const sph_cells *c)
{
    return c && c->start && c->list && c->info;
}

bool build_args_ok(const sph_grid *g, const sph_state *src, const sph_state *dst,
                   const sph_cells *cells, const int32_t *perm, const int32_t *dev_status)
{
    if (!grid_ok(g) || !state_ok(src) || !dst || !cells_ok(cells) || !dev_status) return false;
    if (src->n > 0 && (!perm || !dst->cell || !dst->pos || !dst->velrho || !dst->velrho_prev ||
                       !dst->id))
        return false;
    if (src->n > 0 && (src->cell == dst->cell || src->pos == dst->pos ||
                       src->velrho == dst->velrho || src->velrho_prev == dst->velrho_prev ||
                       src->id == dst->id))
        return false;
    // FP64 positions are carried through when both sides hold them
    if ((src->pos64 == nullptr) != (dst->pos64 == nullptr)) return false;
    if (src->n > 0 && src->pos64 && src->pos64 == dst->pos64) return false;
    return true;
}

sph_status ws_check(const sph_grid *g, int32_t n, void *ws, size_t ws_bytes, Workspace *w)
{
    layout_workspace(g, n, nullptr, w);
    if (!ws || ws_bytes < w->bytes) return SPH_ERR_WORKSPACE;
    layout_workspace(g, n, ws, w);
    return SPH_OK;
}

sph_status hip_status(hipError_t e) { return e == hipSuccess ? SPH_OK : SPH_ERR_HIP; }

// The library's own scratch for callers that cannot allocate
// (sph_build_cells_static).  Each device holds its copy of the array for the
// life of the process.  In host code `scratch` names a host-side stand-in:
// kernels and copies get the device address that hipGetSymbolAddress
// returns, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SPH_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

hipError_t scratch_of_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!p) return hipErrorInvalidSymbol;
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t sph_abi_version(void) { return SPH_ABI_VERSION; }

size_t sph_ranges_bytes(const sph_grid *g)
{
    if (!grid_ok(g)) return 0;
    const size_t side = 2 * (size_t)g->nsub + 1;
    return (size_t)ncell_of(g) * 2 * side * side * 2 * sizeof(int32_t);
}

size_t sph_workspace_bytes(const sph_grid *g, int32_t n)
{
    if (!grid_ok(g) || n < 0) return 0;
    Workspace w;
    layout_workspace(g, n, nullptr, &w);
    return w.bytes;
}

sph_status sph_encode(const sph_grid *g, const sph_params *p, const double *x, const double *v,
                      const double *rho, sph_state *st, int32_t *dev_status, hipStream_t stream)
{
    if (!grid_ok(g) || !params_ok(g, p) || !state_ok(st) || !dev_status) return SPH_ERR_ARG;
    if (st->n > 0 && (!x || !v || !rho)) return SPH_ERR_ARG;
    return hip_status(launch_encode(g, p, x, v, rho, st, dev_status, stream));
}

sph_status sph_decode(const sph_grid *g, const sph_params *p, const sph_state *st, double *x,
                      double *v, double *rho, hipStream_t stream)
{
    if (!grid_ok(g) || !params_ok(g, p) || !state_ok(st)) return SPH_ERR_ARG;
    if (st->n > 0 && (!x || !v || !rho)) return SPH_ERR_ARG;
    return hip_status(launch_decode(g, p, st, x, v, rho, stream));
}

sph_status sph_build_cells(const sph_grid *g, const sph_state *src, sph_state *dst,
                           sph_cells *cells, int32_t *perm, void *ws, size_t ws_bytes,
                           int32_t *dev_status, hipStream_t stream)
{
    if (!build_args_ok(g, src, dst, cells, perm, dev_status)) return SPH_ERR_ARG;
    Workspace w;
    const sph_status ws_st = ws_check(g, src->n, ws, ws_bytes, &w);
    if (ws_st != SPH_OK) return ws_st;
    return hip_status(launch_build_cells(g, src, dst, cells, perm, w, dev_status, stream));
}

sph_status sph_build_cells_static(const sph_grid *g, const sph_state *src, sph_state *dst,
                                  sph_cells *cells, int32_t *perm, int32_t *dev_status,
                                  hipStream_t stream)
{
    if (!build_args_ok(g, src, dst, cells, perm, dev_status)) return SPH_ERR_ARG;
    // the size check comes before any device call
    Workspace w;
    layout_workspace(g, src->n, nullptr, &w);
    if (w.bytes > (size_t)SPH_STATIC_SCRATCH_BYTES) return SPH_ERR_WORKSPACE;
    void *base = nullptr;
    const hipError_t e = scratch_of_current_device(&base);
    if (e != hipSuccess) return SPH_ERR_HIP;
    layout_workspace(g, src->n, base, &w);
    return hip_status(launch_build_cells(g, src, dst, cells, perm, w, dev_status, stream));
}

sph_status sph_interact(const sph_grid *g, const sph_params *p, const sph_state *st,
                        const sph_cells *cells, unsigned parts, float *ace, float *visc,
                        unsigned long long *npairs, int32_t *nbr_stats, void *ws,
                        size_t ws_bytes, hipStream_t stream)
{
    if (!grid_ok(g) || !params_ok(g, p) || !state_ok(st) || !cells_ok(cells)) return SPH_ERR_ARG;
    if (parts == 0 || (parts & ~SPH_PI_ALL)) return SPH_ERR_ARG;
    if (st->n > 0 && (!ace || !visc)) return SPH_ERR_ARG;
    if (p->pos_policy == SPH_POS_ABS64 &&
        (p->kernel != SPH_WENDLAND5 || p->tensile_dp != 0.0 || nbr_stats ||
         (st->n > 0 && !st->pos64)))
        return SPH_ERR_ARG;
    Workspace w;
    const sph_status ws_st = ws_check(g, st->n, ws, ws_bytes, &w);
    if (ws_st != SPH_OK) return ws_st;
    return hip_status(launch_interact(g, p, st, cells, parts, ace, visc, npairs, nbr_stats, w, stream));
}

sph_status sph_step(const sph_grid *g, const sph_params *p, sph_state *st, const float *ace,
                    const float *visc, double *dt, long long step, unsigned flags,
                    sph_adjoint *adj, void *ws, size_t ws_bytes, int32_t *dev_status,
                    hipStream_t stream)
{
    if (!grid_ok(g) || !params_ok(g, p) || !state_ok(st) || !dt || !dev_status || step < 0)
        return SPH_ERR_ARG;
    if (flags & ~(SPH_FIXED_DT | SPH_ADJOINT)) return SPH_ERR_ARG;
    if (flags & SPH_ADJOINT) {
        if (!adj) return SPH_ERR_ARG;
        if (st->n > 0 && (!ace || !adj->pos_bar || !adj->velrho_bar || !adj->velrho_prev_bar ||
                          !adj->ace_bar))
            return SPH_ERR_ARG;
    } else if (st->n > 0 && (!ace || (!(flags & SPH_FIXED_DT) && !visc))) {
        return SPH_ERR_ARG;
    }
    Workspace w;
    const sph_status ws_st = ws_check(g, st->n, ws, ws_bytes, &w);
    if (ws_st != SPH_OK) return ws_st;
    return hip_status(launch_step(g, p, st, ace, visc, dt, step, flags, adj, w, dev_status, stream));
}

sph_status sph_interact_backward(const sph_grid *g, const sph_params *p, const sph_state *st,
                                 const sph_cells *cells, const float *ace_bar, float *pos_bar,
                                 float *velrho_bar, double *alpha_bar, void *ws,
                                 size_t ws_bytes, hipStream_t stream)
{
    if (!grid_ok(g) || !params_ok(g, p) || !state_ok(st) || !cells_ok(cells) || !alpha_bar)
        return SPH_ERR_ARG;
    if (p->pos_policy != SPH_POS_OFFSET32) return SPH_ERR_ARG;
    if (st->n > 0 && (!ace_bar || !pos_bar || !velrho_bar)) return SPH_ERR_ARG;
    Workspace w;
    const sph_status ws_st = ws_check(g, st->n, ws, ws_bytes, &w);
    if (ws_st != SPH_OK) return ws_st;
    return hip_status(launch_interact_backward(g, p, st, cells, ace_bar, pos_bar, velrho_bar,
                                               alpha_bar, w, stream));
}

sph_status sph_conservation(const sph_grid *g, const sph_params *p, const sph_state *st,
                            const float *ace, double *out, void *ws, size_t ws_bytes,
                            hipStream_t stream)
{
    if (!grid_ok(g) || !params_ok(g, p) || !state_ok(st) || !out) return SPH_ERR_ARG;
    Workspace w;
    const sph_status ws_st = ws_check(g, st->n, ws, ws_bytes, &w);
    if (ws_st != SPH_OK) return ws_st;
    return hip_status(launch_conservation(g, p, st, ace, out, w, stream));
}

sph_status sph_build_cells_backward(const int32_t *perm, int32_t n, const sph_adjoint *dst_bar,
                                    sph_adjoint *src_bar, hipStream_t stream)
{
    if (n < 0 || !dst_bar || !src_bar) return SPH_ERR_ARG;
    if (n > 0 && (!perm || !dst_bar->pos_bar || !dst_bar->velrho_bar ||
                  !dst_bar->velrho_prev_bar || !src_bar->pos_bar || !src_bar->velrho_bar ||
                  !src_bar->velrho_prev_bar))
        return SPH_ERR_ARG;
    if (n > 0 && (dst_bar->pos_bar == src_bar->pos_bar ||
                  dst_bar->velrho_bar == src_bar->velrho_bar ||
                  dst_bar->velrho_prev_bar == src_bar->velrho_prev_bar))
        return SPH_ERR_ARG;
    return hip_status(launch_unsort_adjoint(perm, n, dst_bar, src_bar, stream));
}

}  // extern "C"
