// encode.hip -- FP64 positions <-> integer cell + FP32 offset device state.
#include "sph_internal.h"

namespace sph {

struct GridD {
    double org[3], hi[3];
    double cell;
    int32_t nc[3];
};

static GridD grid_d(const sph_grid *g)
{
    GridD d;
    for (int i = 0; i < 3; ++i) {
        d.org[i] = g->origin[i];
        d.hi[i] = g->hi[i];
        d.nc[i] = g->nc[i];
    }
    d.cell = g->cell;
    return d;
}

__global__ void k_encode(GridD G, double rho0, double B, int32_t n, int32_t nb,
                         const double *__restrict__ x,
                         const double *__restrict__ v, const double *__restrict__ rho,
                         int32_t *__restrict__ cell, float4 *__restrict__ pos,
                         float4 *__restrict__ velrho, float4 *__restrict__ velrho_prev,
                         int32_t *__restrict__ id, double *__restrict__ pos64,
                         int32_t *__restrict__ dev_status)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (pos64) {
        for (int d = 0; d < 3; ++d) pos64[3 * (int64_t)i + d] = x[3 * (int64_t)i + d];
    }
    bool ok = true;
    int64_t k[3];
    float o[3];
    for (int d = 0; d < 3; ++d) {
        const double xd = x[3 * (int64_t)i + d];
        if (!(xd >= G.org[d] && xd < G.hi[d])) { ok = false; break; }
        const double dd = xd - G.org[d];
        const double kf = floor(dd / G.cell);
        if (kf < 0.0 || kf >= (double)G.nc[d]) { ok = false; break; }
        k[d] = (int64_t)kf;
        o[d] = (float)fma(-(kf + 0.5), G.cell, dd);
    }
    const double w = rho[i] - rho0;
    const float pw = (float)p_over_rho2(w, rho0, B);
    const float4 vr = make_float4((float)v[3 * (int64_t)i], (float)v[3 * (int64_t)i + 1],
                                  (float)v[3 * (int64_t)i + 2], (float)w);
    velrho[i] = vr;
    velrho_prev[i] = vr;
    id[i] = i;
    if (!ok) {
        cell[i] = SPH_EXCLUDED;
        pos[i] = make_float4(0.f, 0.f, 0.f, pw);
        atomicOr(dev_status, i < nb ? SPH_DEV_OUT_OF_GRID | SPH_DEV_BOUNDARY_OUT
                                    : SPH_DEV_OUT_OF_GRID);
        return;
    }
    cell[i] = (int32_t)(k[0] + (int64_t)G.nc[0] * (k[1] + (int64_t)G.nc[1] * k[2]));
    pos[i] = make_float4(o[0], o[1], o[2], pw);
}

__global__ void k_decode(GridD G, double rho0, int32_t n, const int32_t *__restrict__ cell,
                         const float4 *__restrict__ pos, const float4 *__restrict__ velrho,
                         const double *__restrict__ pos64, double *__restrict__ x,
                         double *__restrict__ v, double *__restrict__ rho)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cell[i];
    const float4 p = pos[i];
    const float4 vr = velrho[i];
    if (c == SPH_EXCLUDED) {
        x[3 * (int64_t)i] = x[3 * (int64_t)i + 1] = x[3 * (int64_t)i + 2] = __builtin_nan("");
    } else if (pos64) {
        for (int d = 0; d < 3; ++d) x[3 * (int64_t)i + d] = pos64[3 * (int64_t)i + d];
    } else {
        const int32_t kx = c % G.nc[0];
        const int32_t ky = (c / G.nc[0]) % G.nc[1];
        const int32_t kz = c / (G.nc[0] * G.nc[1]);
        x[3 * (int64_t)i] = fma((double)kx + 0.5, G.cell, G.org[0]) + (double)p.x;
        x[3 * (int64_t)i + 1] = fma((double)ky + 0.5, G.cell, G.org[1]) + (double)p.y;
        x[3 * (int64_t)i + 2] = fma((double)kz + 0.5, G.cell, G.org[2]) + (double)p.z;
    }
    v[3 * (int64_t)i] = vr.x;
    v[3 * (int64_t)i + 1] = vr.y;
    v[3 * (int64_t)i + 2] = vr.z;
    rho[i] = rho0 + (double)vr.w;
}

hipError_t launch_encode(const sph_grid *g, const sph_params *p, const double *x, const double *v,
                         const double *rho, sph_state *st, int32_t *dev_status, hipStream_t s)
{
    if (st->n == 0) return hipSuccess;
    const double B = p->c0 * p->c0 * p->rho0 / p->gamma;
    const int threads = 256;
    const int blocks = (st->n + threads - 1) / threads;
    k_encode<<<blocks, threads, 0, s>>>(grid_d(g), p->rho0, B, st->n, st->nb, x, v, rho, st->cell,
                                        (float4 *)st->pos, (float4 *)st->velrho,
                                        (float4 *)st->velrho_prev, st->id, st->pos64, dev_status);
    return hipGetLastError();
}

hipError_t launch_decode(const sph_grid *g, const sph_params *p, const sph_state *st, double *x,
                         double *v, double *rho, hipStream_t s)
{
    if (st->n == 0) return hipSuccess;
    const int threads = 256;
    const int blocks = (st->n + threads - 1) / threads;
    k_decode<<<blocks, threads, 0, s>>>(grid_d(g), p->rho0, st->n, st->cell,
                                        (const float4 *)st->pos, (const float4 *)st->velrho,
                                        st->pos64, x, v, rho);
    return hipGetLastError();
}

}  // namespace sph
