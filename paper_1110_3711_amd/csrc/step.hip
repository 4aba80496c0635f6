// step.hip -- system-update stage (Section 4.1 "SU"): the variable time step
// from global maxima (FP64 block reduction, deterministic) and the Verlet
// update (Table 1) with an FP64 position update that re-bins each particle
// into (cell, FP32 offset).
#include "sph_internal.h"

namespace sph {

struct StepConsts {
    double org[3], hi[3];
    double cell;
    int32_t nc[3];
    double h, rho0, c0, cfl, B;
    int32_t verlet_ns, bound_floor;
};

// Per block: max |a|^2 and max (c + visc) over fluid, non-excluded slots, and
// a flag for non-finite values.  out[3 b + {0,1,2}].
__global__ __launch_bounds__(kReduceThreads) void k_cfl_partial(
    StepConsts C, int32_t n, int32_t nb, const int32_t *__restrict__ cell,
    const float4 *__restrict__ velrho, const float4 *__restrict__ ace,
    const float *__restrict__ visc, double *__restrict__ out)
{
    __shared__ double s_a[kReduceThreads], s_c[kReduceThreads], s_f[kReduceThreads];
    // Every value the update consumes is checked: a non-finite acceleration,
    // density rate or viscosity anywhere (fluid or boundary) flags the step.
    double am = 0.0, cm = 0.0, bad = 0.0;
    const double big = 1.7976931348623157e308;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (cell[i] == SPH_EXCLUDED) continue;
        const float4 a = ace[i];
        if (i < nb) {
            if (!(fabs((double)a.w) <= big)) bad = 1.0;
            continue;
        }
        const double ax = a.x, ay = a.y, az = a.z;
        const double a2 = ax * ax + ay * ay + az * az;
        const double t = (C.rho0 + (double)velrho[i].w) / C.rho0;
        const double cv = C.c0 * t * t * t + (double)visc[i];
        if (!(a2 <= big) || !(cv <= big) || !(fabs((double)a.w) <= big)) bad = 1.0;
        else {
            am = fmax(am, a2);
            cm = fmax(cm, cv);
        }
    }
    const int t = threadIdx.x;
    s_a[t] = am;
    s_c[t] = cm;
    s_f[t] = bad;
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
            s_a[t] = fmax(s_a[t], s_a[t + o]);
            s_c[t] = fmax(s_c[t], s_c[t + o]);
            s_f[t] = fmax(s_f[t], s_f[t + o]);
        }
        __syncthreads();
    }
    if (t == 0) {
        out[3 * blockIdx.x] = s_a[0];
        out[3 * blockIdx.x + 1] = s_c[0];
        out[3 * blockIdx.x + 2] = s_f[0];
    }
}

// dt = cfl * min( sqrt(h / max|a|), h / max(c + visc) ); the minimum over
// particles of a monotone function equals the function of the maximum.
__global__ __launch_bounds__(kReduceThreads) void k_cfl_final(StepConsts C, int nblk,
                                                             const double *__restrict__ part,
                                                             double *__restrict__ dt,
                                                             int32_t *__restrict__ dev_status)
{
    __shared__ double s_a[kReduceThreads], s_c[kReduceThreads], s_f[kReduceThreads];
    const int t = threadIdx.x;
    double am = 0.0, cm = 0.0, bad = 0.0;
    for (int b = t; b < nblk; b += kReduceThreads) {
        am = fmax(am, part[3 * b]);
        cm = fmax(cm, part[3 * b + 1]);
        bad = fmax(bad, part[3 * b + 2]);
    }
    s_a[t] = am;
    s_c[t] = cm;
    s_f[t] = bad;
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
            s_a[t] = fmax(s_a[t], s_a[t + o]);
            s_c[t] = fmax(s_c[t], s_c[t + o]);
            s_f[t] = fmax(s_f[t], s_f[t + o]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double inf = __builtin_inf();
        const double tf = s_a[0] > 0.0 ? sqrt(C.h / sqrt(s_a[0])) : inf;
        const double tc = s_c[0] > 0.0 ? C.h / s_c[0] : inf;
        double d = C.cfl * fmin(tf, tc);
        if (s_f[0] != 0.0 || !(d > 0.0) || !(d < inf)) {
            atomicOr(dev_status, SPH_DEV_NONFINITE);
            d = __builtin_nan("");
        }
        dt[0] = d;
    }
}

// ---------------------------------------------------------------------------
// Global sums of the conservation laws (Section 2), FP64, over the fluid
// slots that are not excluded.  Fixed order: block b takes slots nb + b T + t
// + k G T (T threads, G blocks, G fixed by n), reduces them by a tree in LDS
// and writes kConsSums partials; one block then sums the partials in a fixed
// tree.  Results are bitwise reproducible for a given n.

struct ConsConsts {
    double org[3];
    double cell;
    int32_t nc[3];
    double g[3];
    double mass;
};

// Per-slot terms: m v (3), m f (3), m |v|^2 / 2, -m g.x, m x cross v (3),
// m x cross f (3), 1, m |f|, with f = a - g; the mass is applied at the end.
__global__ __launch_bounds__(kReduceThreads) void k_cons_partial(
    ConsConsts C, int32_t n, int32_t nb, const int32_t *__restrict__ cell,
    const float4 *__restrict__ pos, const float4 *__restrict__ velrho,
    const float4 *__restrict__ ace, double *__restrict__ out)
{
    __shared__ double sh[kConsSums][kReduceThreads];
    double acc[kConsSums];
#pragma unroll
    for (int k = 0; k < kConsSums; ++k) acc[k] = 0.0;
    for (int32_t i = nb + blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x) {
        const int32_t c = cell[i];
        if (c == SPH_EXCLUDED) continue;
        const int32_t k[3] = {c % C.nc[0], (c / C.nc[0]) % C.nc[1], c / (C.nc[0] * C.nc[1])};
        const float4 o = pos[i];
        const float of[3] = {o.x, o.y, o.z};
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = fma((double)k[d] + 0.5, C.cell, C.org[d]) + (double)of[d];
        const float4 vr = velrho[i];
        const double v[3] = {vr.x, vr.y, vr.z};
        acc[0] += v[0];
        acc[1] += v[1];
        acc[2] += v[2];
        acc[6] += 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        acc[7] -= C.g[0] * x[0] + C.g[1] * x[1] + C.g[2] * x[2];
        acc[8] += x[1] * v[2] - x[2] * v[1];
        acc[9] += x[2] * v[0] - x[0] * v[2];
        acc[10] += x[0] * v[1] - x[1] * v[0];
        acc[14] += 1.0;
        if (ace) {
            const float4 a = ace[i];
            const double f[3] = {(double)a.x - C.g[0], (double)a.y - C.g[1], (double)a.z - C.g[2]};
            acc[3] += f[0];
            acc[4] += f[1];
            acc[5] += f[2];
            acc[11] += x[1] * f[2] - x[2] * f[1];
            acc[12] += x[2] * f[0] - x[0] * f[2];
            acc[13] += x[0] * f[1] - x[1] * f[0];
            acc[15] += sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        }
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kConsSums; ++k) sh[k][t] = acc[k];
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int k = 0; k < kConsSums; ++k) sh[k][t] += sh[k][t + o];
        }
        __syncthreads();
    }
    if (t < kConsSums) out[(int64_t)kConsSums * blockIdx.x + t] = sh[t][0];
}

__global__ __launch_bounds__(kReduceThreads) void k_cons_final(ConsConsts C, int nblk,
                                                              const double *__restrict__ part,
                                                              double *__restrict__ result)
{
    __shared__ double sh[kConsSums][kReduceThreads];
    const int t = threadIdx.x;
    double acc[kConsSums];
#pragma unroll
    for (int k = 0; k < kConsSums; ++k) acc[k] = 0.0;
    for (int b = t; b < nblk; b += kReduceThreads) {
#pragma unroll
        for (int k = 0; k < kConsSums; ++k) acc[k] += part[(int64_t)kConsSums * b + k];
    }
#pragma unroll
    for (int k = 0; k < kConsSums; ++k) sh[k][t] = acc[k];
    __syncthreads();
    for (int o = kReduceThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int k = 0; k < kConsSums; ++k) sh[k][t] += sh[k][t + o];
        }
        __syncthreads();
    }
    if (t < kConsSums) result[t] = t == 14 ? sh[t][0] : C.mass * sh[t][0];
}

hipError_t launch_conservation(const sph_grid *g, const sph_params *p, const sph_state *st,
                               const float *ace, double *out, const Workspace &w, hipStream_t s)
{
    ConsConsts C;
    for (int d = 0; d < 3; ++d) {
        C.org[d] = g->origin[d];
        C.nc[d] = g->nc[d];
        C.g[d] = p->g[d];
    }
    C.cell = g->cell;
    C.mass = p->mass;
    const int64_t nf = (int64_t)st->n - st->nb;
    int nblk = (int)((nf + kReduceThreads - 1) / kReduceThreads);
    if (nblk > kReduceBlocksMax) nblk = kReduceBlocksMax;
    if (nblk < 1) nblk = 1;
    k_cons_partial<<<nblk, kReduceThreads, 0, s>>>(C, st->n, st->nb, st->cell,
                                                   (const float4 *)st->pos,
                                                   (const float4 *)st->velrho,
                                                   (const float4 *)ace, w.reduce);
    k_cons_final<<<1, kReduceThreads, 0, s>>>(C, nblk, w.reduce, out);
    return hipGetLastError();
}

__device__ inline void decode_cell(int32_t c, const int32_t *nc, int32_t &kx, int32_t &ky, int32_t &kz)
{
    kx = c % nc[0];
    ky = (c / nc[0]) % nc[1];
    kz = c / (nc[0] * nc[1]);
}

__global__ void k_verlet(StepConsts C, int32_t n, int32_t nb, int corrective,
                         const double *__restrict__ dtp, int32_t *__restrict__ cell,
                         float4 *__restrict__ pos, float4 *__restrict__ velrho,
                         float4 *__restrict__ velrho_prev, const float4 *__restrict__ ace,
                         double *__restrict__ pos64, int32_t *__restrict__ dev_status)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dt = dtp[0];
    if (!(dt > 0.0 && dt < __builtin_inf())) return;  // non-finite time step: state kept
    const int32_t c = cell[i];
    if (c == SPH_EXCLUDED) return;
    const float4 a = ace[i];
    const float4 vr = velrho[i];
    const float4 vp = velrho_prev[i];
    const double D = a.w;
    double w1 = corrective ? (double)vr.w + dt * D : (double)vp.w + 2.0 * dt * D;
    if (i < nb) {
        if (C.bound_floor && w1 < 0.0) w1 = 0.0;
        velrho_prev[i] = vr;
        velrho[i] = make_float4(vr.x, vr.y, vr.z, (float)w1);
        pos[i].w = (float)p_over_rho2(w1, C.rho0, C.B);
        return;
    }
    int32_t k[3];
    decode_cell(c, C.nc, k[0], k[1], k[2]);
    const float of[3] = {pos[i].x, pos[i].y, pos[i].z};
    const float vf[3] = {vr.x, vr.y, vr.z};
    const float pf[3] = {vp.x, vp.y, vp.z};
    const float af[3] = {a.x, a.y, a.z};
    float on[3], vn[3];
    bool out = false;
    for (int d = 0; d < 3; ++d) {
        if (pos64) {
            // FP64 absolute position: update it, then bin it as sph_encode does
            const double xn = pos64[3 * (int64_t)i + d] + dt * (double)vf[d] +
                              0.5 * dt * dt * (double)af[d];
            pos64[3 * (int64_t)i + d] = xn;
            const double dd = xn - C.org[d];
            const double kf = floor(dd / C.cell);
            if (!(xn >= C.org[d] && xn < C.hi[d]) || kf < 0.0 || kf >= (double)C.nc[d]) out = true;
            const int64_t kn = out ? 0 : (int64_t)kf;
            on[d] = (float)fma(-((double)kn + 0.5), C.cell, dd);
            k[d] = (int32_t)kn;
        } else {
            const double u = (double)of[d] + dt * (double)vf[d] + 0.5 * dt * dt * (double)af[d];
            const double sh = floor(u / C.cell + 0.5);
            const int64_t kn = (int64_t)k[d] + (int64_t)sh;
            on[d] = (float)fma(-sh, C.cell, u);
            const double xabs = fma((double)kn + 0.5, C.cell, C.org[d]) + (double)on[d];
            if (kn < 0 || kn >= C.nc[d] || !(xabs >= C.org[d] && xabs < C.hi[d])) out = true;
            k[d] = (int32_t)kn;
        }
        vn[d] = (float)(corrective ? (double)vf[d] + dt * (double)af[d]
                                   : (double)pf[d] + 2.0 * dt * (double)af[d]);
    }
    velrho_prev[i] = vr;
    velrho[i] = make_float4(vn[0], vn[1], vn[2], (float)w1);
    const float pw = (float)p_over_rho2(w1, C.rho0, C.B);
    if (out) {
        cell[i] = SPH_EXCLUDED;
        pos[i] = make_float4(0.f, 0.f, 0.f, pw);
        atomicOr(dev_status, SPH_DEV_OUT_OF_GRID);
        return;
    }
    cell[i] = k[0] + C.nc[0] * (k[1] + C.nc[1] * k[2]);
    pos[i] = make_float4(on[0], on[1], on[2], pw);
}


// Transpose of k_verlet for a frozen time step (state arrays at level n, ace
// the forward (a, D) of level n).  Adjoints in: x, (v, rho) of level n+1 and
// of the stored level-n copy (velrho_prev_bar); out: the adjoint of (a, D)
// and the level-n / level-(n-1) adjoints through the update.  A floored
// boundary density blocks its adjoint; excluded slots pass through unchanged.
__global__ void k_verlet_adj(StepConsts C, int32_t n, int32_t nb, int corrective,
                             const double *__restrict__ dtp, const int32_t *__restrict__ cell,
                             const float4 *__restrict__ velrho, const float4 *__restrict__ velrho_prev,
                             const float4 *__restrict__ ace, float4 *__restrict__ pos_bar,
                             float4 *__restrict__ velrho_bar, float4 *__restrict__ velrho_prev_bar,
                             float4 *__restrict__ ace_bar)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cell[i] == SPH_EXCLUDED) {
        ace_bar[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const double dt = dtp[0];
    const float4 vb1 = velrho_bar[i];
    const float4 pb1 = velrho_prev_bar[i];
    double rbar1 = vb1.w;
    if (i < nb && C.bound_floor) {
        const double D = ace[i].w;
        const double w1 = corrective ? (double)velrho[i].w + dt * D
                                     : (double)velrho_prev[i].w + 2.0 * dt * D;
        if (w1 < 0.0) rbar1 = 0.0;
    }
    const double Dbar = (corrective ? dt : 2.0 * dt) * rbar1;
    const double rb_new = corrective ? (double)pb1.w + rbar1 : (double)pb1.w;
    const double rpb_new = corrective ? 0.0 : rbar1;
    if (i < nb) {
        ace_bar[i] = make_float4(0.f, 0.f, 0.f, (float)Dbar);
        velrho_bar[i].w = (float)rb_new;
        velrho_prev_bar[i].w = (float)rpb_new;
        return;
    }
    const float4 xb1 = pos_bar[i];
    const double kv = corrective ? dt : 2.0 * dt;
    const double h2 = 0.5 * dt * dt;
    ace_bar[i] = make_float4((float)(h2 * xb1.x + kv * vb1.x), (float)(h2 * xb1.y + kv * vb1.y),
                             (float)(h2 * xb1.z + kv * vb1.z), (float)Dbar);
    const double cv = corrective ? 1.0 : 0.0;
    velrho_bar[i] = make_float4((float)(dt * xb1.x + pb1.x + cv * vb1.x),
                                (float)(dt * xb1.y + pb1.y + cv * vb1.y),
                                (float)(dt * xb1.z + pb1.z + cv * vb1.z), (float)rb_new);
    velrho_prev_bar[i] = corrective ? make_float4(0.f, 0.f, 0.f, (float)rpb_new)
                                    : make_float4(vb1.x, vb1.y, vb1.z, (float)rpb_new);
}

// Transpose of the gather of sph_build_cells: src_bar[perm[i]] = dst_bar[i].
__global__ void k_unsort(int32_t n, const int32_t *__restrict__ perm, const float4 *__restrict__ d0,
                         const float4 *__restrict__ d1, const float4 *__restrict__ d2,
                         float4 *__restrict__ s0, float4 *__restrict__ s1, float4 *__restrict__ s2)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = min(max(perm[i], 0), n - 1);
    s0[j] = d0[i];
    s1[j] = d1[i];
    s2[j] = d2[i];
}

hipError_t launch_unsort_adjoint(const int32_t *perm, int32_t n, const sph_adjoint *dst_bar,
                                 sph_adjoint *src_bar, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_unsort<<<(n + 255) / 256, 256, 0, s>>>(n, perm, (const float4 *)dst_bar->pos_bar,
                                             (const float4 *)dst_bar->velrho_bar,
                                             (const float4 *)dst_bar->velrho_prev_bar,
                                             (float4 *)src_bar->pos_bar,
                                             (float4 *)src_bar->velrho_bar,
                                             (float4 *)src_bar->velrho_prev_bar);
    return hipGetLastError();
}

hipError_t launch_step(const sph_grid *g, const sph_params *p, sph_state *st, const float *ace,
                       const float *visc, double *dt, long long step, unsigned flags,
                       sph_adjoint *adj, const Workspace &w, int32_t *dev_status, hipStream_t s)
{
    StepConsts C;
    for (int d = 0; d < 3; ++d) {
        C.org[d] = g->origin[d];
        C.hi[d] = g->hi[d];
        C.nc[d] = g->nc[d];
    }
    C.cell = g->cell;
    C.h = p->h;
    C.rho0 = p->rho0;
    C.c0 = p->c0;
    C.cfl = p->cfl;
    C.B = p->c0 * p->c0 * p->rho0 / p->gamma;
    C.verlet_ns = p->verlet_ns;
    C.bound_floor = p->bound_floor;
    const int32_t n = st->n, nb = st->nb;
    const int corrective = step == 0 || ((step + 1) % p->verlet_ns) == 0;
    if (flags & SPH_ADJOINT) {
        if (n > 0)
            k_verlet_adj<<<(n + 255) / 256, 256, 0, s>>>(
                C, n, nb, corrective, dt, st->cell, (const float4 *)st->velrho,
                (const float4 *)st->velrho_prev, (const float4 *)ace, (float4 *)adj->pos_bar,
                (float4 *)adj->velrho_bar, (float4 *)adj->velrho_prev_bar, (float4 *)adj->ace_bar);
        return hipGetLastError();
    }
    if (!(flags & SPH_FIXED_DT)) {
        int nblk = (int)(((int64_t)n + kReduceThreads - 1) / kReduceThreads);
        if (nblk > kReduceBlocksMax) nblk = kReduceBlocksMax;
        if (nblk < 1) nblk = 1;
        k_cfl_partial<<<nblk, kReduceThreads, 0, s>>>(C, n, nb, st->cell, (const float4 *)st->velrho,
                                                      (const float4 *)ace, visc, w.reduce);
        k_cfl_final<<<1, kReduceThreads, 0, s>>>(C, nblk, w.reduce, dt, dev_status);
    }
    if (n > 0)
        k_verlet<<<(n + 255) / 256, 256, 0, s>>>(C, n, nb, corrective, dt, st->cell,
                                                 (float4 *)st->pos, (float4 *)st->velrho,
                                                 (float4 *)st->velrho_prev, (const float4 *)ace,
                                                 st->pos64, dev_status);
    return hipGetLastError();
}

}  // namespace sph
