/*
 * sph_run.c -- a plain C program that drives the library through its C ABI
 * alone (no Python, no torch): it reads a particle set, runs K time steps
 * (NL -> PI -> SU, Section 2) on the default HIP device and writes the final
 * state.  It shows the calling sequence a C or C++ host uses.
 *
 * usage: sph_run <in.bin> <out.bin>
 *
 * in.bin (little endian, packed):
 *   int32   n, nb, steps
 *   double  origin[3], hi[3], cell;  int32 nc[3], nsub          (sph_grid)
 *   double  h, rho0, gamma, c0, alpha, eta2, g[3], mass, cfl;
 *   int32   kernel, verlet_ns, bound_floor;  double tensile_dp (sph_params)
 *   double  x[3n], v[3n], rho[n]              (particle i; [0, nb) boundary)
 * out.bin:
 *   double  x[3n], v[3n], rho[n]              (same particle order as in.bin)
 *   double  t                                 (sum of the time steps)
 *   int32   dev_status
 * Exit status 0 on success; any failed call prints its name and exits 1.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sph.h"

#define HIP_OK(call)                                                           \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));         \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

#define SPH_OK_(call)                                                          \
    do {                                                                       \
        sph_status s_ = (call);                                                \
        if (s_ != SPH_OK) {                                                    \
            fprintf(stderr, "%s: status %d\n", #call, (int)s_);                \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

static void get(void *dst, size_t bytes, FILE *f)
{
    if (fread(dst, 1, bytes, f) != bytes) {
        fprintf(stderr, "sph_run: input file too short\n");
        exit(1);
    }
}

static void *dev(size_t bytes)
{
    void *p = NULL;
    HIP_OK(hipMalloc(&p, bytes > 0 ? bytes : 1));
    return p;
}

static void alloc_state(sph_state *s, int32_t n, int32_t nb)
{
    s->n = n;
    s->nb = nb;
    s->cell = (int32_t *)dev(sizeof(int32_t) * (size_t)n);
    s->pos = (float *)dev(sizeof(float) * 4 * (size_t)n);
    s->velrho = (float *)dev(sizeof(float) * 4 * (size_t)n);
    s->velrho_prev = (float *)dev(sizeof(float) * 4 * (size_t)n);
    s->id = (int32_t *)dev(sizeof(int32_t) * (size_t)n);
    s->pos64 = NULL; /* positions as cell + FP32 offset only */
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: sph_run <in.bin> <out.bin>\n");
        return 2;
    }
    if (sph_abi_version() != SPH_ABI_VERSION) {
        fprintf(stderr, "sph_run: library ABI %d, header %d\n", sph_abi_version(), SPH_ABI_VERSION);
        return 1;
    }
    FILE *fi = fopen(argv[1], "rb");
    if (!fi) {
        perror(argv[1]);
        return 1;
    }
    int32_t hdr[3];
    get(hdr, sizeof hdr, fi);
    const int32_t n = hdr[0], nb = hdr[1], steps = hdr[2];
    if (n < 0 || nb < 0 || nb > n || steps < 0) {
        fprintf(stderr, "sph_run: bad header\n");
        return 1;
    }
    sph_grid g;
    memset(&g, 0, sizeof g);
    get(g.origin, sizeof g.origin, fi);
    get(g.hi, sizeof g.hi, fi);
    get(&g.cell, sizeof g.cell, fi);
    get(g.nc, sizeof g.nc, fi);
    get(&g.nsub, sizeof g.nsub, fi);
    sph_params p;
    memset(&p, 0, sizeof p);
    double pd[11];
    get(pd, sizeof pd, fi);
    p.h = pd[0];
    p.rho0 = pd[1];
    p.gamma = pd[2];
    p.c0 = pd[3];
    p.alpha = pd[4];
    p.eta2 = pd[5];
    p.g[0] = pd[6];
    p.g[1] = pd[7];
    p.g[2] = pd[8];
    p.mass = pd[9];
    p.cfl = pd[10];
    int32_t pi[3];
    get(pi, sizeof pi, fi);
    p.kernel = pi[0];
    p.verlet_ns = pi[1];
    p.bound_floor = pi[2];
    get(&p.tensile_dp, sizeof p.tensile_dp, fi);
    const size_t n3 = 3 * (size_t)n;
    double *hx = (double *)malloc(sizeof(double) * (n3 + 1));
    double *hv = (double *)malloc(sizeof(double) * (n3 + 1));
    double *hr = (double *)malloc(sizeof(double) * ((size_t)n + 1));
    int32_t *hid = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    double *ox = (double *)malloc(sizeof(double) * (n3 + 1));
    double *ov = (double *)malloc(sizeof(double) * (n3 + 1));
    double *orr = (double *)malloc(sizeof(double) * ((size_t)n + 1));
    if (!hx || !hv || !hr || !hid || !ox || !ov || !orr) {
        fprintf(stderr, "sph_run: out of host memory\n");
        return 1;
    }
    get(hx, sizeof(double) * n3, fi);
    get(hv, sizeof(double) * n3, fi);
    get(hr, sizeof(double) * (size_t)n, fi);
    fclose(fi);

    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));
    /* device memory: two state buffers, cell arrays, outputs, workspace */
    sph_state a, b;
    alloc_state(&a, n, nb);
    alloc_state(&b, n, nb);
    const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    sph_cells cells;
    cells.start = (int32_t *)dev(sizeof(int32_t) * (size_t)(2 * ncell + 2));
    cells.list = (int32_t *)dev(sizeof(int32_t) * (size_t)n);
    cells.info = (int32_t *)dev(sizeof(int32_t) * 4);
    cells.ranges = NULL;
    int32_t *perm = (int32_t *)dev(sizeof(int32_t) * (size_t)n);
    float *ace = (float *)dev(sizeof(float) * 4 * (size_t)n);
    float *visc = (float *)dev(sizeof(float) * (size_t)n);
    double *dt = (double *)dev(sizeof(double));
    double *dsum = (double *)dev(sizeof(double));
    int32_t *status = (int32_t *)dev(sizeof(int32_t));
    const size_t wsb = sph_workspace_bytes(&g, n);
    if (wsb == 0) {
        fprintf(stderr, "sph_run: invalid grid\n");
        return 1;
    }
    void *ws = dev(wsb);
    double *dx = (double *)dev(sizeof(double) * n3);
    double *dv = (double *)dev(sizeof(double) * n3);
    double *dr = (double *)dev(sizeof(double) * (size_t)n);
    HIP_OK(hipMemcpy(dx, hx, sizeof(double) * n3, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dv, hv, sizeof(double) * n3, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dr, hr, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
    HIP_OK(hipMemset(status, 0, sizeof(int32_t)));
    HIP_OK(hipMemset(dsum, 0, sizeof(double)));

    SPH_OK_(sph_encode(&g, &p, dx, dv, dr, &a, status, s));
    double t = 0.0;
    for (int32_t k = 0; k < steps; ++k) {
        SPH_OK_(sph_build_cells(&g, &a, &b, &cells, perm, ws, wsb, status, s));
        sph_state tmp = a;
        a = b;
        b = tmp;
        SPH_OK_(sph_interact(&g, &p, &a, &cells, SPH_PI_ALL, ace, visc, NULL, NULL, ws, wsb, s));
        SPH_OK_(sph_step(&g, &p, &a, ace, visc, dt, k, 0u, NULL, ws, wsb, status, s));
        double h_dt = 0.0;
        HIP_OK(hipMemcpyAsync(&h_dt, dt, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        t += h_dt;
    }
    SPH_OK_(sph_decode(&g, &p, &a, dx, dv, dr, s));
    HIP_OK(hipStreamSynchronize(s));
    int32_t hstatus = 0;
    HIP_OK(hipMemcpy(ox, dx, sizeof(double) * n3, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(ov, dv, sizeof(double) * n3, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(orr, dr, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hid, a.id, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&hstatus, status, sizeof(int32_t), hipMemcpyDeviceToHost));
    /* slot order -> input order */
    for (int32_t i = 0; i < n; ++i) {
        const int32_t q = hid[i];
        if (q < 0 || q >= n) {
            fprintf(stderr, "sph_run: bad particle id %d\n", q);
            return 1;
        }
        memcpy(hx + 3 * (size_t)q, ox + 3 * (size_t)i, 3 * sizeof(double));
        memcpy(hv + 3 * (size_t)q, ov + 3 * (size_t)i, 3 * sizeof(double));
        hr[q] = orr[i];
    }
    FILE *fo = fopen(argv[2], "wb");
    if (!fo) {
        perror(argv[2]);
        return 1;
    }
    if (fwrite(hx, sizeof(double), n3, fo) != n3 || fwrite(hv, sizeof(double), n3, fo) != n3 ||
        fwrite(hr, sizeof(double), (size_t)n, fo) != (size_t)n || fwrite(&t, sizeof t, 1, fo) != 1 ||
        fwrite(&hstatus, sizeof hstatus, 1, fo) != 1) {
        fprintf(stderr, "sph_run: write failed\n");
        return 1;
    }
    fclose(fo);
    HIP_OK(hipStreamDestroy(s));
    printf("sph_run: n=%d steps=%d t=%.9g status=%d\n", n, steps, t, hstatus);
    return 0;
}
