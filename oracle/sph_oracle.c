/*
 * sph_oracle.c -- plain, slow, FP64 CPU oracle of the WCSPH particle step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the HIP library; the two meet only
 * through the seeded input layouts and through arrays compared in the tests.
 *
 * What it computes (the method of Domínguez, Crespo & Gómez-Gesteira,
 * "Optimization strategies for parallel CPU and GPU implementations of a
 * meshfree particle method"):
 *   - Section 2: each step is neighbour list -> particle interaction ->
 *     system update.  Particles interact when closer than the kernel support
 *     (2h, the pseudocode's "< 2h" of Fig. 5 / Fig. 11); boundary-boundary
 *     pairs are never evaluated, only F-F, F-B and B-F.
 *   - Table 1 formulation: Verlet time integration, variable time step,
 *     artificial viscosity, Tait equation of state, dynamic boundaries.  The
 *     paper defers the equations to its ref. [11]; the standard forms of the
 *     cited schemes are used, each written out above the function that
 *     computes it.
 *   - Kernel: Wendland quintic (default) or the paper's cubic spline.
 *   - Optional tensile correction (the per-particle "tensil" of Table 3,
 *     following the paper's ref. [34]); off unless tensile_dp > 0.
 *
 * Summation order: the neighbours of a target are summed in ascending id
 * order, so the O(N^2) brute-force search and the cell-list search give
 * bit-identical FP64 results when they find the same neighbour sets.
 *
 * Parity status of each function is stated above it: "pinned by" names the
 * independent check in tests/ that would fail on a plausible mistake.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORA_EXPORT __attribute__((visibility("default")))

typedef struct {
    double h;          /* smoothing length; support radius is 2h               */
    double rho0;       /* reference density                                     */
    double gamma;      /* Tait exponent                                         */
    double c0;         /* reference speed of sound                              */
    double alpha;      /* artificial-viscosity coefficient                      */
    double eta2;       /* regulariser in mu_ab denominator                      */
    double g[3];       /* body acceleration on fluid particles                  */
    double mass;       /* particle mass (same for fluid and boundary)           */
    double cfl;        /* Courant factor of the variable time step              */
    int32_t kernel;    /* 0 Wendland quintic, 1 cubic spline                    */
    int32_t verlet_ns; /* a corrective Verlet step every verlet_ns steps        */
    int32_t bound_floor; /* 1: boundary density never falls below rho0          */
    int32_t pad_;
    double tensile_dp;   /* tensile correction: spacing dp of f = W(r)/W(dp); 0 off */
} ora_params;

/* ------------------------------------------------------------------------ */
/* Smoothing kernel.  Pinned by: integral of W over R^3 equals 1 (quadrature),
 * F r equals the finite-difference derivative dW/dr, lattice gradient
 * consistency, and the two-particle closed forms.                            */

static const double ORA_PI = 3.14159265358979323846;

ORA_EXPORT double ora_w(const ora_params *p, double r)
{
    const double h = p->h, q = r / h;
    if (q >= 2.0) return 0.0;
    if (p->kernel == 0) {                     /* Wendland quintic, 3-D */
        const double ad = 21.0 / (16.0 * ORA_PI * h * h * h);
        const double t = 1.0 - 0.5 * q;
        return ad * t * t * t * t * (2.0 * q + 1.0);
    }
    const double ad = 1.0 / (ORA_PI * h * h * h); /* cubic spline, 3-D */
    if (q < 1.0) return ad * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
    return 0.25 * ad * (2.0 - q) * (2.0 - q) * (2.0 - q);
}

/* F with grad_a W(|r_a - r_b|) = F * (r_a - r_b), i.e. F = (dW/dr) / r.      */
ORA_EXPORT double ora_f(const ora_params *p, double r)
{
    const double h = p->h, q = r / h;
    if (q >= 2.0) return 0.0;
    if (p->kernel == 0) {
        const double ad = 21.0 / (16.0 * ORA_PI * h * h * h);
        const double t = 1.0 - 0.5 * q;
        return -5.0 * ad * t * t * t / (h * h);
    }
    const double ad = 1.0 / (ORA_PI * h * h * h);
    if (q < 1.0) return ad * (-3.0 + 2.25 * q) / (h * h);
    if (r == 0.0) return 0.0;
    return -0.75 * ad * (2.0 - q) * (2.0 - q) / (h * h * q);
}

/* Tait equation of state and the sound speed sqrt(dP/drho).
 * Pinned by: P(rho0) = 0, c(rho0) = c0, and c^2 equal to the
 * finite-difference derivative of P.                                         */
ORA_EXPORT double ora_pressure(const ora_params *p, double rho)
{
    const double B = p->c0 * p->c0 * p->rho0 / p->gamma;
    return B * (pow(rho / p->rho0, p->gamma) - 1.0);
}

ORA_EXPORT double ora_sound(const ora_params *p, double rho)
{
    return p->c0 * pow(rho / p->rho0, 0.5 * (p->gamma - 1.0));
}

/* ------------------------------------------------------------------------ */
/* Neighbour search.  N(a) = { b != a : |x_a - x_b|^2 < (2h)^2, b not
 * excluded, and a or b is fluid }.  Ids [0, nb) are boundary particles.
 * Pinned by: brute force and cell list agree exactly on every set.          */

static inline double dist2(const double *x, int a, int b)
{
    const double rx = x[3 * a] - x[3 * b];
    const double ry = x[3 * a + 1] - x[3 * b + 1];
    const double rz = x[3 * a + 2] - x[3 * b + 2];
    return rx * rx + ry * ry + rz * rz;
}

static inline int admit(int a, int b, int nb, const uint8_t *excl, const double *x, double rc2)
{
    if (b == a || excl[b]) return 0;
    if (a < nb && b < nb) return 0;           /* no boundary-boundary pairs */
    return dist2(x, a, b) < rc2;
}

/* Brute force: every b in ascending id order. */
static int nbr_brute(int a, int n, int nb, const uint8_t *excl, const double *x, double rc2,
                     int *out)
{
    int cnt = 0;
    for (int b = 0; b < n; ++b)
        if (admit(a, b, nb, excl, x, rc2)) out[cnt++] = b;
    return cnt;
}

/* Cell list with cells of side 2h over the box of the non-excluded particles. */
typedef struct {
    double lo[3];
    double side;
    int nc[3];
    int *start;   /* [ncell+1] */
    int *ids;     /* [n] particle ids grouped by cell, ascending within a cell */
    int maxocc;
} cell_list;

static void cells_build(cell_list *cl, int n, const uint8_t *excl, const double *x, double side)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < n; ++i) {
        if (excl[i]) continue;
        for (int d = 0; d < 3; ++d) {
            if (x[3 * i + d] < lo[d]) lo[d] = x[3 * i + d];
            if (x[3 * i + d] > hi[d]) hi[d] = x[3 * i + d];
        }
    }
    cl->side = side;
    long long ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (!(hi[d] >= lo[d])) { lo[d] = 0.0; hi[d] = 0.0; }
        cl->lo[d] = lo[d];
        cl->nc[d] = (int)floor((hi[d] - lo[d]) / side) + 1;
        ncell *= cl->nc[d];
    }
    int *cof = (int *)malloc(sizeof(int) * (size_t)n);
    cl->start = (int *)calloc((size_t)ncell + 1, sizeof(int));
    cl->ids = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        if (excl[i]) { cof[i] = -1; continue; }
        int k[3];
        for (int d = 0; d < 3; ++d) {
            k[d] = (int)floor((x[3 * i + d] - cl->lo[d]) / side);
            if (k[d] >= cl->nc[d]) k[d] = cl->nc[d] - 1;
        }
        cof[i] = k[0] + cl->nc[0] * (k[1] + cl->nc[1] * k[2]);
        cl->start[cof[i] + 1]++;
    }
    cl->maxocc = 0;
    for (long long c = 0; c < ncell; ++c) {
        if (cl->start[c + 1] > cl->maxocc) cl->maxocc = cl->start[c + 1];
        cl->start[c + 1] += cl->start[c];
    }
    int *fill = (int *)calloc((size_t)ncell, sizeof(int));
    for (int i = 0; i < n; ++i)           /* ascending i keeps each cell sorted */
        if (cof[i] >= 0) cl->ids[cl->start[cof[i]] + fill[cof[i]]++] = i;
    free(fill);
    free(cof);
}

static void cells_free(cell_list *cl)
{
    free(cl->start);
    free(cl->ids);
}

static int cmp_int(const void *a, const void *b)
{
    const int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static int nbr_cells(int a, int nb, const uint8_t *excl, const double *x, double rc2,
                     const cell_list *cl, int *out)
{
    int k[3];
    for (int d = 0; d < 3; ++d) {
        k[d] = (int)floor((x[3 * a + d] - cl->lo[d]) / cl->side);
        if (k[d] >= cl->nc[d]) k[d] = cl->nc[d] - 1;
    }
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int cx = k[0] + dx, cy = k[1] + dy, cz = k[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= cl->nc[0] || cy >= cl->nc[1] ||
                    cz >= cl->nc[2])
                    continue;
                const int c = cx + cl->nc[0] * (cy + cl->nc[1] * cz);
                for (int j = cl->start[c]; j < cl->start[c + 1]; ++j)
                    if (admit(a, cl->ids[j], nb, excl, x, rc2)) out[cnt++] = cl->ids[j];
            }
    qsort(out, (size_t)cnt, sizeof(int), cmp_int);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Tensile correction (Table 3 "tensil", following the paper's ref. [34]):
 * per particle R_a = 0.01 P_a/rho_a^2 if P_a > 0, else 0.2 |P_a|/rho_a^2;
 * a pair adds T_ab = (R_a + R_b) f_ab^4, f_ab = W(r_ab)/W(dp), to the pressure
 * factor of the momentum equation.  Pinned by: the closed-form ratios at
 * r = dp (f = 1) and at W(r) = W(dp)/2 (f^4 = 1/16) for both pressure signs,
 * momentum conservation with negative pressures, and the VJP finite
 * differences with the correction on.                                       */
static double tens_r(double p_over_rho2)
{
    return p_over_rho2 > 0.0 ? 0.01 * p_over_rho2 : -0.2 * p_over_rho2;
}

/* dR/d(P/rho^2) on the side of the sign of P/rho^2 */
static double tens_eps(double p_over_rho2) { return p_over_rho2 > 0.0 ? 0.01 : -0.2; }

/* f^4 = (W(r)/W(dp))^4 */
static double tens_f4(const ora_params *p, double r)
{
    const double f = ora_w(p, r) / ora_w(p, p->tensile_dp);
    return (f * f) * (f * f);
}

/* ------------------------------------------------------------------------ */
/* Particle interaction for one target (Section 2 stage PI; Table 1 terms).
 *   grad_a W_ab      = F_ab r_ab,  r_ab = x_a - x_b
 *   continuity       drho_a/dt = sum_b m (v_a - v_b).r_ab F_ab           (any a)
 *   momentum         dv_a/dt   = g - sum_b m (P_a/rho_a^2 + P_b/rho_b^2 + Pi_ab
 *                                              [+ T_ab]) F_ab r_ab
 *   Monaghan viscosity: mu_ab = h v_ab.r_ab / (r^2 + eta2);
 *                    Pi_ab = -alpha cbar mu_ab / rhobar if v_ab.r_ab < 0, else 0
 *   visc_a           = max_b |mu_ab|   (fluid targets; used by the time step)
 * Boundary targets get only the continuity sum (B-F), with their own
 * (zero) velocity.  Pinned by: two-particle closed forms, momentum and angular
 * momentum conservation on a free blob, hydrostatic balance on a lattice,
 * rigid-motion and uniform-expansion continuity, viscous dissipation sign.    */
static void pair_sum(const ora_params *p, int a, int nb, const int *nbr, int cnt,
                     const double *x, const double *v, const double *rho, double out[5])
{
    const double m = p->mass, h = p->h;
    const double ra = rho[a];
    const double pa = ora_pressure(p, ra) / (ra * ra);
    const double ca = ora_sound(p, ra);
    const int fluid_a = a >= nb;
    double sx = 0.0, sy = 0.0, sz = 0.0, sd = 0.0, vmax = 0.0;
    for (int k = 0; k < cnt; ++k) {
        const int b = nbr[k];
        const double rx = x[3 * a] - x[3 * b];
        const double ry = x[3 * a + 1] - x[3 * b + 1];
        const double rz = x[3 * a + 2] - x[3 * b + 2];
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double F = ora_f(p, sqrt(r2));
        const double vx = v[3 * a] - v[3 * b];
        const double vy = v[3 * a + 1] - v[3 * b + 1];
        const double vz = v[3 * a + 2] - v[3 * b + 2];
        const double vdr = vx * rx + vy * ry + vz * rz;
        sd += m * vdr * F;
        if (!fluid_a) continue;
        const double rb = rho[b];
        const double pb = ora_pressure(p, rb) / (rb * rb);
        const double cb = ora_sound(p, rb);
        const double mu = h * vdr / (r2 + p->eta2);
        if (fabs(mu) > vmax) vmax = fabs(mu);
        double Pi = 0.0;
        if (vdr < 0.0) Pi = -p->alpha * (0.5 * (ca + cb)) * mu / (0.5 * (ra + rb));
        double T = 0.0;
        if (p->tensile_dp > 0.0) T = (tens_r(pa) + tens_r(pb)) * tens_f4(p, sqrt(r2));
        const double coef = m * (pa + pb + Pi + T) * F;
        sx -= coef * rx;
        sy -= coef * ry;
        sz -= coef * rz;
    }
    if (fluid_a) {
        out[0] = p->g[0] + sx;
        out[1] = p->g[1] + sy;
        out[2] = p->g[2] + sz;
    } else {
        out[0] = out[1] = out[2] = 0.0;
    }
    out[3] = sd;
    out[4] = vmax;
}

/* mode: 0 = brute force, 1 = cell list.  targets == NULL: all n particles and
 * outputs indexed by id; otherwise outputs indexed by position in targets.
 * ace = [ntarget][4] (ax, ay, az, drho/dt), visc = [ntarget].
 * Returns the number of directed interacting pairs.                          */
ORA_EXPORT long long ora_interact(int n, int nb, const double *x, const double *v,
                                  const double *rho, const uint8_t *excl, const ora_params *p,
                                  int mode, int ntarget, const int *targets, double *ace,
                                  double *visc, int32_t *nnb)
{
    const double rc2 = 4.0 * p->h * p->h;
    cell_list cl;
    memset(&cl, 0, sizeof cl);
    int cap = n;
    if (mode == 1) {
        cells_build(&cl, n, excl, x, 2.0 * p->h);
        cap = 27 * cl.maxocc + 1;
    }
    const int nt = targets ? ntarget : n;
    long long total = 0;
#pragma omp parallel reduction(+ : total)
    {
        int *buf = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
#pragma omp for schedule(dynamic, 64)
        for (int t = 0; t < nt; ++t) {
            const int a = targets ? targets[t] : t;
            double out[5] = {0, 0, 0, 0, 0};
            int cnt = 0;
            if (!excl[a]) {
                cnt = mode == 1 ? nbr_cells(a, nb, excl, x, rc2, &cl, buf)
                                : nbr_brute(a, n, nb, excl, x, rc2, buf);
                pair_sum(p, a, nb, buf, cnt, x, v, rho, out);
            }
            for (int d = 0; d < 4; ++d) ace[4 * (size_t)t + d] = out[d];
            visc[t] = out[4];
            if (nnb) nnb[t] = cnt;
            total += cnt;
        }
        free(buf);
    }
    if (mode == 1) cells_free(&cl);
    return total;
}

/* Neighbour sets as CSR (for the brute-force vs cell-list pin).  Call with
 * cols == NULL to get row counts in rowptr[1..n]; then with cols to fill.   */
ORA_EXPORT long long ora_neighbour_csr(int n, int nb, const double *x, const uint8_t *excl,
                                       double h, int mode, int64_t *rowptr, int32_t *cols)
{
    const double rc2 = 4.0 * h * h;
    cell_list cl;
    memset(&cl, 0, sizeof cl);
    int cap = n;
    if (mode == 1) {
        cells_build(&cl, n, excl, x, 2.0 * h);
        cap = 27 * cl.maxocc + 1;
    }
#pragma omp parallel
    {
        int *buf = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
#pragma omp for schedule(dynamic, 64)
        for (int a = 0; a < n; ++a) {
            int cnt = 0;
            if (!excl[a])
                cnt = mode == 1 ? nbr_cells(a, nb, excl, x, rc2, &cl, buf)
                                : nbr_brute(a, n, nb, excl, x, rc2, buf);
            if (!cols) rowptr[a + 1] = cnt;
            else memcpy(cols + rowptr[a], buf, sizeof(int32_t) * (size_t)cnt);
        }
        free(buf);
    }
    long long tot = 0;
    if (!cols) {
        rowptr[0] = 0;
        for (int a = 0; a < n; ++a) rowptr[a + 1] += rowptr[a];
        tot = rowptr[n];
    }
    if (mode == 1) cells_free(&cl);
    return tot;
}

/* ------------------------------------------------------------------------ */
/* Variable time step (Table 1, ref. [25]; Section 4.1 reduces the maxima and
 * minima of force, velocity and sound speed):
 *   dt = cfl * min( min_a sqrt(h / |dv_a/dt|), min_a h / (c_a + visc_a) )
 * over fluid, non-excluded particles.  Pinned by: closed form for isolated
 * particles.                                                                 */
ORA_EXPORT double ora_dt(int n, int nb, const double *rho, const double *ace, const double *visc,
                         const uint8_t *excl, const ora_params *p)
{
    double dtf = INFINITY, dtc = INFINITY;
    for (int a = nb; a < n; ++a) {
        if (excl[a]) continue;
        const double ax = ace[4 * (size_t)a], ay = ace[4 * (size_t)a + 1],
                     az = ace[4 * (size_t)a + 2];
        const double amag = sqrt(ax * ax + ay * ay + az * az);
        if (amag > 0.0) {
            const double t = sqrt(p->h / amag);
            if (t < dtf) dtf = t;
        }
        const double t2 = p->h / (ora_sound(p, rho[a]) + visc[a]);
        if (t2 < dtc) dtc = t2;
    }
    const double m = dtf < dtc ? dtf : dtc;
    return p->cfl * m;
}

/* ------------------------------------------------------------------------ */
/* Global sums behind the conservation laws of Section 2 (the momentum
 * equation is evaluated pair-wise, so the internal forces of fluid pairs
 * cancel; the boundary and gravity are the external forces).  Over the fluid
 * particles that are not excluded, with m the particle mass, x the position,
 * v the velocity, a the acceleration (ace, which includes gravity g) and
 * f = a - g the internal part of it:
 *   out[0..2]   sum m v                 linear momentum
 *   out[3..5]   sum m f                 internal force
 *   out[6]      sum m |v|^2 / 2         kinetic energy
 *   out[7]      -sum m g . x            gravitational potential energy
 *   out[8..10]  sum m x cross v         angular momentum about the origin
 *   out[11..13] sum m x cross f         internal torque about the origin
 *   out[14]     number of particles summed
 *   out[15]     sum m |f|               scale of the internal-force sum
 * Plain sequential sums in slot order.  ace may be NULL: then out[3..5],
 * out[11..13] and out[15] are 0.  Pinned by: closed forms for a uniform
 * translation, a rigid rotation and a resting lattice block (momentum,
 * kinetic and potential energy, angular momentum from lattice moment sums);
 * zero internal force and torque for pair-wise central forces on a free
 * blob.                                                                      */
ORA_EXPORT void ora_conservation(int n, int nb, const double *x, const double *v,
                                 const double *ace, const uint8_t *excl, const ora_params *p,
                                 double *out)
{
    for (int k = 0; k < 16; ++k) out[k] = 0.0;
    const double m = p->mass;
    for (int a = nb; a < n; ++a) {
        if (excl[a]) continue;
        const double *xa = x + 3 * (size_t)a, *va = v + 3 * (size_t)a;
        for (int d = 0; d < 3; ++d) out[d] += m * va[d];
        out[6] += 0.5 * m * (va[0] * va[0] + va[1] * va[1] + va[2] * va[2]);
        out[7] -= m * (p->g[0] * xa[0] + p->g[1] * xa[1] + p->g[2] * xa[2]);
        out[8] += m * (xa[1] * va[2] - xa[2] * va[1]);
        out[9] += m * (xa[2] * va[0] - xa[0] * va[2]);
        out[10] += m * (xa[0] * va[1] - xa[1] * va[0]);
        out[14] += 1.0;
        if (ace) {
            const double *ac = ace + 4 * (size_t)a;
            const double f[3] = {ac[0] - p->g[0], ac[1] - p->g[1], ac[2] - p->g[2]};
            for (int d = 0; d < 3; ++d) out[3 + d] += m * f[d];
            out[11] += m * (xa[1] * f[2] - xa[2] * f[1]);
            out[12] += m * (xa[2] * f[0] - xa[0] * f[2]);
            out[13] += m * (xa[0] * f[1] - xa[1] * f[0]);
            out[15] += m * sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Verlet step (Table 1, ref. [26]).  Regular step:
 *   x^{n+1} = x^n + dt v^n + dt^2/2 a^n
 *   v^{n+1} = v^{n-1} + 2 dt a^n,  rho^{n+1} = rho^{n-1} + 2 dt D^n
 * corrective step (step 0 and every verlet_ns-th step, (step+1) % ns == 0):
 *   v^{n+1} = v^n + dt a^n,       rho^{n+1} = rho^n + dt D^n.
 * Boundary particles keep x and v; their density follows the same rule and is
 * floored at rho0 when bound_floor is set.  A fluid particle that leaves the
 * domain [lo, hi) is excluded from then on.  Pinned by: exact free fall.     */
ORA_EXPORT void ora_verlet(int n, int nb, double *x, double *v, double *rho, double *vprev,
                           double *rhoprev, const double *ace, double dt, long long step,
                           const double *lo, const double *hi, uint8_t *excl,
                           const ora_params *p)
{
    const int corr = step == 0 || ((step + 1) % p->verlet_ns) == 0;
#pragma omp parallel for schedule(static)
    for (int a = 0; a < n; ++a) {
        if (excl[a]) continue;
        const double *ac = ace + 4 * (size_t)a;
        const double D = ac[3];
        const double r1 = corr ? rho[a] + dt * D : rhoprev[a] + 2.0 * dt * D;
        if (a < nb) {
            rhoprev[a] = rho[a];
            rho[a] = (p->bound_floor && r1 < p->rho0) ? p->rho0 : r1;
            continue;
        }
        int out = 0;
        for (int d = 0; d < 3; ++d) {
            const double xn = x[3 * a + d] + dt * v[3 * a + d] + 0.5 * dt * dt * ac[d];
            const double vn = corr ? v[3 * a + d] + dt * ac[d] : vprev[3 * a + d] + 2.0 * dt * ac[d];
            vprev[3 * a + d] = v[3 * a + d];
            v[3 * a + d] = vn;
            x[3 * a + d] = xn;
            if (!(xn >= lo[d] && xn < hi[d])) out = 1;
        }
        rhoprev[a] = rho[a];
        rho[a] = r1;
        if (out) excl[a] = 1;
    }
}

/* Whole steps: interact (cell list) -> dt -> Verlet, nsteps times from
 * step0.  dts receives the time step of each step.                          */
ORA_EXPORT void ora_run(int n, int nb, double *x, double *v, double *rho, double *vprev,
                        double *rhoprev, uint8_t *excl, const double *lo, const double *hi,
                        const ora_params *p, long long step0, int nsteps, double *dts)
{
    double *ace = (double *)malloc(sizeof(double) * 4 * (size_t)n);
    double *visc = (double *)malloc(sizeof(double) * (size_t)n);
    for (int s = 0; s < nsteps; ++s) {
        ora_interact(n, nb, x, v, rho, excl, p, 1, 0, NULL, ace, visc, NULL);
        const double dt = ora_dt(n, nb, rho, ace, visc, excl, p);
        if (dts) dts[s] = dt;
        ora_verlet(n, nb, x, v, rho, vprev, rhoprev, ace, dt, step0 + s, lo, hi, excl, p);
    }
    free(ace);
    free(visc);
}

/* ------------------------------------------------------------------------ */
/* Integer-cell + FP32-offset position encoding.  A position is stored as the
 * linear index k = kx + nc0 (ky + nc1 kz) of the cell of side `cell` that
 * holds it (origin `org`, X fastest) and the FP32 offset from that cell's
 * centre: d = x - org, k = floor(d / cell), o = fp32(d - (k + 1/2) cell),
 * the last difference taken as one fused multiply-add and rounded once.
 * Outside [lo, hi) the particle is excluded (cell = INT32_MAX, o = 0).
 * Decoding: x = fma(k + 1/2, cell, org) + o.                                 */
#define ORA_EXCLUDED INT32_MAX

ORA_EXPORT void ora_encode(int n, const double *x, const double *org, double cell,
                           const int32_t *nc, const double *lo, const double *hi,
                           int32_t *cellidx, float *off)
{
    for (int i = 0; i < n; ++i) {
        int ok = 1;
        long long k[3];
        float o[3];
        for (int d = 0; d < 3; ++d) {
            const double xd = x[3 * i + d];
            if (!(xd >= lo[d] && xd < hi[d])) { ok = 0; break; }
            const double dd = xd - org[d];
            const double kf = floor(dd / cell);
            if (kf < 0.0 || kf >= (double)nc[d]) { ok = 0; break; }
            k[d] = (long long)kf;
            o[d] = (float)fma(-(kf + 0.5), cell, dd);
        }
        if (!ok) {
            cellidx[i] = ORA_EXCLUDED;
            off[3 * i] = off[3 * i + 1] = off[3 * i + 2] = 0.0f;
            continue;
        }
        cellidx[i] = (int32_t)(k[0] + (long long)nc[0] * (k[1] + (long long)nc[1] * k[2]));
        for (int d = 0; d < 3; ++d) off[3 * i + d] = o[d];
    }
}

ORA_EXPORT void ora_decode(int n, const int32_t *cellidx, const float *off, const double *org,
                           double cell, const int32_t *nc, double *x)
{
    for (int i = 0; i < n; ++i) {
        if (cellidx[i] == ORA_EXCLUDED) {
            x[3 * i] = x[3 * i + 1] = x[3 * i + 2] = NAN;
            continue;
        }
        const long long c = cellidx[i];
        const long long k[3] = {c % nc[0], (c / nc[0]) % nc[1], c / ((long long)nc[0] * nc[1])};
        for (int d = 0; d < 3; ++d)
            x[3 * i + d] = fma((double)k[d] + 0.5, cell, org[d]) + (double)off[3 * i + d];
    }
}

/* ------------------------------------------------------------------------ */
/* Derivative of the kernel gradient factor: dF/dr.  Pinned by: finite
 * differences of ora_f.                                                       */
ORA_EXPORT double ora_fprime(const ora_params *p, double r)
{
    const double h = p->h, q = r / h;
    if (q >= 2.0) return 0.0;
    if (p->kernel == 0) {
        const double ad = 21.0 / (16.0 * ORA_PI * h * h * h);
        const double t = 1.0 - 0.5 * q;
        return 15.0 * ad * t * t / (2.0 * h * h * h);
    }
    const double ad = 1.0 / (ORA_PI * h * h * h);
    if (q < 1.0) return 2.25 * ad / (h * h * h);
    if (r == 0.0) return 0.0;
    return 0.75 * ad * (4.0 - q * q) / (h * h * h * q * q);
}

/* Vector-Jacobian product of ora_interact (no counterpart in the paper).
 * Given abar[4 id + 0..2] = adjoint of the acceleration of a fluid particle
 * and abar[4 id + 3] = adjoint of its density rate (any particle), add
 *   xbar += (d(A, D)/dx)^T abar,  vbar += (d/dv)^T abar,
 *   rhobar += (d/drho)^T abar,     alphabar += (d/dalpha)^T abar
 * for the same neighbour sets as the forward (cell list, ascending ids).
 * Written as the plain chain rule over every directed pair (a target, b
 * neighbour), scattered to both particles; sequential.  The visc output and
 * the time step are not differentiated; the Monaghan switch (v.r < 0) and
 * the neighbour sets are held fixed.  Pinned by: central finite differences
 * of ora_interact along random directions.                                  */
ORA_EXPORT void ora_interact_vjp(int n, int nb, const double *x, const double *v,
                                 const double *rho, const uint8_t *excl, const ora_params *p,
                                 const double *abar, double *xbar, double *vbar, double *rhobar,
                                 double *alphabar)
{
    const double rc2 = 4.0 * p->h * p->h, m = p->mass, h = p->h;
    cell_list cl;
    memset(&cl, 0, sizeof cl);
    cells_build(&cl, n, excl, x, 2.0 * p->h);
    int *buf = (int *)malloc(sizeof(int) * (size_t)(27 * cl.maxocc + 1));
    double ab = 0.0;
    for (int a = 0; a < n; ++a) {
        if (excl[a]) continue;
        const int cnt = nbr_cells(a, nb, excl, x, rc2, &cl, buf);
        const int fluid_a = a >= nb;
        const double Dbar = abar[4 * (size_t)a + 3];
        const double Ab[3] = {abar[4 * (size_t)a], abar[4 * (size_t)a + 1], abar[4 * (size_t)a + 2]};
        const double ra = rho[a];
        const double Pa = ora_pressure(p, ra), ca = ora_sound(p, ra);
        const double pa = Pa / (ra * ra);
        const double dpa = ca * ca / (ra * ra) - 2.0 * Pa / (ra * ra * ra); /* d(P/rho^2)/drho */
        const double dca = 0.5 * (p->gamma - 1.0) * ca / ra;                /* dc/drho */
        for (int k = 0; k < cnt; ++k) {
            const int b = buf[k];
            double r[3], vv[3];
            for (int d = 0; d < 3; ++d) {
                r[d] = x[3 * a + d] - x[3 * b + d];
                vv[d] = v[3 * a + d] - v[3 * b + d];
            }
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double rr = sqrt(r2);
            const double F = ora_f(p, rr);
            const double Fr = rr > 0.0 ? ora_fprime(p, rr) / rr : 0.0; /* dF/dr / r */
            const double vdr = vv[0] * r[0] + vv[1] * r[1] + vv[2] * r[2];
            double gx[3], gv[3];
            /* continuity: S = m vdr F, contributes Dbar S */
            for (int d = 0; d < 3; ++d) {
                gx[d] = Dbar * m * (F * vv[d] + vdr * Fr * r[d]);
                gv[d] = Dbar * m * F * r[d];
            }
            double gra = 0.0, grb = 0.0;
            if (fluid_a) {
                /* momentum: T = -m s F r with s = pa + pb + Pi, contributes Ab . T */
                const double rb = rho[b];
                const double Pb = ora_pressure(p, rb), cb = ora_sound(p, rb);
                const double pb = Pb / (rb * rb);
                const double dpb = cb * cb / (rb * rb) - 2.0 * Pb / (rb * rb * rb);
                const double dcb = 0.5 * (p->gamma - 1.0) * cb / rb;
                const double den = r2 + p->eta2;
                const double mu = h * vdr / den;
                const double cbar = 0.5 * (ca + cb), rbar = 0.5 * (ra + rb);
                double Pi = 0.0, dPi_dmu = 0.0, dPi_dra = 0.0, dPi_drb = 0.0, dPi_dal = 0.0;
                if (vdr < 0.0) {
                    Pi = -p->alpha * cbar * mu / rbar;
                    dPi_dmu = -p->alpha * cbar / rbar;
                    dPi_dra = -p->alpha * mu * (0.5 * dca / rbar - 0.5 * cbar / (rbar * rbar));
                    dPi_drb = -p->alpha * mu * (0.5 * dcb / rbar - 0.5 * cbar / (rbar * rbar));
                    dPi_dal = -cbar * mu / rbar;
                }
                /* tensile term: T = (R_a + R_b) f^4, dT/dx_a = (R_a + R_b) 4 f^3 f' r/|r|,
                 * f' = (dW/dr)/W(dp) = F |r| / W(dp); dT/drho = eps d(P/rho^2)/drho f^4 */
                double T = 0.0, dT_dr = 0.0, dT_dra = 0.0, dT_drb = 0.0;
                if (p->tensile_dp > 0.0) {
                    const double wdp = ora_w(p, p->tensile_dp);
                    const double f = ora_w(p, rr) / wdp;
                    const double Rab = tens_r(pa) + tens_r(pb);
                    T = Rab * f * f * f * f;
                    dT_dr = Rab * 4.0 * f * f * f * F / wdp; /* times r[d] */
                    dT_dra = tens_eps(pa) * dpa * f * f * f * f;
                    dT_drb = tens_eps(pb) * dpb * f * f * f * f;
                }
                const double s = pa + pb + Pi + T;
                const double Q = Ab[0] * r[0] + Ab[1] * r[1] + Ab[2] * r[2];
                for (int d = 0; d < 3; ++d) {
                    const double dmu_dr = h * vv[d] / den - 2.0 * mu * r[d] / den;
                    const double dmu_dv = h * r[d] / den;
                    gx[d] += -m * (F * Q * (dPi_dmu * dmu_dr + dT_dr * r[d]) + s * Q * Fr * r[d] +
                                   s * F * Ab[d]);
                    gv[d] += -m * F * Q * dPi_dmu * dmu_dv;
                }
                gra = -m * F * Q * (dpa + dPi_dra + dT_dra);
                grb = -m * F * Q * (dpb + dPi_drb + dT_drb);
                ab += -m * F * Q * dPi_dal;
            }
            for (int d = 0; d < 3; ++d) {
                xbar[3 * a + d] += gx[d];
                xbar[3 * b + d] -= gx[d];
                vbar[3 * a + d] += gv[d];
                vbar[3 * b + d] -= gv[d];
            }
            rhobar[a] += gra;
            rhobar[b] += grb;
        }
    }
    *alphabar += ab;
    free(buf);
    cells_free(&cl);
}

/* Transpose of ora_verlet for a frozen time step dt (the state arrays are
 * those of level n, before the update; ace is the forward (A, D) of level n).
 * In:  xb, vb, rb  = adjoints of x, v, rho at level n+1,
 *      vpb, rpb    = adjoints of the level-(n+1) copies of v^n, rho^n.
 * Out: abar[4 id + 0..3] = adjoints of (A, D)^n (overwritten);
 *      xb, vb, rb  = adjoints of level n through the update only,
 *      vpb, rpb    = adjoints of v^{n-1}, rho^{n-1}.
 * Boundary particles: x and v fixed (their x, v adjoints are left as they
 * are); a floored boundary density blocks its adjoint.  Excluded particles
 * are left unchanged with zero abar.  Pinned by: rollout gradients against
 * central finite differences.                                               */
ORA_EXPORT void ora_verlet_vjp(int n, int nb, const double *rho, const double *rhoprev,
                               const double *ace, double dt, long long step, const uint8_t *excl,
                               const ora_params *p, double *xb, double *vb, double *rb,
                               double *vpb, double *rpb, double *abar)
{
    const int corr = step == 0 || ((step + 1) % p->verlet_ns) == 0;
    for (int a = 0; a < n; ++a) {
        double *ab4 = abar + 4 * (size_t)a;
        ab4[0] = ab4[1] = ab4[2] = ab4[3] = 0.0;
        if (excl[a]) continue;
        const double D = ace[4 * (size_t)a + 3];
        double rbar1 = rb[a];
        if (a < nb && p->bound_floor) {
            const double r1 = corr ? rho[a] + dt * D : rhoprev[a] + 2.0 * dt * D;
            if (r1 < p->rho0) rbar1 = 0.0;
        }
        if (corr) {
            ab4[3] = dt * rbar1;
            rb[a] = rpb[a] + rbar1;
            rpb[a] = 0.0;
        } else {
            ab4[3] = 2.0 * dt * rbar1;
            rb[a] = rpb[a];
            rpb[a] = rbar1;
        }
        if (a < nb) continue;
        for (int d = 0; d < 3; ++d) {
            const double xb1 = xb[3 * a + d], vb1 = vb[3 * a + d];
            ab4[d] = 0.5 * dt * dt * xb1 + (corr ? dt : 2.0 * dt) * vb1;
            vb[3 * a + d] = dt * xb1 + vpb[3 * a + d] + (corr ? vb1 : 0.0);
            vpb[3 * a + d] = corr ? 0.0 : vb1;
            /* xb unchanged: x^{n+1} depends on x^n with unit weight */
        }
    }
}

ORA_EXPORT int ora_num_threads(void)
{
    return omp_get_max_threads();
}
