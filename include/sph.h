/*
 * sph.h -- C ABI of the MI355X (gfx950) WCSPH particle-interaction library.
 *
 * The library implements one time step of the weakly compressible SPH method
 * of Domínguez, Crespo & Gómez-Gesteira, "Optimization strategies for parallel
 * CPU and GPU implementations of a meshfree particle method" (Section 2: each
 * step is NL -> PI -> SU), as hand-written HIP kernels:
 *
 *   sph_build_cells        NL: cell key, stable radix sort, cell ranges,
 *                          reorder of the particle arrays (Section 4.1).
 *   sph_interact           PI: F-F + F-B interactions of fluid targets and
 *                          B-F interactions of boundary targets (Sections 2,
 *                          4.3-4.5; Table 1 formulation).
 *   sph_step               SU: variable time step from global maxima and the
 *                          Verlet update (Section 4.1, Table 1).
 *   sph_interact_backward  vector-Jacobian product of sph_interact (no
 *                          counterpart in the paper).
 *   sph_step(SPH_ADJOINT)  transpose of the Verlet update;
 *   sph_build_cells_backward  transpose of the reorder of sph_build_cells.
 *   sph_encode/sph_decode  FP64 <-> device state conversion.
 *   sph_conservation       FP64 global sums of the conservation laws
 *                          (momentum, energy, internal force) on the device.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller; struct
 *     arguments (sph_grid, sph_params, sph_state, sph_cells) are host structs
 *     whose array members are device pointers.  The library allocates no
 *     memory and keeps no global state; it is re-entrant.  (One exception,
 *     for callers that cannot allocate: sph_build_cells_static works in a
 *     static scratch array that each device holds, see there.)
 *   - Work is enqueued on `stream` and the call returns without
 *     synchronising.  Host-side validation returns a status immediately and
 *     enqueues nothing on failure.  Conditions found on the device are OR-ed
 *     into the caller-owned bitmask *dev_status (read it after a sync).
 *   - `ws`/`ws_bytes`: one caller-owned device workspace of at least
 *     sph_workspace_bytes(grid, n) bytes, shared by all calls of a simulation.
 *     Calls that share a workspace must be ordered on one stream.
 *   - Sorted-state layout: boundary particles occupy slots [0, nb) and fluid
 *     particles [nb, n); excluded particles (outside the domain) are the last
 *     slots of the fluid range.
 *
 * Positions are an integer cell plus an FP32 offset from the cell centre:
 *   x = origin + (k + 1/2) * cell + offset  (per axis), |offset| <= cell/2,
 * so relative distances keep FP32 accuracy in large domains.  Pair
 * arithmetic is FP32 with FP32 accumulation; the position update and the
 * time-step reduction are FP64.
 */
#ifndef SPH_H_
#define SPH_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 8 /* 2: two-entry npairs; 3: sph_params.tensile_dp; 4: sph_cells.ranges;
                            5: SPH_DEV_BOUNDARY_OUT; 6: sph_conservation;
                            7: sph_state.pos64, sph_params.pos_policy;
                            8: sph_build_cells_static */
#define SPH_API __attribute__((visibility("default")))
#define SPH_EXCLUDED INT32_MAX /* cell index of a particle outside the domain */

typedef enum {
    SPH_OK = 0,
    SPH_ERR_ARG = 1,       /* invalid argument (null pointer, bad size, bad grid) */
    SPH_ERR_WORKSPACE = 2, /* ws_bytes smaller than sph_workspace_bytes()        */
    SPH_ERR_HIP = 3        /* a kernel launch failed (hipGetLastError)            */
} sph_status;

/* bits OR-ed into *dev_status by the kernels */
enum {
    SPH_DEV_OUT_OF_GRID = 1, /* a particle left the domain and is now excluded */
    SPH_DEV_NONFINITE = 2,   /* non-finite acceleration/time step; state kept  */
    SPH_DEV_BOUNDARY_OUT = 4 /* INVALID STATE: a boundary slot [0, nb) holds a particle
                                outside the domain (cell SPH_EXCLUDED).  Boundary particles
                                never move, so this can only come from the input; the
                                sorted layout (boundary slots first) cannot hold it and
                                every later output is meaningless.  Refuse such input. */
};

/* Cell grid of the neighbour list (Section 2: domain divided into cells so the
 * search covers the own and adjacent cells; Section 3.2: cells of side
 * support/n; Section 4.4: cells ordered X fastest, then Y, then Z).
 * The stencil is (2*nsub+1)^3 cells, read as (2*nsub+1)^2 X-runs. */
typedef struct {
    double origin[3]; /* lower corner of cell (0,0,0) = lower corner of the domain  */
    double hi[3];     /* upper corner of the domain; outside [origin, hi) = excluded */
    double cell;      /* cell side; requires nsub * cell >= 2h (1 + 2^-21)           */
    int32_t nc[3];    /* cells per axis; ncell = nc0*nc1*nc2 < 2^30 - 1             */
    int32_t nsub;     /* 1 (cell = support 2h) or 2 (cell = h)                       */
} sph_grid;

/* Smoothing kernels (Section 2: both have compact support q = r/h < 2).
 *   SPH_WENDLAND5:    W = aD (1 - q/2)^4 (2q + 1),            aD = 21 / (16 pi h^3)
 *   SPH_CUBIC_SPLINE: W = aD (1 - 3q^2/2 + 3q^3/4) for q < 1,
 *                     W = aD (2 - q)^3 / 4 for 1 <= q < 2,     aD = 1 / (pi h^3)
 *                     (the Table 1 kernel). */
#define SPH_WENDLAND5 0
#define SPH_CUBIC_SPLINE 1

/* Physical constants (Table 1: Verlet, variable time step, Monaghan artificial
 * viscosity, Tait equation of state, dynamic boundaries). */
typedef struct {
    double h;        /* smoothing length; kernel support is 2h                   */
    double rho0;     /* reference density                                        */
    double gamma;    /* Tait exponent; must be 7                                 */
    double c0;       /* reference sound speed; Tait B = c0^2 rho0 / gamma        */
    double alpha;    /* artificial-viscosity coefficient                         */
    double eta2;     /* regulariser of mu_ab = h v.r / (r^2 + eta2)              */
    double g[3];     /* gravity, applied to fluid particles                      */
    double mass;     /* particle mass (fluid and boundary)                       */
    double cfl;      /* Courant factor of the variable time step                 */
    int32_t kernel;  /* SPH_WENDLAND5 or SPH_CUBIC_SPLINE                        */
    int32_t verlet_ns;   /* corrective Verlet step every verlet_ns steps (>= 1)  */
    int32_t bound_floor; /* 1: boundary density floored at rho0 after each step  */
    int32_t pos_policy;  /* position load of sph_interact: SPH_POS_OFFSET32 (0) or
                          * SPH_POS_ABS64, see below                              */
    double tensile_dp;   /* tensile correction (Table 3 "tensil", ref. [34]): 0 = off;
                          * > 0: the particle spacing dp, 0 < dp < 2h.  A pair then
                          * adds (R_a + R_b) f^4, f = W(r)/W(dp), to the pressure
                          * factor of the momentum equation, with R = 0.01 P/rho^2
                          * for P > 0 and 0.2 |P|/rho^2 for P < 0.                 */
} sph_params;

/* Position-load policies of the pair kernel (sph_params.pos_policy).
 *   SPH_POS_OFFSET32: r_ab from the FP32 offsets in the frame of the target's
 *     cell: o_a - (o_b + (k_b - k_a) cell), the shift exact, the sum rounded
 *     once (the default, and the only policy of the adjoint).
 *   SPH_POS_ABS64: r_ab = fp32(x_a - x_b) from FP64 absolute positions (the
 *     state's pos64, relative to the target cell's centre in FP64); all other
 *     pair arithmetic is the same FP32.  A measurement variant of the forward
 *     pair kernel with the Wendland kernel: sph_interact refuses it
 *     (SPH_ERR_ARG) with nbr_stats, the cubic spline, the tensile correction
 *     or a state without pos64, and sph_interact_backward refuses it. */
#define SPH_POS_OFFSET32 0
#define SPH_POS_ABS64 1

/* Particle state (structure of arrays); one instance per side of a double
 * buffer.  All members are device arrays of length n (x4 where noted). */
typedef struct {
    int32_t n;            /* particles                                              */
    int32_t nb;           /* boundary particles (slots [0, nb))                     */
    int32_t *cell;        /* [n] linear cell index kx + nc0 (ky + nc1 kz), or SPH_EXCLUDED */
    float *pos;           /* [4n] (ox, oy, oz, P/rho^2): offset from the cell centre */
    float *velrho;        /* [4n] (vx, vy, vz, rho - rho0) at level n               */
    float *velrho_prev;   /* [4n] the same at level n-1 (Verlet)                     */
    int32_t *id;          /* [n] original particle id                               */
    double *pos64;        /* optional [3n] FP64 absolute positions, or NULL.  When set:
                             sph_encode writes x, sph_build_cells gathers it (src and dst
                             both set, or both NULL), sph_step updates it in FP64 and
                             re-bins (cell, offset) from it, sph_decode returns it;
                             needed by SPH_POS_ABS64                                  */
} sph_state;

/* Output of the neighbour list (CellBeginEnd of Section 4.1, stored as one
 * prefix array).  Keys: boundary cell k -> k, fluid cell k -> ncell + k,
 * excluded -> 2 ncell.
 *
 * ranges (optional, NULL = not used): the interaction ranges of every cell
 * precomputed by sph_build_cells (Section 4.4, optimisation D: the 27 cells,
 * 125 with nsub = 2, of a stencil read as (2 nsub + 1)^2 X-runs of
 * consecutive cells, each one range of sorted slots).  Layout: int32
 * [ncell][2][(2 nsub + 1)^2][2]: for cell c, particle type t (0 boundary,
 * 1 fluid) and run r = (dy + nsub) + (2 nsub + 1)(dz + nsub), the pair
 * (first slot, end slot) of the type-t particles in the cells
 * (max(cx - nsub, 0) .. min(cx + nsub, nc0 - 1), cy + dy, cz + dz); (0, 0)
 * for a run outside the grid.  144 bytes per cell with nsub = 1, 400 with
 * nsub = 2: sph_ranges_bytes().  sph_build_cells writes the rows of the cells
 * that hold particles (other rows are left as they are); sph_interact and
 * sph_interact_backward then read each target cell's runs from its row
 * instead of deriving them from start[], with bitwise identical results. */
typedef struct {
    int32_t *start;  /* [2*ncell + 2]: start[key] = first sorted slot with that key or a
                        larger one; particles of key k are [start[k], start[k+1])         */
    int32_t *list;   /* [n] non-empty keys in ascending order (boundary cells first)      */
    int32_t *info;   /* [4] (device): non-empty boundary cells, non-empty fluid cells,
                        excluded particles, reserved                                     */
    int32_t *ranges; /* optional [sph_ranges_bytes(g) / 4], see above; NULL: not used    */
} sph_cells;

/* Adjoint buffers (device, [4n] each, in the slot order of one state).  The
 * time step and the neighbour sets are held fixed; the Monaghan switch
 * (v.r < 0) and the boundary density floor act as masks. */
typedef struct {
    float *pos_bar;         /* adjoint of x (xyz; w unused); boundary slots unused        */
    float *velrho_bar;      /* adjoint of (v, rho) of the current level                   */
    float *velrho_prev_bar; /* adjoint of (v, rho) stored as the previous level           */
    float *ace_bar;         /* adjoint of (a, drho/dt) of one step (written by sph_step)  */
} sph_adjoint;

/* Size in bytes of the workspace needed by all calls for n particles on
 * grid g; 0 if the arguments are invalid. */
SPH_API size_t sph_workspace_bytes(const sph_grid *g, int32_t n);

/* Size in bytes of the optional interaction-range table of grid g
 * (sph_cells.ranges): ncell * 2 * (2 nsub + 1)^2 * 8; 0 if g is invalid. */
SPH_API size_t sph_ranges_bytes(const sph_grid *g);

/* ABI version of the loaded library (SPH_ABI_VERSION). */
SPH_API int32_t sph_abi_version(void);

/* Fill a state from FP64 host-order arrays already on the device (x [3n],
 * v [3n], rho [n]; ids [0, nb) are boundary particles).  Position encoding:
 * d = x - origin, k = floor(d / cell), offset = fp32(fma(-(k + 1/2), cell, d));
 * a particle outside [origin, hi) gets cell SPH_EXCLUDED and sets
 * SPH_DEV_OUT_OF_GRID, and also SPH_DEV_BOUNDARY_OUT if it is a boundary
 * particle (an invalid input: the caller must not use the state).
 * velrho_prev = velrho, pos.w = P/rho^2, id = index. */
SPH_API sph_status sph_encode(const sph_grid *g, const sph_params *p, const double *x,
                      const double *v, const double *rho, sph_state *st, int32_t *dev_status,
                      hipStream_t stream);

/* Decode a state to FP64 arrays in slot order: x = fma(k + 1/2, cell, origin)
 * + offset, v, rho = rho0 + (rho - rho0); NaN positions for excluded slots. */
SPH_API sph_status sph_decode(const sph_grid *g, const sph_params *p, const sph_state *st, double *x,
                      double *v, double *rho, hipStream_t stream);

/* NL (Section 4.1): key = (slot < nb ? 0 : ncell) + cell, or 2 ncell when
 * excluded (a boundary slot with cell SPH_EXCLUDED sets SPH_DEV_BOUNDARY_OUT:
 * invalid input, outputs meaningless but every access stays in bounds);
 * stable LSD radix sort of (key, slot), ties keeping the src order;
 * cell ranges and the list of non-empty keys; gather of every state array
 * into dst in sorted order.  perm[i] = src slot of dst slot i.  src and dst
 * must not overlap.  dst->n and dst->nb are set from src. */
SPH_API sph_status sph_build_cells(const sph_grid *g, const sph_state *src, sph_state *dst,
                           sph_cells *cells, int32_t *perm, void *ws, size_t ws_bytes,
                           int32_t *dev_status, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as sph_build_cells, same kernels and bitwise the same outputs,
 * with the library's own scratch in place of the caller's workspace.  The
 * scratch is one static device array of SPH_STATIC_SCRATCH_BYTES (64 MiB) per
 * device, held from the library's load until the process ends; its device
 * address is looked up on the first call on each device.  The call allocates
 * nothing.  Errors: SPH_ERR_ARG as sph_build_cells; SPH_ERR_WORKSPACE (before
 * any device call) when sph_workspace_bytes(g, src->n) exceeds the scratch,
 * e.g. beyond about 2.1M particles on a 475,300-cell grid; SPH_ERR_HIP if the
 * scratch address cannot be obtained or a launch fails.  All calls on one
 * device share its scratch and every call rewrites what it reads: calls that
 * overlap in time on one device (two streams, two threads) race and must be
 * ordered by the caller, e.g. on one stream.  Calls on different devices are
 * independent. */
#define SPH_STATIC_SCRATCH_BYTES (64u << 20)
SPH_API sph_status sph_build_cells_static(const sph_grid *g, const sph_state *src,
                                          sph_state *dst, sph_cells *cells, int32_t *perm,
                                          int32_t *dev_status, hipStream_t stream);

/* PI (Section 2 interaction classes F-F, F-B, B-F; never B-B).  For a fluid
 * target a and every b != a within the support (r_ab^2 < 4 h^2, decided in
 * FP32 from the encoded positions):
 *   ace[a].xyz = g - m sum_b (P_a/rho_a^2 + P_b/rho_b^2 + Pi_ab) F_ab r_ab
 *   ace[a].w   = m sum_b (v_a - v_b).r_ab F_ab              (drho/dt)
 *   visc[a]    = max_b |mu_ab|
 * with grad_a W_ab = F_ab r_ab (the kernel p->kernel), mu_ab = h v_ab.r_ab /
 * (r^2 + eta2), Pi_ab = -alpha cbar mu_ab / rhobar when v_ab.r_ab < 0 else 0,
 * Tait P = B((rho/rho0)^7 - 1), c = c0 (rho/rho0)^3.  Boundary targets get
 * (0, 0, 0, drho/dt) over fluid neighbours and visc 0; excluded slots get 0.
 * parts: SPH_PI_FLUID and/or SPH_PI_BOUNDARY.  SPH_PI_ALL (a full stage)
 * enqueues a counter reset, the boundary-cell filter and ONE pair kernel that
 * takes the fluid target cells and then the boundary cells with fluid in
 * reach; a single part enqueues that part's own pair kernel.
 * npairs (may be NULL): [2] u64, npairs[0] += directed interacting pairs with
 * a fluid target, npairs[1] += those with a boundary target.
 * nbr_stats (may be NULL, diagnostic, slower): [2n] per slot (neighbour
 * count, sum over neighbours of uint32(id * 2654435761)). */
#define SPH_PI_FLUID 1u    /* fluid targets: F-F + F-B (Section 4.5 fused kernel) */
#define SPH_PI_BOUNDARY 2u /* boundary targets: B-F, plus zeroing of excluded slots */
#define SPH_PI_ALL 3u
SPH_API sph_status sph_interact(const sph_grid *g, const sph_params *p, const sph_state *st,
                        const sph_cells *cells, unsigned parts, float *ace, float *visc,
                        unsigned long long *npairs, int32_t *nbr_stats, void *ws,
                        size_t ws_bytes, hipStream_t stream);

#define SPH_FIXED_DT 1u /* use *dt as given instead of the CFL time step      */
#define SPH_ADJOINT 2u  /* run the transpose of the Verlet map (needs adj)    */

/* SU (Section 4.1, Table 1).  Time step (FP64 reduction over fluid slots):
 *   dt = cfl * min( sqrt(h / max|a|), h / max(c + visc) ),
 * written to dt[0] (device) unless SPH_FIXED_DT.  Verlet: regular step
 *   x += dt v + dt^2/2 a,  (v, rho)^{n+1} = (v, rho)^{n-1} + 2 dt (a, D),
 * corrective step when step == 0 or (step + 1) % verlet_ns == 0:
 *   (v, rho)^{n+1} = (v, rho)^n + dt (a, D);
 * the position update is FP64 and re-bins (cell, offset).  Boundary slots
 * keep position and velocity; their density follows the same rule and is
 * floored at rho0 if bound_floor.  Unless SPH_FIXED_DT, a non-finite value
 * in ace or visc (any slot) or a non-finite time step (also: no fluid slot,
 * hence no limit on dt) sets SPH_DEV_NONFINITE, writes NaN to dt[0] and
 * leaves the state unchanged.
 * Adjoint mode (flags SPH_ADJOINT, adj != NULL): st, ace and dt[0] are the
 * state, (a, D) and time step of the forward step being transposed (st before
 * its update).  In: adj->pos_bar, velrho_bar, velrho_prev_bar = adjoints of
 * level n+1.  Out: adj->ace_bar = adjoint of (a, D)^n:
 *   regular:    abar = dt^2/2 xbar' + 2 dt vbar',  Dbar = 2 dt rhobar',
 *   corrective: abar = dt^2/2 xbar' + dt vbar',    Dbar = dt rhobar',
 * and the three adjoint arrays replaced by those of level n (through the
 * update only; add the interaction's VJP with sph_interact_backward):
 *   xbar = xbar',  vbar = dt xbar' + vprevbar' (+ vbar' if corrective),
 *   rhobar = rhoprevbar' (+ rhobar' if corrective),
 *   (vprevbar, rhoprevbar) = regular ? (vbar', rhobar') : 0.
 * Boundary slots: only the density entries; excluded slots unchanged. */
SPH_API sph_status sph_step(const sph_grid *g, const sph_params *p, sph_state *st, const float *ace,
                    const float *visc, double *dt, long long step, unsigned flags,
                    sph_adjoint *adj, void *ws, size_t ws_bytes, int32_t *dev_status,
                    hipStream_t stream);

/* VJP of sph_interact at state st with the cells of the same build:
 * ace_bar [4n] = (abar, Dbar) per slot (abar of boundary slots is ignored).
 * Accumulates (+=), each slot written by exactly one thread:
 *   pos_bar[i].xyz    += (d(a, D)/dx_i)^T ace_bar      (fluid slots)
 *   velrho_bar[i].xyz += (d(a, D)/dv_i)^T ace_bar      (fluid slots)
 *   velrho_bar[i].w   += (d(a, D)/drho_i)^T ace_bar    (all slots)
 *   alpha_bar[0]      += (d a/d alpha)^T abar          (FP64, fixed-order sum)
 * Gather form: for each particle, over its neighbours b, the derivative of the
 * pair term (abar_a - abar_b) . T_ab + (Dbar_a + Dbar_b) S_ab, where
 * T_ab = -m (P_a/rho_a^2 + P_b/rho_b^2 + Pi_ab) F_ab r_ab and
 * S_ab = m (v_ab . r_ab) F_ab are the momentum and continuity pair terms. */
SPH_API sph_status sph_interact_backward(const sph_grid *g, const sph_params *p, const sph_state *st,
                                 const sph_cells *cells, const float *ace_bar, float *pos_bar,
                                 float *velrho_bar, double *alpha_bar, void *ws,
                                 size_t ws_bytes, hipStream_t stream);

/* Global sums of the conservation laws (Section 2: the momentum equation is
 * evaluated pair-wise, so the internal forces of fluid pairs cancel; gravity
 * and the boundary particles act from outside).  FP64 sums over the fluid
 * slots [nb, n) whose cell is not SPH_EXCLUDED, with m the particle mass,
 * x = fma(k + 1/2, cell, origin) + offset the decoded position, v the velocity
 * of level n (velrho) and f = ace.xyz - g the internal acceleration:
 *   out[0..2]   sum m v            linear momentum
 *   out[3..5]   sum m f            internal force (0 for a free fluid body)
 *   out[6]      sum m |v|^2 / 2    kinetic energy
 *   out[7]      -sum m g . x       gravitational potential energy
 *   out[8..10]  sum m x cross v    angular momentum about the origin
 *   out[11..13] sum m x cross f    internal torque about the origin
 *   out[14]     number of slots summed
 *   out[15]     sum m |f|          scale of the internal-force sum
 * out: [16] doubles (device).  ace: the output of sph_interact on this same
 * state (so call it between sph_interact and sph_step), or NULL: then
 * out[3..5], out[11..13] and out[15] are 0.  The sums run in a fixed order
 * (block partials, then one block): bitwise reproducible for a given state.
 * The call uses the workspace's reduction area, like sph_step: order it with
 * the other calls sharing the workspace on one stream. */
#define SPH_CONSERVATION_SUMS 16
SPH_API sph_status sph_conservation(const sph_grid *g, const sph_params *p, const sph_state *st,
                                    const float *ace, double *out, void *ws, size_t ws_bytes,
                                    hipStream_t stream);

/* Transpose of the reorder of sph_build_cells: src_bar[perm[i]] = dst_bar[i]
 * for pos_bar, velrho_bar and velrho_prev_bar (ace_bar is not used).  perm
 * is the array that sph_build_cells wrote; the two adjoint sets must not
 * share arrays. */
SPH_API sph_status sph_build_cells_backward(const int32_t *perm, int32_t n,
                                            const sph_adjoint *dst_bar, sph_adjoint *src_bar,
                                            hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H_ */
