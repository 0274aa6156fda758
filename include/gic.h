/*
 * gic.h -- C ABI of the Granule-In-Cell granule hot path for AMD MI355X
 * (gfx950).
 *
 * Paper: Tang, Zhu, Ni, Chen, "The Granule-In-Cell Method for Simulating
 * Sand-Water Mixtures", ACM TOG 44(6) 2025 (arXiv 2504.00745).
 *
 * One call of each stage below, in the order
 *     gic_sort_cells -> gic_reorder -> gic_g2p -> gic_drag ->
 *     gic_contact_forces -> gic_integrate -> gic_p2g
 * is one sand sub-step of Alg. 2 (SandSubstep): coupling force from the grid
 * (Sec. 5.2), collision handling (Sec. 3.1, Eq. 1), move (Sec. 4, symplectic
 * ordering), and the transfer of the granules' volume fraction (Sec. 5.1,
 * Eq. 7a) and momentum to the grid.  gic_step runs the same sub-step through
 * the same kernels in one call.
 *
 * Shape of the interface
 *   - Sorting and reordering are separate calls: gic_sort_cells returns
 *     keys, the stable order and the cell ranges; gic_reorder gathers the
 *     granule arrays into that order.  The stepping calls (gic_step,
 *     gic_sand_step) fuse the reorder into the gather that samples the
 *     grid (gic_gather_g2p_drag / _fluid) and the move into the P2G
 *     (gic_integrate_p2g).
 *   - gic_contact_forces returns the touching pairs of its own kernel as a
 *     fixed number of entries per granule (pair_ids, column-major, -1
 *     after the last), not a compressed list.
 *   - gic_get_error returns the latched code and granule index separately
 *     and can clear them.
 *   - gic_integrate_vjp takes the cotangents of x' and v' and returns the
 *     cotangent of the force and the updated cotangent of v in place.
 *   - Every output that depends on an order of floating-point additions
 *     (force sums, the unquantised transfers, parameter gradients) is
 *     computed in an order fixed by the sorted state, so repeated calls on
 *     the same inputs give the same bits.
 *
 * Conventions
 *   Memory.   Every array argument is a DEVICE pointer owned by the caller.
 *             The library never frees or keeps it beyond the work the call
 *             enqueues (gic_step and gic_sand_step remember the addresses of
 *             the grids their last call wrote, only to compare them with the
 *             next call's).  The context owns only its scratch (sort
 *             buffers, tiles, error word), allocated by gic_create for n_max
 *             granules; no stage call allocates.
 *   Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *             stream).  Stage calls only enqueue work on it and never
 *             synchronise; gic_get_error and gic_destroy do.
 *   Layout.   Per-granule 3-vectors are structure of arrays: a[0..n) holds x
 *             components, a[n..2n) y, a[2n..3n) z.  Grid fields are
 *             x-fastest: node (i,j,k) at i + nx (j + ny k), node centre at
 *             ((i+1/2) dx, (j+1/2) dx, (k+1/2) dx); a 3-vector grid field is
 *             three consecutive G-node planes (G = nx ny nz).  The box is
 *             [0, n_a dx) per axis.
 *   Types.    Positions, velocities and radii are always double.  "real"
 *             arrays (forces, fluid velocity, sampled velocity and fraction)
 *             are float in the FP32 form (precision GIC_FP32) and double in
 *             the plain form (GIC_FP64).  Fixed-point grids are int64.
 *   Sorted order.  gic_contact_forces and gic_p2g take granules in the order
 *             produced by gic_reorder from the `order` of gic_sort_cells on
 *             those same positions, with the cell tables of that sort.
 *             Granules that moved after the sort (gic_p2g after
 *             gic_integrate) are still handled exactly; only speed depends on
 *             the order.
 *   Errors.   Calls return gic_status and never print, throw or abort.
 *             Argument errors (NULL, n < 0 or n > n_max, bad parameters) are
 *             detected on the host and return GIC_E_ARG before anything is
 *             enqueued.  A failed launch returns GIC_E_HIP.  Conditions found
 *             by the kernels (a non-finite position or velocity, a granule
 *             centre outside the box, a radius above r_max, a fixed-point
 *             value out of range) latch the first code and granule index in
 *             the context; gic_get_error reads them.
 *   Threads.  A context is used by one host thread and one stream at a time.
 */
#ifndef GIC_H
#define GIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GIC_OK = 0,
    GIC_E_ARG = 1,       /* invalid argument, nothing enqueued            */
    GIC_E_HIP = 2,       /* HIP runtime or launch failure                 */
    GIC_E_ALLOC = 3,     /* device allocation failed in gic_create        */
    GIC_E_DOMAIN = 4,    /* latched: granule centre outside the box       */
    GIC_E_NONFINITE = 5, /* latched: non-finite position or velocity      */
    GIC_E_RANGE = 6      /* latched: radius > r_max, a fixed-point
                            contribution of magnitude >= 2^51 units, or
                            cell ranges / sorted order that do not match
                            the positions (ranges and order indices are
                            clipped to [0, n) before any access); in the
                            density projection a cell label outside 0..2
                            or alpha_f' not in (0, inf) on a fluid or air
                            cell (index = the cell)                      */
} gic_status;

typedef enum { GIC_FP64 = 0, GIC_FP32 = 1 } gic_precision;

/* Parameters of the granule step.
 *   n[3], dx      grid nodes per axis (1 .. 32767) and spacing [m]; nodes at cell centres
 *                 (Sec. 5.1: the solid fractions live at the cell centres).
 *   nc[3], cell   neighbour-search cells per axis and their edge [m];
 *                 cell >= 2 r_max and nc[a] cell <= n[a] dx; the last cell
 *                 of an axis extends to the box face.
 *   kn            normal stiffness k_n of Eq. (1a) [N/m].
 *   restitution   e in (0,1]: the normal dashpot gamma_n = 2 zeta
 *                 sqrt(m_eff k_n), zeta = -ln e / sqrt(pi^2 + ln^2 e).
 *   kt_ratio      k_t of Eq. (1c) = kt_ratio * gamma_n [N s/m].
 *   mu            tan(phi) of Eq. (1b); the cap is mu k_n delta.
 *   rho_s         granule density [kg/m^3] (Sec. 6: 2.5e3).
 *   eta_f, c_drag drag F_d = c_drag 6 pi eta_f r alpha_f (u - v) (Eq. 5b,
 *                 App. A relaxation drag in Stokes form).
 *   alpha_max     node clamp of alpha_s (Sec. 5.1: 0.740 in 3D).
 *   g[3], dt      gravity [m/s^2] and step [s].
 *   r_max         largest granule radius that will be passed [m].
 *   walls         bit 2a: wall on the low face of axis a; bit 2a+1: high.
 *   precision     gic_precision.
 * Remaining interphase forces (Sec. 3.3 Eq. 5a-5c; Sec. 5.2 Eq. 9), all off
 * when zero:
 *   rho_f         fluid density rho_f = rho_0 [kg/m^3] >= 0: the pressure-
 *                 gradient force is -V grad p (V = 4/3 pi r^3) whenever a
 *                 grad p grid is passed; rho_f enters the quadratic drag and
 *                 the virtual mass.
 *   drag_model    0: the linear drag above; 1: Eq. (5b) as printed,
 *                 F_d = 12 pi r^2 rho_f c_quad |u - v| (u - v), c_quad >= 0
 *                 the dimensionless coefficient.
 *   vmass         1: virtual mass: (m + rho_f V / 2) dv/dt = F_c + F_d + F_p
 *                 + (rho_f V / 2) a_f + m g with a_f the fluid acceleration
 *                 grid (Eq. 9); 0: none.
 *   f_unit        unit of the fixed-point exchange-force grid [N] (> 0 for
 *                 gic_exchange_p2g and gic_sand_step with an exchange grid).
 * Capillary (concentration-gradient) pair force, Sec. 5.4, applied by
 * gic_contact_capillary_forces only:
 *   sigma         surface tension [N/m] >= 0 (0: off).
 *   vbridge       liquid-bridge volume as a fraction of the pair's mean
 *                 granule volume (Sec. 5.4: 1e-4), > 0 when sigma > 0.
 *   sr_peak       moisture ratio where the moisture curve Gamma peaks (the
 *                 maximum absorption ratio of Sec. 5.3), in (0, 1).
 *                 With sigma > 0, cell >= 2 r_max + d_r(r_max) is required.
 * Absorbed water, Sec. 5.3:
 *   absorb_max    the maximum absorption ratio r_max of Sec. 5.3 (held water
 *                 per unit granule volume), >= 0 (0: dry).  Held water fills
 *                 part of the voids, so every clamp of alpha_s (G2P, the
 *                 density projection's target) is alpha_max (1 + absorb_max),
 *                 the 0.740 (1 + r_max) of Sec. 5.3.
 * The adjoint form (the *_vjp calls) covers drag_model 0 without virtual
 * mass and returns GIC_E_ARG otherwise. */
typedef struct gic_params {
    int32_t n[3];
    int32_t pad0;
    double dx;
    int32_t nc[3];
    int32_t pad1;
    double cell;
    double kn, restitution, kt_ratio, mu;
    double rho_s, eta_f, c_drag, alpha_max;
    double g[3];
    double dt;
    double r_max;
    uint32_t walls;
    int32_t precision;
    double rho_f;
    double c_quad;
    double f_unit;
    int32_t drag_model;
    int32_t vmass;
    double sigma;
    double vbridge;
    double sr_peak;
    double absorb_max;
} gic_params;

typedef struct gic_ctx gic_ctx;

/* Number of neighbour-cell keys K: the length of cell_begin / cell_end.
 * Keys order cells in bricks of 4x4x4, bricks x-fastest, cells x-fastest
 * inside a brick.  Returns -1 for invalid parameters. */
int64_t gic_key_space(const gic_params *p);

/* Create a context on the current HIP device for up to n_max granules;
 * allocates the sort scratch and the error word.  *out is set on success. */
gic_status gic_create(const gic_params *p, int64_t n_max, gic_ctx **out);

/* Replace the parameters (same grid, cells and precision; e.g. mu, c_drag,
 * dt).  Returns GIC_E_ARG if the grid, cells or precision change.  The next
 * gic_step or gic_sand_step builds its neighbour list afresh and writes its
 * grids whole. */
gic_status gic_set_params(gic_ctx *ctx, const gic_params *p);

/* Synchronise the device and free the context's scratch. */
gic_status gic_destroy(gic_ctx *ctx);

/* Synchronise `stream` and read the latched error: *code = 0 or a
 * gic_status, *index = the first granule index that raised it (-1 if none).
 * clear != 0 resets the latch. */
gic_status gic_get_error(gic_ctx *ctx, void *stream, int32_t *code, int64_t *index, int32_t clear);

/* ---- a1: binning and stable radix sort -----------------------------------
 * Neighbour search support for the contact test of Sec. 3.1.
 *   x           3n positions (any order).
 *   key         out, n: cell key of granule i, cell coordinate per axis
 *               clamp(floor(x / cell), 0, nc - 1).
 *   order       out, n: order[q] = index of the granule at sorted position q;
 *               a stable sort by key (ties in input order).
 *   cell_begin, cell_end   out, K each: sorted positions [begin, end) of the
 *               granules of each key: begin[c] = number of granules with a
 *               smaller key, end[c] = number with a key not larger.  Empty
 *               cells have begin = end, so consecutive keys have contiguous
 *               ranges. */
gic_status gic_sort_cells(gic_ctx *ctx, int64_t n, const double *x, uint32_t *key, int32_t *order,
                          int32_t *cell_begin, int32_t *cell_end, void *stream);

/* Build the context's list of occupied bricks (the schedule of the brick
 * kernels) for the cell tables cell_begin, cell_end (K each, from
 * gic_sort_cells), and keep it: the calls that follow and are given these
 * same tables use it instead of building their own, until the next
 * gic_sort_cells, stepping call or gic_brick_list.  The caller must not
 * change the tables' contents meanwhile.  Without this call every brick
 * kernel call builds the list (three small kernels) itself. */
gic_status gic_brick_list(gic_ctx *ctx, const int32_t *cell_begin, const int32_t *cell_end, void *stream);

/* Gather granule arrays into sorted order: out[q] = in[order[q]] for x, v
 * (3n each) and r, id (n each).  id / id_out may both be NULL.  Outputs must
 * not alias inputs. */
gic_status gic_reorder(gic_ctx *ctx, int64_t n, const int32_t *order, const double *x, const double *v,
                       const double *r, const int32_t *id, double *x_out, double *v_out, double *r_out,
                       int32_t *id_out, void *stream);

/* ---- a2 + a3: contact forces (Sec. 3.1, Eq. 1a-c) -------------------------
 * Granules i, j touch iff d^2 < (r_i + r_j)^2 in double with d^2 =
 * (dx*dx + dy*dy) + dz*dz.  Per pair: n = x_ij / d, delta = r_i + r_j - d,
 * v_n = v_ij . n, F_n = (k_n delta - gamma_n v_n) n, f_t = -k_t (v_ij - v_n
 * n), F_t = f_t capped to mu k_n delta along f_t.  Enabled box walls act as
 * infinite-mass partners with the same law.  Positions, position
 * differences, d^2 and the contact test are double in both forms; the
 * overlap is R - d in double (plain form) or (R^2 - d^2) / (R + d) with the
 * cancelling difference R^2 - d^2 in double and the quotient in float (FP32
 * form); the pair force arithmetic and the per-granule sum are in the
 * form's real type, over the touching partners in canonical order (by
 * distance |j - q| in sorted order from the granule q, the lower position j
 * first at equal distance), then the walls.  Without pair_ids the forces come straight from the cells (the
 * brick's 6x6x6-cell shell in LDS); with pair_ids the call builds the
 * context's neighbour list (every granule closer than r_i + r_j + skin, in
 * that order; see gic_step) and evaluates the forces from it.  Both give
 * the same bits.
 *   x, v, r     sorted order (see Conventions).
 *   f_contact   out, 3n real: force per granule [N].
 *   n_contacts  out (optional, NULL = skip), n: touching partners + walls.
 *   pair_ids    out (optional, NULL = skip), pair_cap x n int32,
 *               column-major: pair_ids[k n + q] is the sorted position of
 *               the k-th partner touching granule q (k < pair_cap), in the
 *               order its force is summed, then -1 up to pair_cap; the pair
 *               set is the exact test's, from the same kernel that sums the
 *               forces.
 *   pair_cap    entries per granule in pair_ids (0 with pair_ids NULL). */
gic_status gic_contact_forces(gic_ctx *ctx, int64_t n, const double *x, const double *v, const double *r,
                              const int32_t *cell_begin, const int32_t *cell_end, void *f_contact,
                              int32_t *n_contacts, int32_t *pair_ids, int32_t pair_cap, void *stream);

/* Number of neighbour-list builds on this context so far (gic_contact_forces
 * builds once per call, gic_step and gic_sand_step when their list must be
 * rebuilt).  Synchronises the stream. */
gic_status gic_neighbour_builds(gic_ctx *ctx, void *stream, int64_t *builds);

/* ---- f3: moisture ratio (Sec. 5.4, the definition following Eq. 26) -------
 * sr_i = held_i + alpha_f,i / (1 - alpha_f,i): the water granule i holds
 * (per unit granule volume; the absorption of Sec. 5.3 that changes it is
 * not part of this library) plus the free water around it per unit sand
 * volume.  Evaluated in double, stored in the form's real type; +inf where
 * alpha_f = 1.  n each, any order as long as the three agree; sr may alias
 * neither input.
 *   held      n double: water held by each granule (>= 0), the same array
 *             the wet masses of Eq. 19 take.
 *   alpha_f   n real: fluid fraction sampled at each granule (gic_g2p).
 *   sr        out, n real: moisture ratio. */
gic_status gic_moisture_ratio(gic_ctx *ctx, int64_t n, const double *held, const void *alpha_f, void *sr,
                              void *stream);

/* ---- f3: contact plus capillary liquid-bridge forces (Sec. 5.4) ----------
 * gic_contact_forces plus, for every pair that does not touch and whose
 * surface gap s = d - (r_i + r_j) lies in (0, d_r), the bridge force on i
 *     -Gamma((sr_i + sr_j) / 2) F^st(s) (x_i - x_j) / d,
 *     F^st = 2 pi sigma rb (1 - (1 + 2 V* / (pi rb s^2))^(-1/2)),
 * with rb = (r_i + r_j) / 2, V* = vbridge (4/3) pi rb^3, d_r = V*^(1/3) +
 * 0.1 V*^(2/3) and Gamma the moisture curve: u (2 - u) with u = sr / sr_peak
 * up to sr_peak, 1 - u^2 with u = (sr - sr_peak) / (1 - sr_peak) after it,
 * 0 outside (0, 1).  The bridge force is evaluated in double and added to
 * the granule's sum in the form's real type, in the same partner order as
 * the contact forces.  Requires sigma > 0 (GIC_E_ARG otherwise).
 *   sr          n real (the form's type), sorted order: moisture ratio per
 *               granule (Sec. 5.3).
 *   held        n double, sorted order (optional, NULL = dry masses): water
 *               each granule holds per unit of its volume; the contact
 *               damping then uses the wet masses V (rho_s + held rho_f) of
 *               Eq. 19.
 *   f_contact   out, 3n real: contact plus bridge force per granule [N].
 *   n_contacts  out (optional), n: touching partners + walls (bridged
 *               pairs are not counted). */
gic_status gic_contact_capillary_forces(gic_ctx *ctx, int64_t n, const double *x, const double *v,
                                        const double *r, const void *sr, const double *held,
                                        const int32_t *cell_begin, const int32_t *cell_end, void *f_contact,
                                        int32_t *n_contacts, void *stream);

/* ---- a5: G2P of fluid velocity and fraction (Sec. 5.2; Sec. 5.1 clamp) ----
 * Quadratic B-spline on cell-centred nodes, out-of-range nodes folded onto
 * the edge node.  u_at = sum_k w_k u_k; alpha_f = 1 - sum_k w_k min(alpha_k,
 * alpha_max) with alpha_k = alpha_fx[k] 2^-32 (fixed point) or alpha_real[k]
 * (cell volumes); exactly one of alpha_fx, alpha_real is non-NULL.
 *   u           3G real fluid velocity at the nodes [m/s].
 *   u_at        out, 3n real;  alpha_f  out, n real. */
gic_status gic_g2p(gic_ctx *ctx, int64_t n, const double *x, const void *u, const int64_t *alpha_fx,
                   const double *alpha_real, void *u_at, void *alpha_f, void *stream);

/* ---- a6: drag (Eq. 5b, App. A) ---------------------------------------------
 * f_drag = c_drag 6 pi eta_f r alpha_f (u_at - v), all real, 3n out. */
gic_status gic_drag(gic_ctx *ctx, int64_t n, const double *r, const double *v, const void *u_at,
                    const void *alpha_f, void *f_drag, void *stream);

/* ---- a7: integration (Sec. 4, semi-implicit Euler, double) ----------------
 * v += dt ((f_contact + f_drag) / m + g); x += dt v, with m = rho_s 4/3 pi
 * r^3.  x and v are updated in place.  f_drag may be NULL (no drag). */
gic_status gic_integrate(gic_ctx *ctx, int64_t n, const double *r, const void *f_contact, const void *f_drag,
                         double *x, double *v, void *stream);

/* ---- a4: P2G of volume fraction and momentum (Sec. 5.1, Eq. 7a) ------------
 * Fixed point: alpha in 2^-32 cell volumes, momentum in 2^-32 rho_s dx^3
 * (1 m/s) units.  Per granule and channel the total is Q = rint(S) with
 * S = frac 2^32 (alpha) or (frac v_c) 2^32 (momentum), frac = (4/3 pi r^3)
 * / dx^3; each of the 26 outer stencil nodes takes w S rounded once to the
 * nearest integer (the exact product of the double weight w and S, ties to
 * even) and the centre node takes Q minus their sum, so every granule
 * deposits exactly Q.  Integer sums make the grid independent of the order
 * of accumulation.
 *   alpha_fx    G int64, mom_fx 3G int64 (mom_fx may be NULL).
 *   accumulate  0: the grids are cleared first; 1: added to. */
gic_status gic_p2g(gic_ctx *ctx, int64_t n, const double *x, const double *v, const double *r,
                   const int32_t *cell_begin, const int32_t *cell_end, int64_t *alpha_fx, int64_t *mom_fx,
                   int32_t accumulate, void *stream);

/* Unquantised P2G for the differentiable form: alpha in cell volumes
 * (sum w frac), momentum in kg m/s (sum w m v), double; accumulation order is
 * not fixed, so results agree with a sequential sum to rounding only. */
gic_status gic_p2g_real(gic_ctx *ctx, int64_t n, const double *x, const double *v, const double *r,
                        const int32_t *cell_begin, const int32_t *cell_end, double *alpha, double *mom,
                        int32_t accumulate, void *stream);

/* ---- fused stages (same results, bit for bit, as the separate calls) ------
 * gic_gather_g2p_drag = gic_reorder, then gic_g2p with alpha_fx, then
 * gic_drag, in one pass over the bricks of cells (Sec. 5.2; Eq. 5b, App. A):
 * the state of granule order[q] is written to position q of the _out
 * arrays, and its drag force to f_drag[q].  u_at and alpha_f (3n and n
 * real) receive the sampled fluid velocity and fraction, or are skipped
 * when NULL.  cell_begin, cell_end: ranges of the sort that gave `order`. */
gic_status gic_gather_g2p_drag(gic_ctx *ctx, int64_t n, const int32_t *order, const double *x, const double *v,
                               const double *r, const int32_t *id, double *x_out, double *v_out, double *r_out,
                               int32_t *id_out, const void *u, const int64_t *alpha_fx, const int32_t *cell_begin,
                               const int32_t *cell_end, void *f_drag, void *u_at, void *alpha_f, void *stream);

/* gic_integrate_p2g = gic_integrate (x, v advanced in place with f_contact +
 * f_drag), then gic_p2g of the new state (Sec. 4; Sec. 5.1, Eq. 7a), in one
 * pass: each granule is moved and deposited by the same thread.  x, v, r in
 * the sorted order of cell_begin, cell_end.  accumulate as in gic_p2g. */
gic_status gic_integrate_p2g(gic_ctx *ctx, int64_t n, double *x, double *v, const double *r, const void *f_contact,
                             const void *f_drag, const int32_t *cell_begin, const int32_t *cell_end,
                             int64_t *alpha_fx, int64_t *mom_fx, int32_t accumulate, void *stream);

/* gic_integrate_p2g for wet granules (Sec. 5.3, Eq. 19): held (n double,
 * sorted order, required for n > 0) is the water each granule holds per unit
 * of its volume; the integrator uses the mass V (rho_s + held rho_f) (with
 * virtual mass: that mass plus rho_f V (1 + held) / 2, gravity on the wet
 * mass), the fraction channel deposits frac (1 + held) (the absorbed water
 * counts as volume in alpha_s, Sec. 5.3) and the momentum channels
 * (frac + frac held rho_f / rho_s) v.  held = 0 gives gic_integrate_p2g's
 * bits. */
gic_status gic_integrate_p2g_wet(gic_ctx *ctx, int64_t n, double *x, double *v, const double *r, const double *held,
                                 const void *f_contact, const void *f_drag, const int32_t *cell_begin,
                                 const int32_t *cell_end, int64_t *alpha_fx, int64_t *mom_fx, int32_t accumulate,
                                 void *stream);

/* ---- one full sub-step -------------------------------------------------------
 * Sort, reorder, G2P (alpha_fx at the current positions, as left by the
 * previous step's P2G), drag, contact, integrate, P2G, run as
 * gic_sort_cells -> gic_gather_g2p_drag -> gic_contact_forces ->
 * gic_integrate_p2g.  The granule state is double-buffered: x, v, r, id are
 * read from the `cur` arrays and written, advanced and in the new sorted
 * order, to the `nxt` arrays (same sizes); the caller swaps them.  alpha_fx
 * is read, then overwritten with the fraction at the new positions; mom_fx
 * receives the new momentum.  Both are complete after every step; when they
 * are the arrays of the previous step on this context, the step rewrites
 * only the 4-node x-segments that a granule's stencil reaches now or reached
 * then (the rest hold that step's zeros and are left as they are), so a
 * caller that writes into them between steps passes other arrays or calls
 * gic_set_params first (calls on the context that write grids into them
 * are noticed).  Scratch arrays (caller-owned): key, order (n
 * int32), cell_begin, cell_end (K int32), f_contact, f_drag (3n real; they
 * hold the step's forces afterwards); u_at (3n real) and alpha_f (n real)
 * receive the sampled fluid velocity and fraction, or are skipped when
 * NULL.
 * Neighbour list: the contact stage keeps the context's list of every pair
 * closer than r_i + r_j + skin (skin = min(r_max / 10, cell - 2 r_max)) from
 * one step to the next while x_cur is the x_nxt of the previous gic_step on
 * this context with the same n, the sort finds no changed cell key and no
 * granule has moved by skin / 2 since the list was built (measured on the
 * device from the positions of the build); otherwise the step rebuilds it.
 * The exact contact test runs on every listed pair every step, and a
 * granule's forces are summed over its touching partners in canonical order
 * either way, so f_contact is the same bits as gic_contact_forces on the
 * sorted state.  Calls of gic_sort_cells or gic_contact_forces on the
 * context, gic_set_params, or radii changed by the caller between steps:
 * the first two and the third make the next step rebuild; radii must only
 * change through new arrays (x_cur then differs) or gic_set_params. */
gic_status gic_step(gic_ctx *ctx, int64_t n, const double *x_cur, const double *v_cur, const double *r_cur,
                    const int32_t *id_cur, double *x_nxt, double *v_nxt, double *r_nxt, int32_t *id_nxt,
                    const void *u, int64_t *alpha_fx, int64_t *mom_fx, uint32_t *key, int32_t *order,
                    int32_t *cell_begin, int32_t *cell_end, void *f_contact, void *f_drag, void *u_at,
                    void *alpha_f, void *stream);

/* Stage timing of gic_step and gic_sand_step for measurement: with
 * max_steps > 0 the next max_steps (sub-)steps record HIP events on their
 * stream between their stages (creates the events; 0 switches timing off and
 * destroys them).  gic_stage_times synchronises the stream and returns, over
 * the (sub-)steps recorded since the last call, the summed milliseconds of
 * ms[0] sort (keys, sort, cell ranges, brick list), ms[1] gather + G2P +
 * fluid force, ms[2] contact (neighbour-list build when needed, forces),
 * ms[3] exchange deposit (0 in gic_step), ms[4] grid clear, ms[5] integrate
 * + P2G (the brick-tile kernel, or the atomic deposit into cleared grids),
 * ms[6] the grids assembled from the brick tiles, with the granules whose
 * stencil left their tile (0 on the atomic path); ms holds 7 doubles;
 * *steps receives their number. */
gic_status gic_stage_timing(gic_ctx *ctx, int32_t max_steps);
gic_status gic_stage_times(gic_ctx *ctx, void *stream, double *ms, int32_t *steps);

/* ---- remaining interphase forces and the sand step -------------------------
 * gic_gather_g2p_fluid = gic_gather_g2p_drag with the whole fluid force of
 * Sec. 3.3 (Eq. 5a-5c) written to f_fluid (3n real): the drag of
 * params.drag_model, plus -V grad p with grad_p (3 x G real, the pressure
 * gradient of the fluid step, Sec. 5.2) interpolated like u, plus
 * (rho_f V / 2) a_f under params.vmass with acc_f (3 x G real, the fluid
 * acceleration dv_f/dt of the grid, Eq. 12), V = 4/3 pi r^3.  grad_p and
 * acc_f may be NULL (no such term).  The a_s part of the virtual-mass force
 * is the effective mass of the integrator (gic_integrate_p2g with vmass).
 * held, held_out (n double each, both or neither): wet granules (Sec. 5.3):
 * held (input order) is the water each granule holds per unit of its
 * volume and counts as volume, V = 4/3 pi r^3 (1 + held), in -V grad p and
 * the virtual mass (the drag keeps the granule's radius); it is written in
 * sorted order to held_out.  The _out arrays must not alias the inputs. */
gic_status gic_gather_g2p_fluid(gic_ctx *ctx, int64_t n, const int32_t *order, const double *x, const double *v,
                                const double *r, const int32_t *id, double *x_out, double *v_out, double *r_out,
                                int32_t *id_out, const void *u, const int64_t *alpha_fx, const void *grad_p,
                                const void *acc_f, const int32_t *cell_begin, const int32_t *cell_end,
                                void *f_fluid, const double *held, double *held_out, void *stream);

/* Exchange momentum of one sub-step (Sec. 5.2): adds -weight f_j N(x_j - x)
 * to fs_fx (3 x G int64, x-plane then y and z, units of 2^-32
 * params.f_unit), f_j the whole fluid force on granule j: f_fluid, and under
 * params.vmass minus (rho_f V / 2) a_s with a_s = ((f_contact + f_fluid) +
 * m g) / (m + rho_f V / 2), the sub-step's acceleration.  Per granule and
 * component the deposit totals rint(S), S = (-weight / f_unit) f 2^32, the 26
 * outer nodes taking w S rounded once and the centre the rest (integer, so bit-exact
 * in any order).  x, r, f_contact, f_fluid in the sorted order of
 * cell_begin, cell_end (positions before the move).  held (n double,
 * sorted order, or NULL): wet granules take the wet mass V (rho_s + held
 * rho_f) and the volume V (1 + held) in a_s and the virtual mass (Sec. 5.3).
 * GIC_E_ARG if params.f_unit <= 0.  Latches GIC_E_RANGE for |S| >= 2^51. */
gic_status gic_exchange_p2g(gic_ctx *ctx, int64_t n, const double *x, const double *r, const void *f_contact,
                            const void *f_fluid, const int32_t *cell_begin, const int32_t *cell_end, double weight,
                            int64_t *fs_fx, const double *held, void *stream);

/* One sand step (Alg. 2) of length Dt: N = ceil(Dt / params.dt) equal
 * sub-steps of Dt / N with the fluid fields u, grad_p, acc_f frozen, each
 * gic_sort_cells -> gic_gather_g2p_fluid -> gic_contact_forces ->
 * gic_exchange_p2g (weight 1/N; skipped when fs_fx is NULL) ->
 * gic_integrate_p2g.  The state ping-pongs between the a and b arrays,
 * starting in a; *which = 0 if it ends in a, 1 if in b; *nsub = N.  fs_fx
 * accumulates (clear it before the first sand step of a fluid step);
 * alpha_fx, mom_fx hold the P2G of the final state (rewritten as by
 * gic_step: only where a stencil reaches now or did at the last write of the
 * same arrays).  Scratch as for gic_step; f_contact, f_fluid hold the last
 * sub-step's forces. */
gic_status gic_sand_step(gic_ctx *ctx, int64_t n, double Dt, double *x_a, double *v_a, double *r_a, int32_t *id_a,
                         double *x_b, double *v_b, double *r_b, int32_t *id_b, const void *u, const void *grad_p,
                         const void *acc_f, int64_t *alpha_fx, int64_t *mom_fx, int64_t *fs_fx, uint32_t *key,
                         int32_t *order, int32_t *cell_begin, int32_t *cell_end, void *f_contact, void *f_fluid,
                         int32_t *nsub, int32_t *which, void *stream);

/* ---- a9: adjoint form ------------------------------------------------------
 * Vector-Jacobian products of the stages of the differentiable step (all
 * double; the context must be GIC_FP64).  The forward of the differentiable
 * step uses unquantised transfers (gic_p2g_real):
 *   A = P2G_alpha(x);  (u_at, alpha_f) = G2P(x; u, A);
 *   F_d = c_drag 6 pi eta_f r alpha_f (u_at - v);  F_c = contact(x, v; mu);
 *   v' = v + dt ((F_c + F_d)/m + g);  x' = x + dt v'.
 * Cotangents named g_*; "+=" outputs accumulate, "=" outputs are written.
 * The alpha clamp and the Coulomb cap take the derivative of the branch in
 * effect (the clamp passes no gradient at or above alpha_max).  Per-granule
 * parameter contributions (g_mu, g_cdrag) are written per granule; gic_sum
 * adds them in a fixed order, so results are reproducible run to run. */

/* Contact pullback (Sec. 3.1, Eq. 1a-c) in gather form: granule i collects,
 * for every touching partner j, the pair term with cotangent g_f[i] - g_f[j].
 *   g_f 3n;  g_x, g_v 3n (+=);  g_mu n (=, dL/dmu per granule). */
gic_status gic_contact_forces_vjp(gic_ctx *ctx, int64_t n, const double *x, const double *v, const double *r,
                                  const int32_t *cell_begin, const int32_t *cell_end, const double *g_f, double *g_x,
                                  double *g_v, double *g_mu, void *stream);

/* Drag pullback (Eq. 5b, App. A):  g_v += -beta alpha_f g_f;  g_u_at =
 * beta alpha_f g_f;  g_alpha_f = beta (u_at - v).g_f;  g_cdrag[i] =
 * 6 pi eta_f r alpha_f (u_at - v).g_f  (beta = c_drag 6 pi eta_f r). */
gic_status gic_drag_vjp(gic_ctx *ctx, int64_t n, const double *r, const double *v, const double *u_at,
                        const double *alpha_f, const double *g_f, double *g_v, double *g_u_at, double *g_alpha_f,
                        double *g_cdrag, void *stream);

/* Integration pullback (Sec. 4): on entry g_x, g_v are dL/dx', dL/dv'; on
 * return g_v = g_v + dt g_x (the adjoint of v through the identity term)
 * and g_f = dt/m times it (dL/d(F_c + F_d)); g_x is unchanged (= its
 * identity part for x). */
gic_status gic_integrate_vjp(gic_ctx *ctx, int64_t n, const double *r, const double *g_x, double *g_v, double *g_f,
                             void *stream);

/* G2P pullback (Sec. 5.2) with a real alpha grid:  g_x += sum_k grad w_k
 * (u_k . g_u_at - min(A_k, alpha_max) g_alpha_f);  g_alpha (G, =, optional)
 * = -sum_i w_ik g_alpha_f[i] on nodes below the clamp, 0 elsewhere.  The grid part needs
 * the sorted order and cell tables of x (as gic_p2g). */
gic_status gic_g2p_vjp(gic_ctx *ctx, int64_t n, const double *x, const double *u, const double *alpha_real,
                       const double *g_u_at, const double *g_alpha_f, const int32_t *cell_begin,
                       const int32_t *cell_end, double *g_x, double *g_alpha, void *stream);

/* P2G pullback (Sec. 5.1, Eq. 7a) of the real transfers: g_alpha (G) and/or
 * g_mom (3G) given;  g_x += ..., g_v += m sum_k w_k g_mom_k. */
gic_status gic_p2g_vjp(gic_ctx *ctx, int64_t n, const double *x, const double *v, const double *r,
                       const double *g_alpha, const double *g_mom, double *g_x, double *g_v, void *stream);

/* *out (device double) = (accumulate ? *out : 0) + sum of a[i] (b == NULL)
 * or of a[i] b[i], i < n, summed in a fixed order (reproducible). */
gic_status gic_sum(gic_ctx *ctx, int64_t n, const double *a, const double *b, double *out, int32_t accumulate,
                   void *stream);

/* gic_sum without a context, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and summation order as gic_sum (so the same
 * bits), with its 1,024 partial sums in a fixed 8 KiB array that the library
 * holds on each device until the process ends.  Nothing is allocated, and
 * the call neither synchronises nor clears memory (the partials are written
 * before they are read).  GIC_E_ARG for n > 2^30 (1,024 partials of at most
 * 2^20 values), n < 0, a or out NULL; GIC_E_HIP if the array's address
 * cannot be looked up.  Every call on one GPU uses that GPU's one array:
 * calls that overlap on a GPU (concurrent streams) race and must be
 * serialised by the caller. */
gic_status gic_sum_noalloc(int64_t n, const double *a, const double *b, double *out, int32_t accumulate,
                           void *stream);

/* out[i] = (factor s[0]) a[i], i < n, with s a DEVICE scalar: e.g. the
 * cotangent of the rollout loss L = sum P^2, dL/dP = (2 gL) P, formed
 * without reading gL back to the host.  out may alias a. */
gic_status gic_scale(gic_ctx *ctx, int64_t n, const double *a, const double *s, double factor, double *out,
                     void *stream);

/* Permute comps (1..6) planes of n doubles (six: positions and velocities
 * held as one array, x then v): scatter = 0: out[c n + q] =
 * in[c n + order[q]];  scatter = 1: out[c n + order[q]] = in[c n + q]. */
gic_status gic_permute(gic_ctx *ctx, int64_t n, int32_t comps, const int32_t *order, const double *in, double *out,
                       int32_t scatter, void *stream);

/* ==== f4: density projection of the fluid fraction (Sec. 5.1) =============
 * Eq. 12b on the MAC grid of App. B.  The cells are the transfer grid's nodes
 * (params n, dx; cell centres, x fastest, G = n0 n1 n2 cells).  All grids
 * here are double in both forms; labels are uint8 per cell: 0 fluid, 1 air,
 * 2 solid.  With the scaled pressure q = (dt^2 / (rho_0 dx^2)) p_2 every
 * fluid cell c satisfies
 *     (L q)_c = sum_j beta_cj (q_c - q_j) = alpha_f'(c) (clamp(alpha_f*(c) / alpha_f'(c), 0.5, 1.5) - 1)
 * over its six face neighbours j that are not solid and inside the box, with
 * beta_cj = (alpha_f'(c) + alpha_f'(j)) / 2; air neighbours enter with
 * q_j = 0 (p = 0 at the free surface), solid neighbours and the box boundary
 * close the face (zero normal flux).  Rows of non-fluid cells are the
 * identity with a zero right-hand side, so L is symmetric positive definite
 * when every connected fluid region touches air, and the solution is zero
 * off the fluid.  Reading: the sign of Eq. 12b is kept (the fluid moves out
 * of a cell whose fraction exceeds its target); App. B prints the operator
 * with the opposite sign of its right-hand side.
 *
 * A label outside 0..2 (setup, solve) or alpha_t not in (0, inf) on a fluid
 * or air cell (solve) latches GIC_E_RANGE with the cell's index.
 *
 * gic_idp_setup: alpha_t = 1 - min(alpha_fx 2^-32, alpha_max (1 + absorb_max)) (the target
 * fraction from the P2G grid, G int64) and rhs (the right-hand side above,
 * zero off the fluid) from alpha_star (G, the fluid particles' own fraction,
 * Eq. 7b: an input) and label.  Asynchronous. */
gic_status gic_idp_setup(gic_ctx *ctx, const int64_t *alpha_fx, const double *alpha_star, const uint8_t *label,
                         double *alpha_t, double *rhs, void *stream);

/* out = L q (G doubles, out must not alias q).  Asynchronous. */
gic_status gic_idp_apply(gic_ctx *ctx, const double *alpha_t, const uint8_t *label, const double *q, double *out,
                         void *stream);

/* Bytes of the caller-owned device workspace that gic_idp_solve and
 * gic_density_projection need with either preconditioner (about 80 G; -1
 * for a NULL context). */
int64_t gic_idp_workspace_bytes(const gic_ctx *ctx);

/* Solves L q = rhs by preconditioned conjugate gradients, starting from the
 * q passed in (q = 0 for a cold start).  precond 0: Jacobi (1 / diag L);
 * precond 1: one multigrid V-cycle per iteration (levels halve each axis,
 * rounding up, down to at most 256 cells; a coarse cell is air if a child
 * is, else fluid if a child is, else solid, with the mean alpha_f' of its
 * children that are not solid; level l uses 4^l L of its own cells;
 * piecewise-constant prolongation and its transpose; one damped Jacobi
 * sweep, omega = 2/3, before and one after the coarse correction; 48 sweeps
 * on the coarsest level),
 * a symmetric preconditioner, so CG applies.  Stops when
 * |r|_2 <= tol |rhs|_2 (recursively updated residual) or after max_iter
 * iterations.  Enqueues check_every iterations at a time and SYNCHRONISES the
 * stream after each chunk to read the state; iterations of a chunk after
 * convergence return at once.  *iters (host, optional) receives the
 * iterations done, *relres (host, optional) |r| / |rhs| at the end (|r| when
 * rhs = 0).  GIC_OK also when max_iter is reached: check *relres.  work: at
 * least gic_idp_workspace_bytes bytes of device memory, 256-byte aligned. */
gic_status gic_idp_solve(gic_ctx *ctx, const double *alpha_t, const uint8_t *label, const double *rhs, double *q,
                         void *work, int32_t max_iter, double tol, int32_t check_every, int32_t precond,
                         int32_t *iters, double *relres, void *stream);

/* Position change on the MAC faces (Eq. 13 in q): for the face between cell
 * c and its +axis neighbour j, dx (q_c - q_j) (air sides count as q = 0; a
 * positive value moves fluid along +axis) where one side is fluid and
 * neither is solid, else 0; clamped to [-dx, dx] (Sec. 5.1).  Faces on the
 * box boundary are 0.  fx: n2 x n1 x (n0 + 1), fy: n2 x (n1 + 1) x n0,
 * fz: (n2 + 1) x n1 x n0, x fastest; face i + 1/2 along an axis is stored at
 * index i + 1.  Asynchronous. */
gic_status gic_idp_displacement(gic_ctx *ctx, const double *q, const uint8_t *label, double *fx, double *fy,
                                double *fz, void *stream);

/* The whole projection: gic_idp_setup into the workspace, gic_idp_solve
 * (q in: initial guess, out: solution) and gic_idp_displacement.
 * Synchronises like gic_idp_solve. */
gic_status gic_density_projection(gic_ctx *ctx, const int64_t *alpha_fx, const double *alpha_star,
                                  const uint8_t *label, double *q, double *fx, double *fy, double *fz, void *work,
                                  int32_t max_iter, double tol, int32_t check_every, int32_t precond,
                                  int32_t *iters, double *relres, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GIC_H */
