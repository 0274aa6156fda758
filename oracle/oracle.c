/*
 * Granule-In-Cell granule step: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * library never links, includes or calls it, and it includes nothing from the
 * product library.
 *
 * Paper: Tang, Zhu, Ni, Chen, "The Granule-In-Cell Method for Simulating
 * Sand-Water Mixtures", ACM TOG 44(6) 2025 (arXiv 2504.00745).
 *
 * Passages followed:
 *   contact force .......... Sec. 3.1, Eq. (1a)-(1c)
 *   interphase drag ........ Sec. 3.3, Eq. (5b) and App. A (linear relaxation
 *                            drag M_s = a_s rho_s (v_f - v_s) / tau_s)
 *   sub-step loop .......... Alg. 2 (SandSubstep): coupling force, collision,
 *                            move
 *   integrator ............. Sec. 4 (semi-implicit, symplectic Euler type)
 *   volume fraction P2G .... Sec. 5.1, Eq. (7a), at cell centres
 *   alpha_s limit 0.740 .... Sec. 5.1 (densest sphere packing, 3D)
 *   fluid velocity G2P ..... Sec. 5.2 (grid fluid velocity interpolated to
 *                            each granule's position)
 *
 * Readings where the paper is silent (all recorded in the design notes):
 *   - normal dashpot from a restitution coefficient (Eq. 1a has none);
 *     gamma_n = 2 zeta sqrt(m_eff k_n), zeta = -ln e / sqrt(pi^2 + ln^2 e);
 *     no tensile clamp;
 *   - k_t = kt_ratio * gamma_n (k_t multiplies a velocity in Eq. 1c);
 *   - Coulomb cap = tan(phi) * k_n * delta, i.e. the norm of Eq. 1a's spring
 *     force; mu = tan(phi);
 *   - polydisperse: 2r -> r_i + r_j, strict "<";
 *   - six planar box walls, infinite-mass partners, same law;
 *   - drag F_d = C_d 6 pi eta_f r alpha_f (u - v) (Stokes form of App. A's
 *     relaxation drag, scaled by the local fluid fraction);
 *   - grid nodes at cell centres (i + 1/2) dx, quadratic B-spline kernel,
 *     out-of-range nodes folded onto the edge node;
 *   - alpha_s clamped at the nodes, then interpolated; alpha_f = 1 - alpha_s;
 *   - int64 fixed point, 2^-32 units, round half to even (each outer
 *     node's contribution w S rounded once, from the exact product), the
 *     per-granule remainder goes to the centre node so each granule deposits
 *     exactly rint(frac * 2^32);
 *   - coincident centres (d == 0) exert no force.
 *
 * Arrays are structure-of-arrays: x[0..n) = x-coordinates, x[n..2n) = y,
 * x[2n..3n) = z; the same for v and for every 3-vector per granule.  Grid
 * arrays are x-fastest: node (i,j,k) sits at i + nx (j + ny k); 3-vector grid
 * fields are three consecutive G-sized planes.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (see build.py).
 * No contracted multiply-add anywhere: every product and sum below is
 * rounded on its own, in the order written.  The one fused operation is the
 * explicit fma() of orc_round_product, which rounds a fixed-point
 * contribution w S to an integer in a single step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_C43PI (4.0 * ORC_PI / 3.0)
#define ORC_C6PI (6.0 * ORC_PI)
#define ORC_TWO32 4294967296.0
#define ORC_TWOM32 (1.0 / 4294967296.0)
#define ORC_BRICK 4 /* neighbour cells per brick edge in the cell key */

typedef struct {
    int32_t n[3];       /* grid nodes per axis; node i sits at (i + 1/2) dx */
    double dx;          /* grid spacing [m]                                */
    int32_t nc[3];      /* neighbour cells per axis                         */
    double cell;        /* neighbour cell edge [m], >= 2 r_max              */
    double kn;          /* normal stiffness [N/m]                           */
    double restitution; /* normal coefficient of restitution e in (0,1]     */
    double kt_ratio;    /* k_t = kt_ratio * gamma_n                         */
    double mu;          /* Coulomb coefficient tan(phi)                     */
    double rho_s;       /* granule density [kg/m^3]                         */
    double eta_f;       /* fluid viscosity [Pa s]                           */
    double c_drag;      /* drag coefficient C_d (dimensionless)             */
    double alpha_max;   /* node clamp of alpha_s (0.740)                    */
    double g[3];        /* gravity [m/s^2]                                  */
    double dt;          /* step [s]                                         */
    uint32_t walls;     /* bit 2a: low face of axis a, bit 2a+1: high face  */
    int32_t pad;
    double absorb_max;  /* maximum absorption ratio r_max of Sec. 5.3 (0: dry) */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Small helpers                                                            */
/* ------------------------------------------------------------------------ */

static double orc_mass(const orc_params *p, double r)
{
    /* m = rho_s * (4/3) pi r^3 */
    return p->rho_s * (((ORC_C43PI * r) * r) * r);
}

static double orc_volume(double r)
{
    return ((ORC_C43PI * r) * r) * r;
}

/* Damping ratio of the linear spring-dashpot that gives restitution e. */
/* Volume of a granule with its absorbed water (Sec. 5.3): V (1 + held),
 * written so that held = 0 gives V exactly. */
static double orc_wet_volume(double r, double held)
{
    double V = orc_volume(r);
    return held != 0.0 ? V + V * held : V;
}

/* Clamp of alpha_s (Sec. 5.1), raised to 0.740 (1 + r_max) when granules
 * absorb water (Sec. 5.3): the held water fills part of the voids, so the
 * densest packing of wet granules holds more than the sand's own volume. */
static double orc_alpha_clamp(const orc_params *p) { return p->alpha_max * (1.0 + p->absorb_max); }

static double orc_zeta(double e)
{
    double le = log(e);
    return -le / sqrt(ORC_PI * ORC_PI + le * le);
}

static int64_t orc_nodes(const orc_params *p)
{
    return (int64_t)p->n[0] * p->n[1] * p->n[2];
}

/* Neighbour-cell coordinate along one axis: clamp(floor(x / cell), 0, nc-1).
 * NaN maps to 0. */
static int32_t orc_cell_coord(double x, double inv_cell, int32_t nc)
{
    double t = floor(x * inv_cell);
    if (!(t >= 0.0)) return 0;
    if (t > (double)(nc - 1)) return nc - 1;
    return (int32_t)t;
}

/* Key of a neighbour cell: bricks of 4x4x4 cells in x-fastest brick order,
 * cells x-fastest inside a brick. */
static uint32_t orc_key_of_cell(const orc_params *p, int32_t cx, int32_t cy, int32_t cz)
{
    int32_t nbx = (p->nc[0] + ORC_BRICK - 1) / ORC_BRICK;
    int32_t nby = (p->nc[1] + ORC_BRICK - 1) / ORC_BRICK;
    uint32_t brick = (uint32_t)(((cz / ORC_BRICK) * nby + (cy / ORC_BRICK)) * nbx + (cx / ORC_BRICK));
    uint32_t local = (uint32_t)(((cz % ORC_BRICK) * ORC_BRICK + (cy % ORC_BRICK)) * ORC_BRICK + (cx % ORC_BRICK));
    return brick * (uint32_t)(ORC_BRICK * ORC_BRICK * ORC_BRICK) + local;
}

int64_t orc_key_space(const orc_params *p)
{
    int64_t nbx = (p->nc[0] + ORC_BRICK - 1) / ORC_BRICK;
    int64_t nby = (p->nc[1] + ORC_BRICK - 1) / ORC_BRICK;
    int64_t nbz = (p->nc[2] + ORC_BRICK - 1) / ORC_BRICK;
    return nbx * nby * nbz * ORC_BRICK * ORC_BRICK * ORC_BRICK;
}

/* ------------------------------------------------------------------------ */
/* Binning and stable sort (neighbour search support)                        */
/* ------------------------------------------------------------------------ */

void orc_cell_keys(const orc_params *p, int64_t n, const double *x, uint32_t *key)
{
    double inv_cell = 1.0 / p->cell;
    for (int64_t i = 0; i < n; ++i) {
        int32_t cx = orc_cell_coord(x[i], inv_cell, p->nc[0]);
        int32_t cy = orc_cell_coord(x[n + i], inv_cell, p->nc[1]);
        int32_t cz = orc_cell_coord(x[2 * n + i], inv_cell, p->nc[2]);
        key[i] = orc_key_of_cell(p, cx, cy, cz);
    }
}

typedef struct {
    uint32_t key;
    int32_t idx;
} orc_kv;

static int orc_kv_cmp(const void *a, const void *b)
{
    const orc_kv *u = (const orc_kv *)a, *w = (const orc_kv *)b;
    if (u->key != w->key) return u->key < w->key ? -1 : 1;
    /* ties keep input order: the sort is stable */
    return (u->idx > w->idx) - (u->idx < w->idx);
}

/* order[p] = index of the granule at sorted position p; ties in input order. */
void orc_stable_sort(int64_t n, const uint32_t *key, int32_t *order)
{
    orc_kv *kv = (orc_kv *)malloc(sizeof(orc_kv) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        kv[i].key = key[i];
        kv[i].idx = (int32_t)i;
    }
    qsort(kv, (size_t)n, sizeof(orc_kv), orc_kv_cmp);
    for (int64_t i = 0; i < n; ++i) order[i] = kv[i].idx;
    free(kv);
}

/* begin[c], end[c] for every key c of the key space: the sorted positions
 * [begin, end) of the granules in cell c, i.e. begin[c] = number of granules
 * with a smaller key and end[c] = number with a key not larger (an empty cell
 * has begin = end, so consecutive cells have contiguous ranges). */
void orc_cell_ranges(const orc_params *p, int64_t n, const uint32_t *key, const int32_t *order,
                     int32_t *begin, int32_t *end)
{
    int64_t K = orc_key_space(p);
    int64_t *count = (int64_t *)calloc((size_t)K, sizeof(int64_t));
    for (int64_t q = 0; q < n; ++q) count[key[order[q]]] += 1;
    int64_t below = 0;
    for (int64_t k = 0; k < K; ++k) {
        begin[k] = (int32_t)below;
        below += count[k];
        end[k] = (int32_t)below;
    }
    free(count);
}

/* ------------------------------------------------------------------------ */
/* Contact test and pair list                                                */
/* ------------------------------------------------------------------------ */

/* Sec. 3.1: granules i, j touch iff d_ij < r_i + r_j; the test is done on
 * squared distances with d^2 = (dx*dx + dy*dy) + dz*dz. */
static int orc_touch(int64_t n, const double *x, const double *r, int64_t i, int64_t j, double dv[3],
                     double *d2)
{
    dv[0] = x[i] - x[j];
    dv[1] = x[n + i] - x[n + j];
    dv[2] = x[2 * n + i] - x[2 * n + j];
    *d2 = (dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2];
    double R = r[i] + r[j];
    return *d2 < R * R;
}

/* All touching pairs i < j by the plain O(N^2) definition.  Returns the pair
 * count; writes at most cap pairs. */
int64_t orc_pairs_brute(int64_t n, const double *x, const double *r, int64_t cap, int32_t *pi,
                        int32_t *pj)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double dv[3], d2;
            if (orc_touch(n, x, r, i, j, dv, &d2)) {
                if (cnt < cap) {
                    pi[cnt] = (int32_t)i;
                    pj[cnt] = (int32_t)j;
                }
                ++cnt;
            }
        }
    return cnt;
}

/* Cell list built from the keys, for the cell-based search below. */
typedef struct {
    uint32_t *key;
    int32_t *order;
    int32_t *begin;
    int32_t *end;
} orc_cells;

static void orc_cells_build(const orc_params *p, int64_t n, const double *x, orc_cells *c)
{
    int64_t K = orc_key_space(p);
    c->key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    c->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    c->begin = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    c->end = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    orc_cell_keys(p, n, x, c->key);
    orc_stable_sort(n, c->key, c->order);
    orc_cell_ranges(p, n, c->key, c->order, c->begin, c->end);
}

static void orc_cells_free(orc_cells *c)
{
    free(c->key);
    free(c->order);
    free(c->begin);
    free(c->end);
}

/* Largest number of granules in one cell. */
static int64_t orc_cells_maxocc(const orc_params *p, const orc_cells *c)
{
    int64_t K = orc_key_space(p), m = 0;
    for (int64_t k = 0; k < K; ++k)
        if (c->end[k] - c->begin[k] > m) m = c->end[k] - c->begin[k];
    return m;
}

/* Candidates of granule i: every j != i in the 27 cells around i's cell (the
 * cell edge is at least the largest diameter, so every touching partner is
 * among them).  Writes them to out and returns their number. */
static int64_t orc_candidates(const orc_params *p, int64_t n, const double *x, const orc_cells *cl, int64_t i,
                              int64_t *out)
{
    double inv_cell = 1.0 / p->cell;
    int32_t ci[3];
    for (int a = 0; a < 3; ++a) ci[a] = orc_cell_coord(x[a * n + i], inv_cell, p->nc[a]);
    int64_t cnt = 0;
    for (int32_t cz = ci[2] - 1; cz <= ci[2] + 1; ++cz)
        for (int32_t cy = ci[1] - 1; cy <= ci[1] + 1; ++cy)
            for (int32_t cx = ci[0] - 1; cx <= ci[0] + 1; ++cx) {
                if (cx < 0 || cy < 0 || cz < 0 || cx >= p->nc[0] || cy >= p->nc[1] || cz >= p->nc[2]) continue;
                uint32_t k = orc_key_of_cell(p, cx, cy, cz);
                for (int32_t q = cl->begin[k]; q < cl->end[k]; ++q)
                    if (cl->order[q] != i) out[cnt++] = cl->order[q];
            }
    return cnt;
}

/* Same pair set as orc_pairs_brute, found through the cell list. */
int64_t orc_pairs_cells(const orc_params *p, int64_t n, const double *x, const double *r, int64_t cap,
                        int32_t *pi, int32_t *pj)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    int64_t cnt = 0;
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)(27 * orc_cells_maxocc(p, &cl) + 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t nc_ = orc_candidates(p, n, x, &cl, i, cand);
        for (int64_t s = 0; s < nc_; ++s) {
            int64_t j = cand[s];
            double dv[3], d2;
            if (j > i && orc_touch(n, x, r, i, j, dv, &d2)) {
                if (cnt < cap) {
                    pi[cnt] = (int32_t)i;
                    pj[cnt] = (int32_t)j;
                }
                ++cnt;
            }
        }
    }
    free(cand);
    orc_cells_free(&cl);
    return cnt;
}

/* Touching partners of sampled granules idx[0..m) through the cell list:
 * the partners of idx[s] go to part[s cap + k] (k < cap, in candidate
 * order), their number to cnt[s]. */
void orc_pairs_sample(const orc_params *p, int64_t n, const double *x, const double *r, int64_t m,
                      const int64_t *idx, int64_t cap, int32_t *part, int32_t *cnt)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    int64_t ccap = 27 * orc_cells_maxocc(p, &cl) + 1;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)ccap);
#pragma omp for schedule(static)
        for (int64_t s = 0; s < m; ++s) {
            int64_t i = idx[s], k = 0;
            int64_t nc_ = orc_candidates(p, n, x, &cl, i, cand);
            for (int64_t t = 0; t < nc_; ++t) {
                double dv[3], d2;
                if (orc_touch(n, x, r, i, cand[t], dv, &d2)) {
                    if (k < cap) part[s * cap + k] = (int32_t)cand[t];
                    ++k;
                }
            }
            cnt[s] = (int32_t)k;
        }
        free(cand);
    }
    orc_cells_free(&cl);
}

/* ------------------------------------------------------------------------ */
/* Pair force, Eq. (1a)-(1c) with the dashpot reading                        */
/* ------------------------------------------------------------------------ */

/* Force on the first partner of a touching pair.
 *   nh     : unit normal x_ij / d (from the partner to this granule)
 *   delta  : overlap (r_i + r_j) - d  (> 0)
 *   w      : relative velocity v_i - v_j
 *   meff   : effective mass m_i m_j / (m_i + m_j) (m_i for a wall)
 * Writes the force; returns 1 if the tangential force was capped (sliding). */
static int orc_pair_force(const orc_params *p, double zeta, const double nh[3], double delta,
                          const double w[3], double meff, double F[3])
{
    double gam = 2.0 * zeta * sqrt(meff * p->kn);
    double kt = p->kt_ratio * gam;
    double vn = (w[0] * nh[0] + w[1] * nh[1]) + w[2] * nh[2];
    double fn = p->kn * delta - gam * vn; /* Eq. (1a) + dashpot */
    double ft[3];
    for (int a = 0; a < 3; ++a) ft[a] = -kt * (w[a] - vn * nh[a]); /* Eq. (1c) */
    double fts = sqrt((ft[0] * ft[0] + ft[1] * ft[1]) + ft[2] * ft[2]);
    double cap = p->mu * (p->kn * delta); /* Eq. (1b): ||F_n|| tan(phi) */
    int slide = fts > cap;
    double s = slide ? cap / fts : 1.0;
    for (int a = 0; a < 3; ++a) F[a] = fn * nh[a] + (slide ? ft[a] * s : ft[a]);
    return slide;
}

/* Contact force of granule i with every touching granule (cell list) and
 * every enabled wall.  Fabs[i] (optional) = sum of the norms of the pair and
 * wall forces, the scale of the sum's rounding error. */
static void orc_contact_one(const orc_params *p, double zeta, int64_t n, const double *x, const double *v,
                            const double *r, const double *mass, const orc_cells *cl, int64_t i, int64_t *cand,
                            double Fi[3], double *fabs_i, int32_t *ncont, int32_t *nslide)
{
    /* mass: per-granule masses (wet granules, Eq. 19), NULL for rho_s V */
    double mi = mass ? mass[i] : orc_mass(p, r[i]);
    double acc[3] = {0.0, 0.0, 0.0};
    double sabs = 0.0;
    int32_t nc_ = 0, ns_ = 0;
    int64_t ncand = orc_candidates(p, n, x, cl, i, cand);
    for (int64_t s = 0; s < ncand; ++s) {
        int64_t j = cand[s];
        double dv[3], d2;
        if (!orc_touch(n, x, r, i, j, dv, &d2)) continue;
        if (d2 == 0.0) continue; /* coincident centres: no normal, no force */
        double d = sqrt(d2);
        double nh[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
        double delta = (r[i] + r[j]) - d;
        double w[3] = {v[i] - v[j], v[n + i] - v[n + j], v[2 * n + i] - v[2 * n + j]};
        double mj = mass ? mass[j] : orc_mass(p, r[j]);
        double meff = (mi * mj) / (mi + mj);
        double F[3];
        ns_ += orc_pair_force(p, zeta, nh, delta, w, meff, F);
        ++nc_;
        for (int a = 0; a < 3; ++a) acc[a] += F[a];
        sabs += sqrt((F[0] * F[0] + F[1] * F[1]) + F[2] * F[2]);
    }
    for (int a = 0; a < 3; ++a) {
        double L = (double)p->n[a] * p->dx;
        for (int side = 0; side < 2; ++side) {
            if (!(p->walls & (1u << (2 * a + side)))) continue;
            double xa = x[a * n + i];
            double dist = side == 0 ? xa : L - xa;
            double delta = r[i] - dist;
            if (!(delta > 0.0)) continue;
            double nh[3] = {0.0, 0.0, 0.0};
            nh[a] = side == 0 ? 1.0 : -1.0;
            double w[3] = {v[i], v[n + i], v[2 * n + i]};
            double F[3];
            ns_ += orc_pair_force(p, zeta, nh, delta, w, mi, F);
            ++nc_;
            for (int b = 0; b < 3; ++b) acc[b] += F[b];
            sabs += sqrt((F[0] * F[0] + F[1] * F[1]) + F[2] * F[2]);
        }
    }
    for (int a = 0; a < 3; ++a) Fi[a] = acc[a];
    if (fabs_i) *fabs_i = sabs;
    if (ncont) *ncont = nc_;
    if (nslide) *nslide = ns_;
}

/* F (3n, SoA) = contact force per granule; fabs, ncont, nslide optional. */
void orc_contact_forces(const orc_params *p, int64_t n, const double *x, const double *v, const double *r,
                        double *F, double *fabs_out, int32_t *ncont, int32_t *nslide)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    double zeta = orc_zeta(p->restitution);
    int64_t cap = 27 * orc_cells_maxocc(p, &cl) + 1;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double Fi[3], fa;
            int32_t c1, c2;
            orc_contact_one(p, zeta, n, x, v, r, NULL, &cl, i, cand, Fi, &fa, &c1, &c2);
            for (int a = 0; a < 3; ++a) F[a * n + i] = Fi[a];
            if (fabs_out) fabs_out[i] = fa;
            if (ncont) ncont[i] = c1;
            if (nslide) nslide[i] = c2;
        }
        free(cand);
    }
    orc_cells_free(&cl);
}

/* Contact force on the granules listed in idx[0..m) only (sampled parity at
 * sizes where the full oracle would be slow). */
void orc_contact_forces_sample(const orc_params *p, int64_t n, const double *x, const double *v,
                               const double *r, int64_t m, const int64_t *idx, double *F, double *fabs_out)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    double zeta = orc_zeta(p->restitution);
    int64_t cap = 27 * orc_cells_maxocc(p, &cl) + 1;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t s = 0; s < m; ++s) {
            double Fi[3], fa;
            orc_contact_one(p, zeta, n, x, v, r, NULL, &cl, idx[s], cand, Fi, &fa, NULL, NULL);
            for (int a = 0; a < 3; ++a) F[a * m + s] = Fi[a];
            if (fabs_out) fabs_out[s] = fa;
        }
        free(cand);
    }
    orc_cells_free(&cl);
}

/* Force of one pair, exposed for the closed-form and antisymmetry pins.
 * xi, xj, vi, vj: 3-vectors; returns 0 if the pair does not touch. */
int orc_pair(const orc_params *p, const double *xi, const double *xj, const double *vi, const double *vj,
             double ri, double rj, double *F, int32_t *slide)
{
    double X[6] = {xi[0], xj[0], xi[1], xj[1], xi[2], xj[2]};
    double R2[2] = {ri, rj};
    double dv[3], d2;
    if (!orc_touch(2, X, R2, 0, 1, dv, &d2) || d2 == 0.0) {
        F[0] = F[1] = F[2] = 0.0;
        if (slide) *slide = 0;
        return 0;
    }
    double d = sqrt(d2);
    double nh[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
    double w[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
    double mi = orc_mass(p, ri), mj = orc_mass(p, rj);
    int s = orc_pair_force(p, orc_zeta(p->restitution), nh, (ri + rj) - d, w, (mi * mj) / (mi + mj), F);
    if (slide) *slide = s;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Quadratic B-spline stencil on cell-centred nodes (Sec. 5.1, Eq. 7a)        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t node[3][3]; /* node index per axis and stencil slot, folded into range */
    double w[3][3];     /* 1-D weights */
    double dw[3][3];    /* d w / d x (per metre) */
} orc_stencil;

/* Node i sits at (i + 1/2) dx.  t = x/dx; base = floor(t - 1); f = t - base -
 * 1/2 in [1/2, 3/2) is the distance from the first node.  Weights of the
 * quadratic B-spline at distances f, |f-1|, 2-f. */
static void orc_stencil_of(const orc_params *p, double inv_dx, const double xa[3], orc_stencil *s)
{
    for (int a = 0; a < 3; ++a) {
        double t = xa[a] * inv_dx;
        double fb = floor(t - 1.0);
        double f = (t - fb) - 0.5;
        double c0 = 1.5 - f, c1 = f - 1.0, c2 = f - 0.5;
        s->w[a][0] = 0.5 * (c0 * c0);
        s->w[a][1] = 0.75 - c1 * c1;
        s->w[a][2] = 0.5 * (c2 * c2);
        s->dw[a][0] = -c0 * inv_dx;
        s->dw[a][1] = (-2.0 * c1) * inv_dx;
        s->dw[a][2] = c2 * inv_dx;
        /* fold out-of-range nodes onto the edge node */
        double lo = -2.0, hi = (double)p->n[a];
        if (!(fb >= lo)) fb = lo; /* also catches NaN */
        if (fb > hi) fb = hi;
        int32_t b = (int32_t)fb;
        for (int k = 0; k < 3; ++k) {
            int32_t id = b + k;
            if (id < 0) id = 0;
            if (id > p->n[a] - 1) id = p->n[a] - 1;
            s->node[a][k] = id;
        }
    }
}

static int64_t orc_node_index(const orc_params *p, const orc_stencil *s, int a, int b, int c)
{
    return (int64_t)s->node[0][a] + (int64_t)p->n[0] * ((int64_t)s->node[1][b] + (int64_t)p->n[1] * s->node[2][c]);
}

static void orc_pos(int64_t n, const double *x, int64_t i, double xa[3])
{
    xa[0] = x[i];
    xa[1] = x[n + i];
    xa[2] = x[2 * n + i];
}

/* Weights of one granule's stencil, exposed for the B-spline pins:
 * w27[(c*3+b)*3+a] = (wx[a] wy[b]) wz[c], node27 the flat node index. */
void orc_stencil27(const orc_params *p, const double *xa, double *w27, int64_t *node27, double *w1d)
{
    orc_stencil s;
    orc_stencil_of(p, 1.0 / p->dx, xa, &s);
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                int k = (c * 3 + b) * 3 + a;
                w27[k] = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                node27[k] = orc_node_index(p, &s, a, b, c);
            }
    if (w1d)
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 3; ++k) w1d[a * 3 + k] = s.w[a][k];
}

/* ------------------------------------------------------------------------ */
/* P2G: Eq. (7a) volume fraction and granule momentum                        */
/* ------------------------------------------------------------------------ */

/* Nearest integer (ties to even) to the exact product a b, for |a b| <
 * 2^51: a b + M with M = 1.5 2^52 lies in [2^52, 2^53), where doubles are the
 * integers, so the single rounding of the fused multiply-add rounds a b
 * itself; subtracting M is exact.  (Rounding the double product a b first
 * and then to an integer can differ by one where a b lies within half a
 * double ulp of a half-integer.) */
static int64_t orc_round_product(double a, double b)
{
    const double M = 6755399441055744.0; /* 1.5 * 2^52 */
    return (int64_t)(fma(a, b, M) - M);
}

/* exposed for the rounding pin */
int64_t orc_round_product_x(double a, double b) { return orc_round_product(a, b); }

/* Fixed point.  alpha in units of 2^-32 cell volumes; momentum in units of
 * 2^-32 rho_s dx^3 (1 m/s).  Per granule and channel the target total is
 * Q = rint(S) with S = frac * 2^32 (alpha) or (frac * v_c) * 2^32 (momentum),
 * frac = V_i / dx^3.  The 26 outer nodes take w S rounded once to the
 * nearest integer (orc_round_product, w the double weight of the node); the
 * centre node takes Q minus their sum.  Adds into alpha (G) and mom (3G). */
/* Scaled totals S of one granule: fraction, then the three momentum
 * channels. */
static void orc_p2g_totals(const orc_params *p, double inv_vcell, double rho_0, double r, double held, int wet,
                           const double va[3], double S[4])
{
    double frac = orc_volume(r) * inv_vcell;
    /* a wet granule's absorbed water counts as extra volume in alpha_s
     * (Sec. 5.3): frac (1 + held) = frac + frac held (held = 0: frac) */
    double fa = wet ? frac + frac * held : frac;
    /* momentum in rho_s dx^3 units: a wet granule carries m_wet / (rho_s dx^3)
     * = frac (rho_s + held rho_0) / rho_s = frac + frac held rho_0 / rho_s
     * per unit velocity (Eq. 19), written so that held = 0 gives frac exactly */
    double fm = wet ? frac + (frac * (held * rho_0)) / p->rho_s : frac;
    S[0] = fa * ORC_TWO32;
    for (int c = 0; c < 3; ++c) S[1 + c] = (fm * va[c]) * ORC_TWO32;
}

/* exposed for the rounding pin: the dry totals of one granule */
void orc_p2g_totals_x(const orc_params *p, double r, const double *va, double *S)
{
    orc_p2g_totals(p, 1.0 / ((p->dx * p->dx) * p->dx), 0.0, r, 0.0, 0, va, S);
}

static void orc_p2g_fixed_held(const orc_params *p, double rho_0, int64_t n, const double *x, const double *v,
                               const double *r, const double *held, int64_t *alpha, int64_t *mom)
{
    double inv_dx = 1.0 / p->dx;
    double inv_vcell = 1.0 / ((p->dx * p->dx) * p->dx);
    int64_t G = orc_nodes(p);
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        const double va[3] = {v[i], v[n + i], v[2 * n + i]};
        double S[4];
        orc_p2g_totals(p, inv_vcell, rho_0, r[i], held ? held[i] : 0.0, held != NULL, va, S);
        for (int ch = 0; ch < 4; ++ch) {
            int64_t Q = llrint(S[ch]);
            int64_t rest = Q;
            int64_t *dst = ch == 0 ? alpha : mom + (int64_t)(ch - 1) * G;
            for (int c = 0; c < 3; ++c)
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) {
                        if (a == 1 && b == 1 && c == 1) continue;
                        double w = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                        int64_t q = orc_round_product(w, S[ch]);
                        rest -= q;
                        dst[orc_node_index(p, &s, a, b, c)] += q;
                    }
            dst[orc_node_index(p, &s, 1, 1, 1)] += rest;
        }
    }
}

void orc_p2g_fixed(const orc_params *p, int64_t n, const double *x, const double *v, const double *r,
                   int64_t *alpha, int64_t *mom)
{
    orc_p2g_fixed_held(p, 0.0, n, x, v, r, NULL, alpha, mom);
}

/* Unquantised P2G for the differentiable form: alpha in cell volumes
 * (sum_i w frac_i), momentum in kg m/s (sum_i w m_i v_i). */
void orc_p2g_real(const orc_params *p, int64_t n, const double *x, const double *v, const double *r,
                  double *alpha, double *mom)
{
    double inv_dx = 1.0 / p->dx;
    double inv_vcell = 1.0 / ((p->dx * p->dx) * p->dx);
    int64_t G = orc_nodes(p);
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        double frac = orc_volume(r[i]) * inv_vcell;
        double m = orc_mass(p, r[i]);
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    double w = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                    int64_t k = orc_node_index(p, &s, a, b, c);
                    if (alpha) alpha[k] += w * frac;
                    if (mom)
                        for (int d = 0; d < 3; ++d) mom[d * G + k] += w * (m * v[d * n + i]);
                }
    }
}

/* ------------------------------------------------------------------------ */
/* G2P of fluid velocity and volume fraction (Sec. 5.2; Sec. 5.1 clamp)       */
/* ------------------------------------------------------------------------ */

/* u_at (3n) = sum_k w u_k; alpha_f (n) = 1 - sum_k w min(alpha_k, amax), amax
 * the clamp of orc_alpha_clamp.
 * The alpha grid is either fixed point (alpha_fx, 2^-32 units) or real
 * (alpha_real, cell volumes); exactly one is non-NULL. */
void orc_g2p(const orc_params *p, int64_t n, const double *x, const double *u, const int64_t *alpha_fx,
             const double *alpha_real, double *u_at, double *alpha_f)
{
    double inv_dx = 1.0 / p->dx;
    double amax = orc_alpha_clamp(p);
    int64_t G = orc_nodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        double acc[3] = {0.0, 0.0, 0.0}, as = 0.0;
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    double w = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                    int64_t k = orc_node_index(p, &s, a, b, c);
                    for (int d = 0; d < 3; ++d) acc[d] += w * u[d * G + k];
                    double al = alpha_fx ? (double)alpha_fx[k] * ORC_TWOM32 : alpha_real[k];
                    if (al > amax) al = amax;
                    as += w * al;
                }
        for (int d = 0; d < 3; ++d) u_at[d * n + i] = acc[d];
        alpha_f[i] = 1.0 - as;
    }
}

/* ------------------------------------------------------------------------ */
/* Drag (Eq. 5b / App. A, Stokes form scaled by alpha_f) and integration      */
/* ------------------------------------------------------------------------ */

void orc_drag(const orc_params *p, int64_t n, const double *r, const double *v, const double *u_at,
              const double *alpha_f, double *Fd)
{
    double cdrag = (p->c_drag * ORC_C6PI) * p->eta_f;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double beta = (cdrag * r[i]) * alpha_f[i];
        for (int d = 0; d < 3; ++d) Fd[d * n + i] = beta * (u_at[d * n + i] - v[d * n + i]);
    }
}

/* Semi-implicit (symplectic) Euler: v += dt ((Fc + Fd)/m + g); x += dt v. */
void orc_integrate(const orc_params *p, int64_t n, const double *r, const double *Fc, const double *Fd,
                   double *x, double *v)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double m = orc_mass(p, r[i]);
        for (int d = 0; d < 3; ++d) {
            double a = (Fc[d * n + i] + Fd[d * n + i]) / m + p->g[d];
            v[d * n + i] = v[d * n + i] + p->dt * a;
            x[d * n + i] = x[d * n + i] + p->dt * v[d * n + i];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* One step of the granule path (Alg. 2, one sub-step)                       */
/* ------------------------------------------------------------------------ */

/* In: x, v (x^n, v^n), r, u grid (3G), alpha_fx = P2G(x^n) (G, fixed point).
 * Out: x, v = x^{n+1}, v^{n+1}; alpha_fx, mom_fx = P2G(x^{n+1}, v^{n+1});
 * Fc, Fd, u_at, alpha_f (optional, may be NULL) the intermediates. */
void orc_step(const orc_params *p, int64_t n, double *x, double *v, const double *r, const double *u,
              int64_t *alpha_fx, int64_t *mom_fx, double *Fc_out, double *Fd_out, double *uat_out,
              double *af_out)
{
    int64_t G = orc_nodes(p);
    double *Fc = Fc_out ? Fc_out : (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *Fd = Fd_out ? Fd_out : (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *uat = uat_out ? uat_out : (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *af = af_out ? af_out : (double *)malloc(sizeof(double) * (size_t)n);
    orc_g2p(p, n, x, u, alpha_fx, NULL, uat, af);
    orc_drag(p, n, r, v, uat, af, Fd);
    orc_contact_forces(p, n, x, v, r, Fc, NULL, NULL, NULL);
    orc_integrate(p, n, r, Fc, Fd, x, v);
    memset(alpha_fx, 0, sizeof(int64_t) * (size_t)G);
    memset(mom_fx, 0, sizeof(int64_t) * 3 * (size_t)G);
    orc_p2g_fixed(p, n, x, v, r, alpha_fx, mom_fx);
    if (!Fc_out) free(Fc);
    if (!Fd_out) free(Fd);
    if (!uat_out) free(uat);
    if (!af_out) free(af);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ======================================================================== */
/* Differentiable form: unquantised rollout and its reverse pass             */
/* ======================================================================== */
/*
 * Forward (one step, x^n -> x^{n+1}):
 *   A^n = P2G_alpha(x^n) (real);  (u_at, alpha_f) = G2P(x^n; u, A^n);
 *   F_d = C_d 6 pi eta r alpha_f (u_at - v^n);  F_c = contact(x^n, v^n; mu);
 *   v^{n+1} = v^n + dt ((F_c + F_d)/m + g);  x^{n+1} = x^n + dt v^{n+1}.
 * Loss L = sum_k |P_k|^2 with P = P2G_momentum(x^T, v^T) in kg m/s.
 * The reverse pass below is written by hand, step by step, from these
 * definitions; the alpha clamp and the Coulomb cap take the derivative of the
 * branch taken (the clamp's derivative is 0 at and above alpha_max).
 */

/* Reverse of orc_pair_force.  gbar: cotangent of the force on the first
 * partner; gmu: cotangent used for the mu derivative.  Adds to nbar[3],
 * *dbar (overlap), wbar[3] (relative velocity) and *mubar. */
static void orc_pair_force_vjp(const orc_params *p, double zeta, const double nh[3], double delta,
                               const double w[3], double meff, const double gbar[3], const double gmu[3],
                               double nbar[3], double *dbar, double wbar[3], double *mubar)
{
    double gam = 2.0 * zeta * sqrt(meff * p->kn);
    double kt = p->kt_ratio * gam;
    double vn = (w[0] * nh[0] + w[1] * nh[1]) + w[2] * nh[2];
    double fn = p->kn * delta - gam * vn;
    double t[3], ft[3];
    for (int a = 0; a < 3; ++a) {
        t[a] = w[a] - vn * nh[a];
        ft[a] = -kt * t[a];
    }
    double s = sqrt((ft[0] * ft[0] + ft[1] * ft[1]) + ft[2] * ft[2]);
    double cap = p->mu * (p->kn * delta);
    int slide = s > cap;
    /* F = fn n + F_t */
    double fnbar = (gbar[0] * nh[0] + gbar[1] * nh[1]) + gbar[2] * nh[2];
    for (int a = 0; a < 3; ++a) nbar[a] += fn * gbar[a];
    double ftbar[3];
    if (slide) {
        /* F_t = cap ft / s */
        double fh[3] = {ft[0] / s, ft[1] / s, ft[2] / s};
        double gdotf = (gbar[0] * fh[0] + gbar[1] * fh[1]) + gbar[2] * fh[2];
        double capbar = gdotf;
        for (int a = 0; a < 3; ++a) ftbar[a] = (cap / s) * (gbar[a] - gdotf * fh[a]);
        *dbar += capbar * p->mu * p->kn;
        double gmudotf = (gmu[0] * fh[0] + gmu[1] * fh[1]) + gmu[2] * fh[2];
        *mubar += gmudotf * p->kn * delta;
    } else {
        for (int a = 0; a < 3; ++a) ftbar[a] = gbar[a];
    }
    /* ft = -kt t, t = w - vn n */
    double tbar[3];
    for (int a = 0; a < 3; ++a) tbar[a] = -kt * ftbar[a];
    double vnbar = -((tbar[0] * nh[0] + tbar[1] * nh[1]) + tbar[2] * nh[2]);
    for (int a = 0; a < 3; ++a) {
        wbar[a] += tbar[a];
        nbar[a] += -vn * tbar[a];
    }
    /* fn = kn delta - gam vn */
    *dbar += p->kn * fnbar;
    vnbar += -gam * fnbar;
    /* vn = w . n */
    for (int a = 0; a < 3; ++a) {
        wbar[a] += vnbar * nh[a];
        nbar[a] += vnbar * w[a];
    }
}

/* VJP of the contact forces: given gF (3n) = dL/dF_c, adds dL/dx (gx),
 * dL/dv (gv) and dL/dmu (*gmu).  Gather form: granule i collects, for every
 * touching partner j, the pair term with cotangent gF_i - gF_j. */
void orc_contact_vjp(const orc_params *p, int64_t n, const double *x, const double *v, const double *r,
                     const double *gF, double *gx, double *gv, double *gmu)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    double zeta = orc_zeta(p->restitution);
    int64_t cap = 27 * orc_cells_maxocc(p, &cl) + 1;
    double mu_acc = 0.0;
#pragma omp parallel reduction(+ : mu_acc)
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double mi = orc_mass(p, r[i]);
            double gxi[3] = {0, 0, 0}, gvi[3] = {0, 0, 0};
            double gFi[3] = {gF[i], gF[n + i], gF[2 * n + i]};
            int64_t nc_ = orc_candidates(p, n, x, &cl, i, cand);
            for (int64_t s = 0; s < nc_; ++s) {
                int64_t j = cand[s];
                double dv[3], d2;
                if (!orc_touch(n, x, r, i, j, dv, &d2) || d2 == 0.0) continue;
                double d = sqrt(d2);
                double nh[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
                double delta = (r[i] + r[j]) - d;
                double w[3] = {v[i] - v[j], v[n + i] - v[n + j], v[2 * n + i] - v[2 * n + j]};
                double mj = orc_mass(p, r[j]);
                double meff = (mi * mj) / (mi + mj);
                double gbar[3] = {gFi[0] - gF[j], gFi[1] - gF[n + j], gFi[2] - gF[2 * n + j]};
                double nbar[3] = {0, 0, 0}, wbar[3] = {0, 0, 0}, dbar = 0.0, mubar = 0.0;
                orc_pair_force_vjp(p, zeta, nh, delta, w, meff, gbar, gFi, nbar, &dbar, wbar, &mubar);
                /* n = dv / d, delta = R - d, d = |dv| */
                double ndotn = (nbar[0] * nh[0] + nbar[1] * nh[1]) + nbar[2] * nh[2];
                for (int a = 0; a < 3; ++a) {
                    gxi[a] += (nbar[a] - ndotn * nh[a]) / d - dbar * nh[a];
                    gvi[a] += wbar[a];
                }
                mu_acc += mubar;
            }
            for (int a = 0; a < 3; ++a) {
                double L = (double)p->n[a] * p->dx;
                for (int side = 0; side < 2; ++side) {
                    if (!(p->walls & (1u << (2 * a + side)))) continue;
                    double xa = x[a * n + i];
                    double dist = side == 0 ? xa : L - xa;
                    double delta = r[i] - dist;
                    if (!(delta > 0.0)) continue;
                    double nh[3] = {0.0, 0.0, 0.0};
                    nh[a] = side == 0 ? 1.0 : -1.0;
                    double w[3] = {v[i], v[n + i], v[2 * n + i]};
                    double nbar[3] = {0, 0, 0}, wbar[3] = {0, 0, 0}, dbar = 0.0, mubar = 0.0;
                    orc_pair_force_vjp(p, zeta, nh, delta, w, mi, gFi, gFi, nbar, &dbar, wbar, &mubar);
                    /* delta = r - x_a (low face) or r - (L - x_a) (high face) */
                    gxi[a] += side == 0 ? -dbar : dbar;
                    for (int b = 0; b < 3; ++b) gvi[b] += wbar[b];
                    mu_acc += mubar;
                }
            }
            for (int a = 0; a < 3; ++a) {
                gx[a * n + i] += gxi[a];
                gv[a * n + i] += gvi[a];
            }
        }
        free(cand);
    }
    *gmu += mu_acc;
    orc_cells_free(&cl);
}

/* VJP of the drag F_d = beta alpha_f (u_at - v), beta = C_d 6 pi eta r:
 * gv += -beta alpha_f gF; guat = beta alpha_f gF; gaf = beta (u_at - v).gF;
 * *gcd += (F_d / C_d) . gF. */
void orc_drag_vjp(const orc_params *p, int64_t n, const double *r, const double *v, const double *uat,
                  const double *af, const double *gF, double *gv, double *guat, double *gaf, double *gcd)
{
    double c = ORC_C6PI * p->eta_f;
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double beta = (p->c_drag * c) * r[i];
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
            double g = gF[d * n + i];
            double slip = uat[d * n + i] - v[d * n + i];
            gv[d * n + i] += -beta * af[i] * g;
            guat[d * n + i] = beta * af[i] * g;
            s += slip * g;
        }
        gaf[i] = beta * s;
        acc += (c * r[i]) * af[i] * s;
    }
    *gcd += acc;
}

/* VJP of G2P with a real alpha grid: given guat (3n) and gaf (n), adds
 * dL/dx to gx and dL/dA to galpha (G). */
void orc_g2p_vjp(const orc_params *p, int64_t n, const double *x, const double *u, const double *alpha,
                 const double *guat, const double *gaf, double *gx, double *galpha)
{
    double inv_dx = 1.0 / p->dx;
    int64_t G = orc_nodes(p);
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    int64_t k = orc_node_index(p, &s, a, b, c);
                    double w = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                    double gw[3] = {(s.dw[0][a] * s.w[1][b]) * s.w[2][c], (s.w[0][a] * s.dw[1][b]) * s.w[2][c],
                                    (s.w[0][a] * s.w[1][b]) * s.dw[2][c]};
                    double ul = (u[k] * guat[i] + u[G + k] * guat[n + i]) + u[2 * G + k] * guat[2 * n + i];
                    int clamped = !(alpha[k] < orc_alpha_clamp(p));
                    double al = clamped ? orc_alpha_clamp(p) : alpha[k];
                    /* alpha_f = 1 - sum w al */
                    double coef = ul - al * gaf[i];
                    for (int d = 0; d < 3; ++d) gx[d * n + i] += gw[d] * coef;
                    if (!clamped) galpha[k] += -w * gaf[i];
                }
    }
}

/* VJP of the real P2G: alpha_k = sum_i w_ik frac_i, P_k = sum_i w_ik m_i v_i.
 * Given galpha (G, may be NULL) and gmom (3G, may be NULL), adds to gx, gv. */
void orc_p2g_vjp(const orc_params *p, int64_t n, const double *x, const double *v, const double *r,
                 const double *galpha, const double *gmom, double *gx, double *gv)
{
    double inv_dx = 1.0 / p->dx;
    double inv_vcell = 1.0 / ((p->dx * p->dx) * p->dx);
    int64_t G = orc_nodes(p);
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        double frac = orc_volume(r[i]) * inv_vcell;
        double m = orc_mass(p, r[i]);
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    int64_t k = orc_node_index(p, &s, a, b, c);
                    double w = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                    double gw[3] = {(s.dw[0][a] * s.w[1][b]) * s.w[2][c], (s.w[0][a] * s.dw[1][b]) * s.w[2][c],
                                    (s.w[0][a] * s.w[1][b]) * s.dw[2][c]};
                    double coef = 0.0;
                    if (galpha) coef += galpha[k] * frac;
                    if (gmom) {
                        double pv = (gmom[k] * v[i] + gmom[G + k] * v[n + i]) + gmom[2 * G + k] * v[2 * n + i];
                        coef += m * pv;
                        for (int d = 0; d < 3; ++d) gv[d * n + i] += m * w * gmom[d * G + k];
                    }
                    for (int d = 0; d < 3; ++d) gx[d * n + i] += gw[d] * coef;
                }
    }
}

static uint64_t orc_fnv(uint64_t h, const int32_t *a, int64_t m)
{
    for (int64_t i = 0; i < m; ++i) {
        h ^= (uint64_t)(uint32_t)a[i];
        h *= 1099511628211ull;
    }
    return h;
}

/* Nodes read by G2P of granule i at or above the clamp, per granule. */
static void orc_clamp_counts(const orc_params *p, int64_t n, const double *x, const double *alpha, int32_t *cnt)
{
    double inv_dx = 1.0 / p->dx;
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        int32_t c_ = 0;
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) c_ += !(alpha[orc_node_index(p, &s, a, b, c)] < orc_alpha_clamp(p));
        cnt[i] = c_;
    }
}

/* One real-mode step in place; intermediates to the given buffers; the
 * signature (if non-NULL) hashes the contact, sliding and clamp counts. */
static void orc_step_real(const orc_params *p, int64_t n, double *x, double *v, const double *r, const double *u,
                          double *A, double *uat, double *af, double *Fd, double *Fc, int32_t *i1, int32_t *i2,
                          uint64_t *sig)
{
    int64_t G = orc_nodes(p);
    memset(A, 0, sizeof(double) * (size_t)G);
    orc_p2g_real(p, n, x, v, r, A, NULL);
    orc_g2p(p, n, x, u, NULL, A, uat, af);
    orc_drag(p, n, r, v, uat, af, Fd);
    orc_contact_forces(p, n, x, v, r, Fc, NULL, i1, i2);
    if (sig) {
        *sig = orc_fnv(*sig, i1, n);
        *sig = orc_fnv(*sig, i2, n);
        orc_clamp_counts(p, n, x, A, i1);
        *sig = orc_fnv(*sig, i1, n);
    }
    orc_integrate(p, n, r, Fc, Fd, x, v);
}

/* Real-mode rollout of `steps` steps from (x0, v0); returns L = sum |P|^2 of
 * the final momentum grid (written to mom_out, 3G, if non-NULL); *sig (if
 * non-NULL) receives a hash of the contact, sliding and clamp sets. */
double orc_rollout(const orc_params *p, int64_t n, const double *x0, const double *v0, const double *r,
                   const double *u, int32_t steps, double *mom_out, uint64_t *sig)
{
    int64_t G = orc_nodes(p);
    size_t n3 = sizeof(double) * 3 * (size_t)n;
    double *x = (double *)malloc(n3), *v = (double *)malloc(n3);
    memcpy(x, x0, n3);
    memcpy(v, v0, n3);
    double *A = (double *)malloc(sizeof(double) * (size_t)G);
    double *uat = (double *)malloc(n3), *Fd = (double *)malloc(n3), *Fc = (double *)malloc(n3);
    double *af = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t *i1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *i2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (sig) *sig = 1469598103934665603ull;
    for (int32_t s = 0; s < steps; ++s) orc_step_real(p, n, x, v, r, u, A, uat, af, Fd, Fc, i1, i2, sig);
    double *P = (double *)calloc((size_t)(3 * G), sizeof(double));
    orc_p2g_real(p, n, x, v, r, NULL, P);
    double L = 0.0;
    for (int64_t k = 0; k < 3 * G; ++k) L += P[k] * P[k];
    if (mom_out) memcpy(mom_out, P, sizeof(double) * 3 * (size_t)G);
    free(x); free(v); free(A); free(uat); free(Fd); free(Fc); free(af); free(i1); free(i2); free(P);
    return L;
}

/* Reverse pass of orc_rollout: returns L and writes dL/dv0 (3n), adds
 * dL/dmu and dL/dC_d.  The whole trajectory is stored (no checkpoints). */
double orc_rollout_vjp(const orc_params *p, int64_t n, const double *x0, const double *v0, const double *r,
                       const double *u, int32_t steps, double *gv0, double *gmu, double *gcd)
{
    int64_t G = orc_nodes(p);
    size_t n3 = sizeof(double) * 3 * (size_t)n;
    size_t n1 = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *X = (double *)malloc(n3 * (size_t)(steps + 1)), *V = (double *)malloc(n3 * (size_t)(steps + 1));
    memcpy(X, x0, n3);
    memcpy(V, v0, n3);
    double *A = (double *)malloc(sizeof(double) * (size_t)G);
    double *uat = (double *)malloc(n3), *Fd = (double *)malloc(n3), *Fc = (double *)malloc(n3);
    double *af = (double *)malloc(n1);
    int32_t *i1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *i2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t s = 0; s < steps; ++s) {
        memcpy(X + (size_t)(s + 1) * 3 * n, X + (size_t)s * 3 * n, n3);
        memcpy(V + (size_t)(s + 1) * 3 * n, V + (size_t)s * 3 * n, n3);
        orc_step_real(p, n, X + (size_t)(s + 1) * 3 * n, V + (size_t)(s + 1) * 3 * n, r, u, A, uat, af, Fd, Fc, i1,
                      i2, NULL);
    }
    double *xT = X + (size_t)steps * 3 * n, *vT = V + (size_t)steps * 3 * n;
    double *P = (double *)calloc((size_t)(3 * G), sizeof(double));
    orc_p2g_real(p, n, xT, vT, r, NULL, P);
    double L = 0.0;
    for (int64_t k = 0; k < 3 * G; ++k) {
        L += P[k] * P[k];
        P[k] *= 2.0; /* dL/dP */
    }
    double *gx = (double *)calloc((size_t)(3 * n), sizeof(double));
    double *gv = (double *)calloc((size_t)(3 * n), sizeof(double));
    orc_p2g_vjp(p, n, xT, vT, r, NULL, P, gx, gv);
    double *gF = (double *)malloc(n3), *guat = (double *)malloc(n3), *gaf = (double *)malloc(n1);
    double *galpha = (double *)malloc(sizeof(double) * (size_t)G);
    for (int32_t s = steps - 1; s >= 0; --s) {
        double *x = X + (size_t)s * 3 * n, *v = V + (size_t)s * 3 * n;
        memset(A, 0, sizeof(double) * (size_t)G);
        orc_p2g_real(p, n, x, v, r, A, NULL);
        orc_g2p(p, n, x, u, NULL, A, uat, af);
        /* x^{s+1} = x^s + dt v^{s+1};  v^{s+1} = v^s + dt (F/m + g) */
        for (int64_t i = 0; i < n; ++i) {
            double m = orc_mass(p, r[i]);
            for (int d = 0; d < 3; ++d) {
                gv[d * n + i] += p->dt * gx[d * n + i];
                gF[d * n + i] = (p->dt / m) * gv[d * n + i];
            }
        }
        orc_contact_vjp(p, n, x, v, r, gF, gx, gv, gmu);
        orc_drag_vjp(p, n, r, v, uat, af, gF, gv, guat, gaf, gcd);
        memset(galpha, 0, sizeof(double) * (size_t)G);
        orc_g2p_vjp(p, n, x, u, A, guat, gaf, gx, galpha);
        orc_p2g_vjp(p, n, x, v, r, galpha, NULL, gx, gv);
    }
    memcpy(gv0, gv, n3);
    free(X); free(V); free(A); free(uat); free(Fd); free(Fc); free(af); free(i1); free(i2); free(P);
    free(gx); free(gv); free(gF); free(guat); free(gaf); free(galpha);
    return L;
}

/* ======================================================================== */
/* Remaining interphase forces and the full sand step                        */
/* ======================================================================== */
/*
 * Passages followed:
 *   pressure-gradient force . Sec. 3.3 Eq. (5a), F_p = -(4/3) pi r^3 grad p,
 *                             grad p interpolated from the grid (Sec. 5.2)
 *   quadratic drag .......... Sec. 3.3 Eq. (5b), F_d = 12 pi r^2 rho_f C |u - v| (u - v)
 *   virtual mass ............ Sec. 3.3 Eq. (5c) and Sec. 5.2 Eq. (9):
 *                             (m + (2/3) pi r^3 rho_0) dv/dt = (2/3) pi r^3 rho_0 dv_f/dt + F_o,
 *                             dv_f/dt interpolated from the grid (Eq. 10-12: the grid's
 *                             velocity increment)
 *   exchange momentum ....... Sec. 5.2: F_s(x) = -(dt'/dt) sum_i sum_j f_j^i N(x_j^i - x)
 *   sub-step cycle .......... Alg. 1 and 2: N = ceil(dt / dt') sub-steps, fluid fields frozen
 *
 * Readings (recorded in the design notes):
 *   - rho_f of Eq. (5b) and rho_0 of Eq. (9) are the same fluid density;
 *   - the factor written mu in Eq. (5b) is a dimensionless coefficient C
 *     (the product must be a force); the quadratic drag is used as printed,
 *     without the fluid-fraction factor of the linear form;
 *   - the virtual-mass force is F_v = (1/2) rho_f V (a_f - a_s) with
 *     V = (4/3) pi r^3; moving its a_s part to the left of Eq. (9) gives the
 *     effective mass m + (1/2) rho_f V, and gravity acts on m;
 *   - f_j^i of the exchange is the whole fluid force on granule j in
 *     sub-step i: drag + pressure gradient + virtual mass, with a_s the
 *     sub-step's acceleration (F_c + F_fluid + m g) / (m + (1/2) rho_f V);
 *   - a sand step of length dt is cut into N = ceil(dt / dt'_max) equal
 *     sub-steps of dt / N, so each exchange weight dt'/dt is 1/N;
 *   - the exchange grid is int64 fixed point in units of 2^-32 f_unit,
 *     deposited like Eq. (7a): w S rounded once on the 26 outer nodes, the
 *     centre node takes rint(S) minus their sum.
 */

typedef struct {
    double rho_f;       /* fluid density rho_f = rho_0 [kg/m^3]                 */
    double c_quad;      /* dimensionless coefficient of the quadratic drag      */
    double f_unit;      /* exchange-force unit [N]                              */
    int32_t drag_model; /* 0: linear Stokes form x alpha_f; 1: quadratic (5b)   */
    int32_t vmass;      /* 1: virtual mass in the equation of motion (Eq. 9)    */
} orc_coupling;

#define ORC_C12PI (12.0 * ORC_PI)

/* G2P of a 3-vector grid field (3G) to the granules (3n): sum_k w_k f_k. */
static void orc_g2p_vec(const orc_params *p, int64_t n, const double *x, const double *f, double *out)
{
    double inv_dx = 1.0 / p->dx;
    int64_t G = orc_nodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    double w = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                    int64_t k = orc_node_index(p, &s, a, b, c);
                    for (int d = 0; d < 3; ++d) acc[d] += w * f[d * G + k];
                }
        for (int d = 0; d < 3; ++d) out[d * n + i] = acc[d];
    }
}

/* Fluid force on each granule (3n): drag (linear or quadratic) + pressure
 * gradient (if gp) + the explicit virtual-mass term (1/2) rho_f V a_f (if
 * vmass and af).  u, gp, af are 3G grid fields; alpha_fx the fixed-point
 * solid fraction grid (P2G at x).  held (n, or NULL for dry granules): the
 * water a granule holds per unit of its volume, which counts as extra volume
 * in the volume forces (Sec. 5.3): V = (4/3) pi r^3 (1 + held); the drag
 * keeps the granule's radius, which the water does not change. */
void orc_fluid_forces(const orc_params *p, const orc_coupling *cp, int64_t n, const double *x, const double *v,
                      const double *r, const double *held, const double *u, const int64_t *alpha_fx,
                      const double *gp, const double *af, double *Ffl)
{
    double *uat = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *alf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *gpa = gp ? (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1)) : NULL;
    double *afa = (af && cp->vmass) ? (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1)) : NULL;
    orc_g2p(p, n, x, u, alpha_fx, NULL, uat, alf);
    if (gpa) orc_g2p_vec(p, n, x, gp, gpa);
    if (afa) orc_g2p_vec(p, n, x, af, afa);
    if (cp->drag_model == 0) {
        orc_drag(p, n, r, v, uat, alf, Ffl);
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double w[3];
            for (int d = 0; d < 3; ++d) w[d] = uat[d * n + i] - v[d * n + i];
            double sp = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
            double coef = (((ORC_C12PI * r[i]) * r[i]) * cp->rho_f) * cp->c_quad;
            for (int d = 0; d < 3; ++d) Ffl[d * n + i] = (coef * sp) * w[d];
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double V = orc_wet_volume(r[i], held ? held[i] : 0.0);
        double hv = (0.5 * cp->rho_f) * V;
        for (int d = 0; d < 3; ++d) {
            double f = Ffl[d * n + i];
            if (gpa) f = f - V * gpa[d * n + i];
            if (afa) f = f + hv * afa[d * n + i];
            Ffl[d * n + i] = f;
        }
    }
    free(uat);
    free(alf);
    free(gpa);
    free(afa);
}

/* Semi-implicit Euler with the virtual mass of Eq. (9):
 * v += dt ((Fc + Ffl) + m g) / (m + (1/2) rho_f V); x += dt v.
 * Without virtual mass this is orc_integrate. */
void orc_integrate_vm(const orc_params *p, const orc_coupling *cp, int64_t n, const double *r, const double *Fc,
                      const double *Ffl, double *x, double *v)
{
    if (!cp->vmass) {
        orc_integrate(p, n, r, Fc, Ffl, x, v);
        return;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double m = orc_mass(p, r[i]);
        double me = m + (0.5 * cp->rho_f) * orc_volume(r[i]);
        for (int d = 0; d < 3; ++d) {
            double a = ((Fc[d * n + i] + Ffl[d * n + i]) + m * p->g[d]) / me;
            v[d * n + i] = v[d * n + i] + p->dt * a;
            x[d * n + i] = x[d * n + i] + p->dt * v[d * n + i];
        }
    }
}

/* Whole fluid force of the sub-step on each granule (the f_j^i of the
 * exchange): Ffl minus (1/2) rho_f V a_s under virtual mass, where
 * a_s = ((Fc + Ffl) + m g) / (m + (1/2) rho_f V); Ffl otherwise.  held (n,
 * or NULL): wet granules (Sec. 5.3) take the wet mass V (rho_s + held rho_f)
 * of Eq. 19 and the volume V (1 + held). */
void orc_exchange_force(const orc_params *p, const orc_coupling *cp, int64_t n, const double *r,
                        const double *held, const double *Fc, const double *Ffl, double *fex)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double h = held ? held[i] : 0.0;
        double m = held ? orc_volume(r[i]) * (p->rho_s + h * cp->rho_f) : orc_mass(p, r[i]);
        double hv = (0.5 * cp->rho_f) * orc_wet_volume(r[i], h);
        double me = m + hv;
        for (int d = 0; d < 3; ++d) {
            double f = Ffl[d * n + i];
            if (cp->vmass) {
                double as = ((Fc[d * n + i] + f) + m * p->g[d]) / me;
                f = f - hv * as;
            }
            fex[d * n + i] = f;
        }
    }
}

/* Exchange P2G of one sub-step: adds -weight * f_j N(x_j - x) to fs (3G,
 * int64, units of 2^-32 f_unit).  Per granule and component the target total
 * is Q = rint(S), S = (s f) * 2^32 with s = -weight / f_unit; the 26 outer
 * nodes take w S rounded once (orc_round_product), the centre node Q minus
 * their sum. */
void orc_exchange_p2g(const orc_params *p, const orc_coupling *cp, int64_t n, const double *x, const double *r,
                      const double *held, const double *Fc, const double *Ffl, double weight, int64_t *fs)
{
    double inv_dx = 1.0 / p->dx;
    int64_t G = orc_nodes(p);
    double *fex = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    orc_exchange_force(p, cp, n, r, held, Fc, Ffl, fex);
    double sc = -weight / cp->f_unit;
    for (int64_t i = 0; i < n; ++i) {
        double xa[3];
        orc_pos(n, x, i, xa);
        orc_stencil s;
        orc_stencil_of(p, inv_dx, xa, &s);
        for (int ch = 0; ch < 3; ++ch) {
            double S = (sc * fex[ch * n + i]) * ORC_TWO32;
            int64_t Q = llrint(S);
            int64_t rest = Q;
            int64_t *dst = fs + (int64_t)ch * G;
            for (int c = 0; c < 3; ++c)
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) {
                        if (a == 1 && b == 1 && c == 1) continue;
                        double w = (s.w[0][a] * s.w[1][b]) * s.w[2][c];
                        int64_t q = orc_round_product(w, S);
                        rest -= q;
                        dst[orc_node_index(p, &s, a, b, c)] += q;
                    }
            dst[orc_node_index(p, &s, 1, 1, 1)] += rest;
        }
    }
    free(fex);
}

/* Sub-step count of a sand step of length Dt: ceil(Dt / dt'_max). */
int32_t orc_substeps(double Dt, double dt_max)
{
    double q = ceil(Dt / dt_max);
    return q < 1.0 ? 1 : (int32_t)q;
}

/* One sand step (Alg. 2) of length Dt in N = ceil(Dt / p->dt) equal
 * sub-steps, the fluid fields u, gp, af (3G each; gp, af may be NULL) frozen.
 * Per sub-step: fluid forces at x^i (alpha from alpha_fx = P2G(x^i)),
 * contact forces, exchange deposit into fs (weight 1/N), move, P2G of
 * alpha and momentum at x^{i+1} into alpha_fx, mom_fx.  x, v updated in
 * place; fs accumulates.  Returns N. */
int32_t orc_sand_step(const orc_params *p, const orc_coupling *cp, int64_t n, double Dt, double *x, double *v,
                      const double *r, const double *u, const double *gp, const double *af, int64_t *alpha_fx,
                      int64_t *mom_fx, int64_t *fs)
{
    int32_t N = orc_substeps(Dt, p->dt);
    orc_params ps = *p;
    ps.dt = Dt / (double)N;
    double weight = ps.dt / Dt;
    int64_t G = orc_nodes(p);
    size_t n3 = sizeof(double) * 3 * (size_t)(n > 0 ? n : 1);
    double *Fc = (double *)malloc(n3);
    double *Ffl = (double *)malloc(n3);
    for (int32_t i = 0; i < N; ++i) {
        orc_fluid_forces(&ps, cp, n, x, v, r, NULL, u, alpha_fx, gp, af, Ffl);
        orc_contact_forces(&ps, n, x, v, r, Fc, NULL, NULL, NULL);
        if (fs) orc_exchange_p2g(&ps, cp, n, x, r, NULL, Fc, Ffl, weight, fs);
        orc_integrate_vm(&ps, cp, n, r, Fc, Ffl, x, v);
        memset(alpha_fx, 0, sizeof(int64_t) * (size_t)G);
        memset(mom_fx, 0, sizeof(int64_t) * 3 * (size_t)G);
        orc_p2g_fixed(&ps, n, x, v, r, alpha_fx, mom_fx);
    }
    free(Fc);
    free(Ffl);
    return N;
}

/* ======================================================================== */
/* Capillary (concentration-gradient) pair force, Sec. 5.4                   */
/* ======================================================================== */
/*
 * Passages followed: Sec. 5.4, the liquid-bridge energy E = -2 pi sigma r
 * (-s + sqrt(s^2 + 2 V* / (pi r))) cos(theta) with cos(theta) = 1, its force
 * F^st = -2 pi sigma r ((1 + 2 V* / (pi r s^2))^(-1/2) - 1), the rupture
 * distance d_r = V*^(1/3) + 0.1 V*^(2/3), V* = 0.01 % of the granule volume,
 * the moisture ratio sr_i = r_i + alpha_f,i / (1 - alpha_f,i), and the
 * symmetrised pair force F_ij = -Gamma((sr_i + sr_j) / 2) F^st (x_i - x_j) /
 * |x_i - x_j| for 0 < s_ij < d_r, zero otherwise.
 *
 * Readings (recorded in the design notes):
 *   - polydisperse pairs: r of F^st, of V* and of d_r is the pair's mean
 *     radius (r_i + r_j) / 2 and s_ij = |x_i - x_j| - (r_i + r_j);
 *   - d_r is evaluated as printed with lengths in metres (its second term is
 *     negligible at granule scales);
 *   - Gamma's control points are not printed: a piecewise quadratic Bezier
 *     bump, Gamma(sr) = u (2 - u), u = sr / sr_peak on (0, sr_peak], and
 *     1 - u^2, u = (sr - sr_peak) / (1 - sr_peak) on (sr_peak, 1); zero at
 *     sr <= 0 and sr >= 1, one at sr_peak (the maximum absorption ratio).
 *     Parity unpinned for the shape of Gamma between those three points: the
 *     tests pin Gamma(0) = Gamma(1) = 0 and Gamma(sr_peak) = 1 only;
 *   - the water a granule holds, r_i of the moisture ratio, is an input (the
 *     wetting of Sec. 5.3 is not on this path); alpha_f,i is the fluid
 *     fraction the granule samples from the grid (G2P).
 * The cell list finds every bridged pair when cell >= 2 r_max + d_r(r_max).
 */

typedef struct {
    double sigma;   /* surface tension [N/m]                                  */
    double vbridge; /* liquid-bridge volume / granule volume (1e-4)           */
    double sr_peak; /* moisture ratio of Gamma's maximum, in (0, 1)          */
} orc_capillary;

double orc_gamma(const orc_capillary *c, double sr)
{
    if (!(sr > 0.0) || !(sr < 1.0)) return 0.0;
    if (sr <= c->sr_peak) {
        double u = sr / c->sr_peak;
        return u * (2.0 - u);
    }
    double u = (sr - c->sr_peak) / (1.0 - c->sr_peak);
    return 1.0 - u * u;
}

/* Moisture ratio of each granule (the definition following Eq. 26): the water
 * it holds plus the free water around it per unit sand volume,
 *     sr_i = r_i + alpha_f,i / (1 - alpha_f,i),
 * +inf where alpha_f,i = 1 (no sand around: Gamma is zero there). */
void orc_moisture_ratio(int64_t n, const double *held, const double *alpha_f, double *sr)
{
    for (int64_t i = 0; i < n; ++i) sr[i] = held[i] + alpha_f[i] / (1.0 - alpha_f[i]);
}

/* Liquid-bridge volume V* and rupture distance d_r of a pair of mean radius rb. */
void orc_bridge(const orc_capillary *c, double rb, double *vstar, double *dr)
{
    double V = c->vbridge * orc_volume(rb);
    double t = cbrt(V);
    *vstar = V;
    *dr = t + 0.1 * (t * t);
}

/* Bridge energy E(s) and force F^st(s) of a pair of mean radius rb. */
double orc_bridge_energy(const orc_capillary *c, double rb, double s)
{
    double V, dr;
    orc_bridge(c, rb, &V, &dr);
    return -(2.0 * ORC_PI * c->sigma * rb) * (-s + sqrt(s * s + (2.0 * V) / (ORC_PI * rb)));
}

double orc_fst(const orc_capillary *c, double rb, double s)
{
    double V, dr;
    orc_bridge(c, rb, &V, &dr);
    double q = 1.0 + (2.0 * V) / ((ORC_PI * rb) * (s * s));
    return -(2.0 * ORC_PI * c->sigma * rb) * (1.0 / sqrt(q) - 1.0);
}

/* Capillary force of j on i (3), zero outside 0 < s < d_r. */
static void orc_capillary_pair(const orc_capillary *c, const double xi[3], const double xj[3], double ri,
                               double rj, double sri, double srj, double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    double dv[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
    double d2 = (dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2];
    if (d2 == 0.0) return;
    double d = sqrt(d2);
    double s = d - (ri + rj);
    double rb = 0.5 * (ri + rj);
    double V, dr;
    orc_bridge(c, rb, &V, &dr);
    if (!(s > 0.0) || !(s < dr)) return;
    double g = orc_gamma(c, 0.5 * (sri + srj));
    double f = -(g * orc_fst(c, rb, s));
    for (int a = 0; a < 3; ++a) F[a] = f * (dv[a] / d);
}

/* Force on granule i from j alone (pins and brute-force checks). */
void orc_capillary_pair_force(const orc_capillary *c, const double *xi, const double *xj, double ri, double rj,
                              double sri, double srj, double *F)
{
    orc_capillary_pair(c, xi, xj, ri, rj, sri, srj, F);
}

/* Capillary force on the sampled granules idx[0..m) alone (3m, one by one
 * over the 27 cells around each), and the sum of the magnitudes of their
 * bridge forces (fabs_out, m, optional). */
void orc_capillary_forces_sample(const orc_params *p, const orc_capillary *c, int64_t n, const double *x,
                                 const double *r, const double *sr, int64_t m, const int64_t *idx, double *F,
                                 double *fabs_out)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    int64_t cap = 27 * orc_cells_maxocc(p, &cl) + 1;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t s = 0; s < m; ++s) {
            int64_t i = idx[s];
            double xi[3], acc[3] = {0.0, 0.0, 0.0}, fa = 0.0;
            orc_pos(n, x, i, xi);
            int64_t k = orc_candidates(p, n, x, &cl, i, cand);
            for (int64_t t = 0; t < k; ++t) {
                int64_t j = cand[t];
                double xj[3], Fp[3];
                orc_pos(n, x, j, xj);
                orc_capillary_pair(c, xi, xj, r[i], r[j], sr[i], sr[j], Fp);
                for (int a = 0; a < 3; ++a) acc[a] += Fp[a];
                fa += sqrt((Fp[0] * Fp[0] + Fp[1] * Fp[1]) + Fp[2] * Fp[2]);
            }
            for (int a = 0; a < 3; ++a) F[a * m + s] = acc[a];
            if (fabs_out) fabs_out[s] = fa;
        }
        free(cand);
    }
    orc_cells_free(&cl);
}

/* Adds the capillary force of every bridged pair to F (3n); the candidates
 * are the 27 cells around each granule's cell. */
void orc_capillary_forces(const orc_params *p, const orc_capillary *c, int64_t n, const double *x, const double *r,
                          const double *sr, double *F)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    int64_t cap = 27 * orc_cells_maxocc(p, &cl) + 1;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double xi[3], acc[3] = {0.0, 0.0, 0.0};
            orc_pos(n, x, i, xi);
            int64_t m = orc_candidates(p, n, x, &cl, i, cand);
            for (int64_t k = 0; k < m; ++k) {
                int64_t j = cand[k];
                double xj[3], Fp[3];
                orc_pos(n, x, j, xj);
                orc_capillary_pair(c, xi, xj, r[i], r[j], sr[i], sr[j], Fp);
                for (int a = 0; a < 3; ++a) acc[a] += Fp[a];
            }
            for (int a = 0; a < 3; ++a) F[a * n + i] += acc[a];
        }
        free(cand);
    }
    orc_cells_free(&cl);
}

/* ------------------------------------------------------------------------ */
/* Wet granules: mass with the water a granule holds (Sec. 5.3, Eq. 19)      */
/* ------------------------------------------------------------------------ */
/* A granule holding water of held times its own volume has the mass
 * m = V (rho_s + held rho_0), rho_0 the fluid density.  The wet forms below
 * take per-granule masses where the dry ones use rho_s V: the contact's
 * effective mass (damping), the integrator, the momentum deposit.  The held
 * water also counts as volume V held where the fluid sees the granule
 * (Sec. 5.3): in the solid fraction alpha_s that P2G deposits, in the volume
 * forces (pressure gradient, virtual mass; orc_fluid_forces,
 * orc_exchange_force) and in the virtual mass of the integrator; the clamp
 * of alpha_s rises to 0.740 (1 + r_max) (orc_alpha_clamp). */

void orc_wet_mass(const orc_params *p, double rho_0, int64_t n, const double *r, const double *held, double *m)
{
    for (int64_t i = 0; i < n; ++i) m[i] = orc_volume(r[i]) * (p->rho_s + held[i] * rho_0);
}

void orc_contact_forces_wet(const orc_params *p, int64_t n, const double *x, const double *v, const double *r,
                            const double *m, double *F, double *fabs_out, int32_t *ncont)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    double zeta = orc_zeta(p->restitution);
    int64_t cap = 27 * orc_cells_maxocc(p, &cl) + 1;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double Fi[3], fa;
            int32_t c1, c2;
            orc_contact_one(p, zeta, n, x, v, r, m, &cl, i, cand, Fi, &fa, &c1, &c2);
            for (int a = 0; a < 3; ++a) F[a * n + i] = Fi[a];
            if (fabs_out) fabs_out[i] = fa;
            if (ncont) ncont[i] = c1;
        }
        free(cand);
    }
    orc_cells_free(&cl);
}

void orc_contact_forces_sample_wet(const orc_params *p, int64_t n, const double *x, const double *v,
                                   const double *r, const double *mass, int64_t cnt, const int64_t *idx,
                                   double *F, double *fabs_out)
{
    orc_cells cl;
    orc_cells_build(p, n, x, &cl);
    double zeta = orc_zeta(p->restitution);
    int64_t cap = 27 * orc_cells_maxocc(p, &cl) + 1;
#pragma omp parallel
    {
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t s = 0; s < cnt; ++s) {
            double Fi[3], fa;
            orc_contact_one(p, zeta, n, x, v, r, mass, &cl, idx[s], cand, Fi, &fa, NULL, NULL);
            for (int a = 0; a < 3; ++a) F[a * cnt + s] = Fi[a];
            if (fabs_out) fabs_out[s] = fa;
        }
        free(cand);
    }
    orc_cells_free(&cl);
}

/* Semi-implicit Euler with per-granule masses; under virtual mass the
 * effective mass is m + (1/2) rho_f V and gravity acts on m (as
 * orc_integrate_vm), V = (4/3) pi r^3 (1 + held) counting the absorbed water
 * (Sec. 5.3; held may be NULL: dry volume). */
void orc_integrate_wet(const orc_params *p, const orc_coupling *cp, int64_t n, const double *r, const double *held,
                       const double *m, const double *Fc, const double *Fd, double *x, double *v)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double me = cp->vmass ? m[i] + (0.5 * cp->rho_f) * orc_wet_volume(r[i], held ? held[i] : 0.0) : m[i];
        for (int d = 0; d < 3; ++d) {
            double a = cp->vmass ? ((Fc[d * n + i] + Fd[d * n + i]) + m[i] * p->g[d]) / me
                                 : (Fc[d * n + i] + Fd[d * n + i]) / m[i] + p->g[d];
            v[d * n + i] = v[d * n + i] + p->dt * a;
            x[d * n + i] = x[d * n + i] + p->dt * v[d * n + i];
        }
    }
}

/* P2G of the wet granules' volume fraction and momentum (Sec. 5.3, Eq. 19):
 * the fraction channel deposits frac (1 + held), the sand's volume plus the
 * water it holds, and the momentum channels frac (rho_s + held rho_0) / rho_s v. */
void orc_p2g_fixed_wet(const orc_params *p, double rho_0, int64_t n, const double *x, const double *v,
                       const double *r, const double *held, int64_t *alpha, int64_t *mom)
{
    orc_p2g_fixed_held(p, rho_0, n, x, v, r, held, alpha, mom);
}

