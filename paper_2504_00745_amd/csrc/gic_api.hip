// C ABI of the granule path (include/gic.h): argument checks, context and
// scratch management, and the launch sequence of one sub-step (Alg. 2).
#include <math.h>
#include <string.h>

#include <mutex>

#include "../../include/gic.h"
#include "gic_launch.hpp"
#include "idp_launch.hpp"

using namespace gic;

struct gic_ctx {
    gic_params p;
    DevParams dp;
    int64_t n_max;
    int64_t K;
    SortScratch sort;
    int64_t *err;  // device: [code, index]
    double *part;  // device: partial sums of gic_sum
    BrickList bricks;  // device: occupied bricks of the last cell ranges given
    bool in_step;      // inside gic_step, which builds the brick list once
    int device;
    int64_t *fxs;      // device: 4 G int64, integer sums of the unquantised transfers
    double *fxp;       // device: 4 x 1024 partial maxima, then the 4 scales and their inverses
    NbrList nl;        // device: neighbour list of the stepping path
    // device: tiles and escape list of the stepping path's assembled P2G
    // (tiles NULL: the grids are cleared and the tiles added with atomics);
    // the escape counters alternate between consecutive steps
    P2GStore p2gs;
    uint32_t *esc_n2;
    int esc_par;
    // The live flags of p2gs describe the grids live_a, live_m (alpha and
    // momentum) when live_ok: the last write to them was the stepping path's
    // assembly, and no call on the context has written to them since.
    bool live_ok;
    const int64_t *live_a, *live_m;
    // the largest brick shell of the direct contact kernel, for the size of
    // its shell array, and the most granules in a brick of the P2G tile
    // kernel, for its workgroup size (device records, pinned host copies)
    SizeRecord shell, brick_n;
    // The list holds the stepping path's state when nl_n == n and the state
    // to step is the array that the last step wrote (nl_x): its sorted
    // order is the one of the list's last build or check.
    int64_t nl_n;
    const double *nl_x;
    // The cell tables rng_cb, rng_ce hold the ranges of the last sort on the
    // context, and the brick list is theirs (set by the stepping calls,
    // cleared by any other call that sorts or builds a brick list).
    bool rng_ok;
    const int32_t *rng_cb, *rng_ce;
    // gic_brick_list: the brick list built for the cell tables bl_cb, bl_ce,
    // reused by the calls given those tables until the next sort, stepping
    // call or brick list build
    bool bl_pin;
    const int32_t *bl_cb, *bl_ce;
    // stage timing of gic_step / gic_sand_step (gic_stage_timing): events
    // recorded on the step's stream between its stages, kStageEvents per step
    int tm_cap, tm_used;
    hipEvent_t *tm_ev;
};

// Events per timed (sub-)step: start, after the sort and brick list, after
// the gather, after the contact, after the exchange deposit, after the grid
// clear, after integrate + P2G (the tile kernel, or the atomic deposit),
// after the assembly of the grids from the tiles.
constexpr int kStageEvents = 8;

namespace {

int64_t key_space_of(const gic_params *p)
{
    int64_t nb[3];
    for (int a = 0; a < 3; ++a) nb[a] = (p->nc[a] + kBrick - 1) / kBrick;
    return nb[0] * nb[1] * nb[2] * kBrickCells;
}

// Rupture distance of the liquid bridge between two granules of radius r_max
// (Sec. 5.4): d_r = V*^(1/3) + 0.1 V*^(2/3), V* = vbridge (4/3) pi r_max^3;
// 0 without capillary force.
double rupture_max(const gic_params *p)
{
    if (!(p->sigma > 0.0)) return 0.0;
    const double V = p->vbridge * (((4.0 * GIC_PI / 3.0) * p->r_max) * p->r_max) * p->r_max;
    const double t = cbrt(V);
    return t + 0.1 * (t * t);
}

// Reach of the stepping path's neighbour list beyond r_i + r_j: a tenth of
// the largest radius, as far as the cells allow (cell >= 2 r_max + skin keeps
// every listed pair inside the 27 cells); 0 when the cells are exactly
// 2 r_max, and the list is then rebuilt every step.
void nbr_reach(const gic_params *p, NbrList &L)
{
    const double room = p->cell - 2.0 * p->r_max;
    double skin = 0.1 * p->r_max;
    if (skin > room) skin = room;
    if (!(skin > 0.0)) skin = 0.0;
    L.skin = skin;
    // rebuild when a granule has moved by skin / 2 since the build, less the
    // rounding of the single-precision positions kept at the build
    double lmax = 0.0;
    for (int a = 0; a < 3; ++a) lmax = fmax(lmax, (double)p->n[a] * p->dx);
    const double thr = 0.5 * skin - lmax * (1.0 / 1048576.0);
    L.thr2 = thr > 0.0 ? (float)(thr * thr) : -1.0f;
}

bool params_valid(const gic_params *p)
{
    if (!p) return false;
    for (int a = 0; a < 3; ++a) {
        if (p->n[a] < 1 || p->nc[a] < 1 || p->n[a] > 32767) return false;  // stencil bases are 16-bit in LDS
        if ((double)p->nc[a] * p->cell > (double)p->n[a] * p->dx * (1.0 + 1e-12)) return false;
    }
    if (!(p->dx > 0.0) || !(p->cell > 0.0) || !isfinite(p->dx) || !isfinite(p->cell)) return false;
    if (!(p->r_max > 0.0) || p->cell < 2.0 * p->r_max) return false;
    if (!(p->kn > 0.0) || !(p->restitution > 0.0) || !(p->restitution <= 1.0)) return false;
    if (!(p->kt_ratio >= 0.0) || !(p->mu >= 0.0) || !(p->rho_s > 0.0)) return false;
    if (!(p->eta_f >= 0.0) || !(p->c_drag >= 0.0) || !(p->alpha_max > 0.0) || !(p->dt > 0.0)) return false;
    if (!(p->rho_f >= 0.0) || !isfinite(p->rho_f) || !(p->c_quad >= 0.0) || !isfinite(p->c_quad)) return false;
    if (!(p->f_unit >= 0.0) || !isfinite(p->f_unit)) return false;
    if (p->drag_model != 0 && p->drag_model != 1) return false;
    if (p->vmass != 0 && p->vmass != 1) return false;
    if (!(p->sigma >= 0.0) || !isfinite(p->sigma)) return false;
    if (!(p->absorb_max >= 0.0) || !isfinite(p->absorb_max)) return false;
    if (p->sigma > 0.0) {
        if (!(p->vbridge > 0.0) || !isfinite(p->vbridge) || !(p->sr_peak > 0.0) || !(p->sr_peak < 1.0)) return false;
        if (p->cell < 2.0 * p->r_max + rupture_max(p)) return false;  // the cells must reach every bridge
    }
    for (int a = 0; a < 3; ++a)
        if (!isfinite(p->g[a])) return false;
    if (p->precision != GIC_FP64 && p->precision != GIC_FP32) return false;
    if (p->walls > 0x3Fu) return false;
    const int64_t K = key_space_of(p);
    if (K > ((int64_t)1 << 32) || (int64_t)p->n[0] * p->n[1] * p->n[2] > ((int64_t)1 << 40)) return false;
    return true;
}

// Edge of the P2G LDS tile: the nodes touched by a brick's granules plus one
// node of slack on each side.
// Nodes per edge of a brick's node tile: the stencils of granules whose
// cell lies in the brick span 4 cell / dx + 2 nodes when that is an integer
// (the brick starts on a node boundary), one more otherwise.  Granules that
// moved out of their cell since the sort reach outside the tile and take
// the global path.
// Whether a node lies in the tiles of at most two bricks per axis, which
// k_p2g_assemble assumes: tile origins of bricks two apart differ by at
// least the tile edge.  4 cell/dx an integer: cell/dx >= 1/2; otherwise
// 4 cell/dx > 4.  (And at most 2,048 bricks along x.)
bool tiles_assemble(const gic_params *p)
{
    if ((p->nc[0] + kBrick - 1) / kBrick > 512) return false;  // four rows' bricks in 32 KiB of LDS
    const double m4 = (double)kBrick * p->cell / p->dx;
    const double r = floor(m4 + 0.5);
    if (fabs(m4 - r) < 1e-9 * (r > 1.0 ? r : 1.0)) return r >= 2.0;
    return m4 > 4.0;
}

int tile_edge(const gic_params *p)
{
    const double m4 = (double)kBrick * p->cell / p->dx;
    const double r = floor(m4 + 0.5);
    if (fabs(m4 - r) < 1e-9 * (r > 1.0 ? r : 1.0)) return (int)r + 2;
    return (int)ceil(m4) + 3;
}

DevParams derive(const gic_params *p)
{
    DevParams d;
    memset(&d, 0, sizeof(d));
    for (int a = 0; a < 3; ++a) {
        d.n[a] = p->n[a];
        d.nc[a] = p->nc[a];
        d.nb[a] = (p->nc[a] + kBrick - 1) / kBrick;
        d.L[a] = (double)p->n[a] * p->dx;
        d.g[a] = p->g[a];
    }
    d.tile = tile_edge(p);
    d.G = (int64_t)p->n[0] * p->n[1] * p->n[2];
    d.dx = p->dx;
    d.inv_dx = 1.0 / p->dx;
    d.inv_vcell = 1.0 / ((p->dx * p->dx) * p->dx);
    d.cell = p->cell;
    d.inv_cell = 1.0 / p->cell;
    d.kn = p->kn;
    const double le = log(p->restitution);
    d.zeta = -le / sqrt(GIC_PI * GIC_PI + le * le);
    d.kt_ratio = p->kt_ratio;
    d.mu = p->mu;
    d.rho_s = p->rho_s;
    d.cdrag = (p->c_drag * (6.0 * GIC_PI)) * p->eta_f;
    d.c_drag = p->c_drag;
    d.cdrag_unit = (6.0 * GIC_PI) * p->eta_f;
    d.alpha_max = p->alpha_max * (1.0 + p->absorb_max);  // raised for absorbed water (Sec. 5.3)
    d.dt = p->dt;
    d.r_max = p->r_max;
    d.search_scale = 1.0 + 1.0 / 1073741824.0;  // 1 + 2^-30: slack for rounding
    d.walls = p->walls;
    d.rho_f = p->rho_f;
    d.half_rho_f = 0.5 * p->rho_f;
    d.c_quad = p->c_quad;
    d.drag_model = p->drag_model;
    d.vmass = p->vmass;
    d.sigma = p->sigma;
    d.vbridge = p->vbridge;
    d.sr_peak = p->sr_peak;
    d.dr_max = rupture_max(p);
    return d;
}

int sort_passes(int64_t K)
{
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < K) ++bits;
    return (bits + 7) / 8;
}

gic_status hip_status(hipError_t e) { return e == hipSuccess ? GIC_OK : GIC_E_HIP; }

bool fp32(const gic_ctx *c) { return c->p.precision == GIC_FP32; }

bool n_ok(const gic_ctx *c, int64_t n) { return c && n >= 0 && n <= c->n_max; }

constexpr int kSumParts = 1024;
// Largest n of gic_sum_noalloc: 1,024 partial sums of at most 2^20 values each.
constexpr int64_t kSumNoallocMax = (int64_t)kSumParts << 20;

// The brick schedule of the cell ranges a call is given, built on the stream
// before its brick kernel; gic_step builds it once after its sort.
hipError_t brick_list(gic_ctx *c, const int32_t *cb, const int32_t *ce, hipStream_t s)
{
    if (c->in_step) return hipSuccess;
    if (c->bl_pin && c->bl_cb == cb && c->bl_ce == ce) return hipSuccess;  // kept by gic_brick_list
    c->bl_pin = false;
    c->rng_ok = false;  // the brick list is now that of these tables
    return launch_brick_list(cb, ce, c->bricks, s);
}

// Sort of a stepping call: keeps the neighbour list when the last step's
// state continues (force = 0) and the cell tables and brick list when the
// tables are the last step's and no key changed.
hipError_t step_sort(gic_ctx *c, int64_t n, const double *x, uint32_t *key, int32_t *order, int32_t *cb, int32_t *ce,
                     int force, hipStream_t s)
{
    const int keep = c->rng_ok && c->rng_cb == cb && c->rng_ce == ce && c->sort.last_n == n ? 1 : 0;
    c->rng_ok = false;
    c->bl_pin = false;
    hipError_t e = launch_sort_cells(c->dp, n, x, key, order, cb, ce, c->K, c->sort, c->err, s, &c->nl, force, keep);
    if (e == hipSuccess && n > 0) e = launch_brick_list(cb, ce, c->bricks, s, keep ? c->sort.ctl : nullptr);
    if (e == hipSuccess) {
        c->rng_ok = true;
        c->rng_cb = cb;
        c->rng_ce = ce;
    }
    return e;
}

// Density-projection workspace: alpha_f', s, r, d, w, 1/diag (G doubles
// each), the partial sums and the solver state, each 256-byte aligned.
int64_t idp_align(int64_t b) { return (b + 255) & ~(int64_t)255; }

// Levels of the multigrid hierarchy: halve every axis (rounding up) until a
// level has at most kMgCoarsest cells.
int idp_levels(const IdpDims &D0, IdpDims *out)
{
    out[0] = D0;
    int l = 0;
    while (out[l].G > kMgCoarsest && l + 1 < kMgMaxLevels) {
        IdpDims n;
        n.nx = (out[l].nx + 1) / 2;
        n.ny = (out[l].ny + 1) / 2;
        n.nz = (out[l].nz + 1) / 2;
        idp_dims_finish(n);
        out[++l] = n;
    }
    return l + 1;
}

int64_t idp_work_bytes(const IdpDims &D0)
{
    IdpDims lv[kMgMaxLevels];
    const int L = idp_levels(D0, lv);
    int64_t b = 9 * idp_align(D0.G * 8) + idp_align(3 * kIdpMaxBlocks * 8) + idp_align(sizeof(CgState));
    for (int l = 1; l < L; ++l) b += 5 * idp_align(lv[l].G * 8);
    return b;
}

// Carves the workspace: alpha_f' and s slots for gic_density_projection, the
// CG vectors, the fine grid's signed coefficients, and (multigrid) the
// coarser levels; level 0 works on the residual r and the preconditioned
// residual z.
IdpWork idp_carve(void *work, const IdpDims &D0, int precond, double **at, double **s)
{
    char *p = (char *)work;
    const int64_t a = idp_align(D0.G * 8);
    IdpWork W;
    *at = (double *)p;
    *s = (double *)(p + a);
    W.r = (double *)(p + 2 * a);
    W.d = (double *)(p + 3 * a);
    W.w = (double *)(p + 4 * a);
    W.dinv = (double *)(p + 5 * a);
    double *z = (double *)(p + 6 * a), *ac = (double *)(p + 7 * a), *t = (double *)(p + 8 * a);
    p += 9 * a;
    W.part = (double *)p;
    p += idp_align(3 * kIdpMaxBlocks * 8);
    W.state = (CgState *)p;
    p += idp_align(sizeof(CgState));
    IdpDims lv[kMgMaxLevels];
    const int L = idp_levels(D0, lv);
    W.nlev = precond == 1 ? L : 1;
    W.lev[0] = MgLevel{D0, 1.0, ac, W.dinv, W.r, z, t};
    double scale = 1.0;
    for (int l = 1; l < L; ++l) {
        scale *= 4.0;
        const int64_t g = idp_align(lv[l].G * 8);
        MgLevel m;
        m.D = lv[l];
        m.scale = scale;
        m.ac = (double *)p;
        m.dinv = (double *)(p + g);
        m.b = (double *)(p + 2 * g);
        m.e = (double *)(p + 3 * g);
        m.t = (double *)(p + 4 * g);
        p += 5 * g;
        W.lev[l] = m;
    }
    return W;
}

// Runs CG iterations in chunks of check_every, reading the state after each
// chunk; the kernels of a chunk after convergence return at once.
gic_status idp_cg(const gic_ctx *c, const double *at, const uint8_t *label, const double *s, double *q,
                  const IdpWork &W, int32_t max_iter, double tol, int32_t check_every, int32_t *iters,
                  double *relres, hipStream_t st)
{
    const IdpDims D = idp_dims(c->dp);
    hipError_t e = launch_cg_start(D, at, label, s, q, W, tol, c->err, st);
    CgState h;
    int k = 0;
    for (;;) {
        if (e == hipSuccess) e = hipMemcpyAsync(&h, W.state, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return GIC_E_HIP;
        if (h.done >= 0 || k >= max_iter) break;
        const int cnt = max_iter - k < check_every ? max_iter - k : check_every;
        e = launch_cg_iterations(D, at, label, q, W, k, cnt, st);
        k += cnt;
    }
    if (iters) *iters = (int32_t)(h.done >= 0 ? h.done : h.iters);
    if (relres) *relres = h.ss > 0.0 ? sqrt(h.rr / h.ss) : sqrt(h.rr);
    return GIC_OK;
}

}  // namespace

extern "C" {

int64_t gic_key_space(const gic_params *p) { return params_valid(p) ? key_space_of(p) : -1; }

gic_status gic_create(const gic_params *p, int64_t n_max, gic_ctx **out)
{
    if (!out || !params_valid(p) || n_max < 0 || n_max > ((int64_t)1 << 31) - 1) return GIC_E_ARG;
    *out = nullptr;
    const int E = tile_edge(p);
    if ((size_t)E * E * E * 4 * sizeof(double) > 65536) return GIC_E_ARG;  // P2G tile must fit in LDS
    gic_ctx *c = new gic_ctx();  // value-initialised: every pointer starts null
    memset(c, 0, sizeof(*c));
    c->p = *p;
    c->dp = derive(p);
    c->n_max = n_max;
    c->K = key_space_of(p);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return GIC_E_HIP;
    }
    const int64_t nn = n_max > 0 ? n_max : 1;
    const int64_t tiles = sort_tiles_max(nn);
    c->sort.tiles_max = tiles;
    c->sort.passes = sort_passes(c->K);
    bool ok = true;
    ok &= hipMalloc(&c->sort.kA, sizeof(uint32_t) * nn) == hipSuccess;
    ok &= hipMalloc(&c->sort.kB, sizeof(uint32_t) * nn) == hipSuccess;
    ok &= hipMalloc(&c->sort.skeys[0], sizeof(uint32_t) * nn) == hipSuccess;
    ok &= hipMalloc(&c->sort.skeys[1], sizeof(uint32_t) * nn) == hipSuccess;
    c->sort.cur = 0;
    c->sort.last_n = -1;
    ok &= hipMalloc(&c->sort.chg, sizeof(uint64_t) * kChgCap) == hipSuccess;
    ok &= hipMalloc(&c->sort.chg_s, sizeof(uint64_t) * kChgCap) == hipSuccess;
    ok &= hipMalloc(&c->sort.chg_p, sizeof(uint32_t) * kChgCap) == hipSuccess;
    ok &= hipMalloc(&c->sort.ctl, sizeof(int32_t) * 4) == hipSuccess;
    if (ok) ok = hipMemset(c->sort.ctl, 0, sizeof(int32_t) * 4) == hipSuccess;
    ok &= hipMalloc(&c->sort.vA, sizeof(int32_t) * nn) == hipSuccess;
    ok &= hipMalloc(&c->sort.vB, sizeof(int32_t) * nn) == hipSuccess;
    ok &= hipMalloc(&c->sort.rowtot, sizeof(uint32_t) * 256) == hipSuccess;
    ok &= hipMalloc(&c->sort.tcnt, sizeof(uint32_t) * 256 * tiles) == hipSuccess;
    ok &= hipMalloc(&c->sort.sums, sizeof(uint32_t) * 1024) == hipSuccess;
    ok &= hipMalloc(&c->sort.cnt, sizeof(uint32_t) * (c->K > 0 ? c->K : 1)) == hipSuccess;
    if (ok) ok = hipMemset(c->sort.cnt, 0, sizeof(uint32_t) * (c->K > 0 ? c->K : 1)) == hipSuccess;
    ok &= hipMalloc(&c->err, sizeof(int64_t) * 2) == hipSuccess;
    ok &= hipMalloc(&c->part, sizeof(double) * kSumParts) == hipSuccess;
    c->bricks.nbricks = c->K / kBrickCells;
    ok &= hipMalloc(&c->bricks.list, sizeof(int32_t) * (c->bricks.nbricks > 0 ? c->bricks.nbricks : 1)) == hipSuccess;
    ok &= hipMalloc(&c->bricks.count, sizeof(int32_t)) == hipSuccess;
    ok &= hipMalloc(&c->bricks.sums, sizeof(uint32_t) * 1024) == hipSuccess;
    ok &= hipMalloc(&c->bricks.slot_of, sizeof(int32_t) * (c->bricks.nbricks > 0 ? c->bricks.nbricks : 1)) ==
          hipSuccess;
    ok &= hipMalloc(&c->p2gs.esc, sizeof(int32_t) * nn) == hipSuccess;
    ok &= hipMalloc(&c->esc_n2, sizeof(uint32_t) * 2) == hipSuccess;
    if (ok) ok = hipMemset(c->esc_n2, 0, sizeof(uint32_t) * 2) == hipSuccess;
    ok &= hipMalloc(&c->shell.dev, sizeof(int32_t) * 2 * kRecSlots) == hipSuccess;
    if (ok) ok = hipMemset(c->shell.dev, 0, sizeof(int32_t) * 2 * kRecSlots) == hipSuccess;
    ok &= hipHostMalloc(&c->shell.host, sizeof(int32_t) * kRecSlots, hipHostMallocDefault) == hipSuccess;
    if (ok)
        for (int i = 0; i < kRecSlots; ++i) c->shell.host[i] = 0;  // no record yet: the largest shell array
    ok &= hipMalloc(&c->brick_n.dev, sizeof(int32_t) * 2 * kRecSlots) == hipSuccess;
    if (ok) ok = hipMemset(c->brick_n.dev, 0, sizeof(int32_t) * 2 * kRecSlots) == hipSuccess;
    ok &= hipHostMalloc(&c->brick_n.host, sizeof(int32_t) * kRecSlots, hipHostMallocDefault) == hipSuccess;
    if (ok)
        for (int i = 0; i < kRecSlots; ++i) c->brick_n.host[i] = 0;  // no record yet: workgroups of 256
    if (ok && tiles_assemble(p)) {
        // one 4-channel node tile per occupied brick (at most min(bricks, n));
        // beyond 8 GiB the stepping path keeps the cleared grids and atomics
        const int64_t E = c->dp.tile;
        const int64_t slots = c->bricks.nbricks < nn ? c->bricks.nbricks : nn;
        const size_t bytes = (size_t)(slots > 0 ? slots : 1) * 4 * E * E * E * sizeof(unsigned long long);
        const size_t ncov = 4 * ((size_t)p->n[0] + p->n[1] + p->n[2]);
        int32_t *cov = nullptr;
        if (bytes <= ((size_t)8 << 30) && hipMalloc(&c->p2gs.tiles, bytes) == hipSuccess &&
            hipMalloc(&cov, sizeof(int32_t) * ncov) == hipSuccess) {
            int32_t *h = new int32_t[ncov];
            p2g_cover_table(c->dp, h);
            ok &= hipMemcpy(cov, h, sizeof(int32_t) * ncov, hipMemcpyHostToDevice) == hipSuccess;
            delete[] h;
            c->p2gs.cover = cov;
            // live flags: without them every assembly writes every node
            const size_t nlive = (size_t)p->n[1] * p->n[2] * (((size_t)p->n[0] + 3) / 4);
            if (hipMalloc(&c->p2gs.live, nlive) != hipSuccess || hipMemset(c->p2gs.live, 0, nlive) != hipSuccess) {
                (void)hipFree(c->p2gs.live);
                c->p2gs.live = nullptr;
                (void)hipGetLastError();
            }
        } else {
            (void)hipFree(c->p2gs.tiles);
            c->p2gs.tiles = nullptr;  // the fallback path needs neither
            (void)hipGetLastError();
        }
    }
    ok &= hipMalloc(&c->fxs, sizeof(int64_t) * 4 * (size_t)(c->dp.G > 0 ? c->dp.G : 1)) == hipSuccess;
    ok &= hipMalloc(&c->fxp, sizeof(double) * (4 * 1024 + 8)) == hipSuccess;
    ok &= hipMalloc(&c->nl.nbr, sizeof(int32_t) * kNbrCap * nn) == hipSuccess;
    ok &= hipMalloc(&c->nl.cnt, sizeof(int32_t) * nn) == hipSuccess;
    ok &= hipMalloc(&c->nl.xref, sizeof(float) * 3 * nn) == hipSuccess;
    ok &= hipMalloc(&c->nl.ctl, sizeof(uint32_t) * 4) == hipSuccess;
    ok &= hipMalloc(&c->nl.dpart, sizeof(float) * (size_t)((nn + 255) / 256)) == hipSuccess;
    if (ok) ok = hipMemset(c->nl.ctl, 0, sizeof(uint32_t) * 4) == hipSuccess;
    nbr_reach(p, c->nl);
    c->nl_n = -1;
    c->nl_x = nullptr;
    if (ok) ok = hipMemset(c->err, 0, sizeof(int64_t) * 2) == hipSuccess;
    if (!ok) {
        gic_destroy(c);
        return GIC_E_ALLOC;
    }
    *out = c;
    return GIC_OK;
}

gic_status gic_set_params(gic_ctx *c, const gic_params *p)
{
    if (!c || !params_valid(p)) return GIC_E_ARG;
    for (int a = 0; a < 3; ++a)
        if (p->n[a] != c->p.n[a] || p->nc[a] != c->p.nc[a]) return GIC_E_ARG;
    if (p->dx != c->p.dx || p->cell != c->p.cell || p->precision != c->p.precision) return GIC_E_ARG;
    c->p = *p;
    c->dp = derive(p);
    nbr_reach(p, c->nl);
    c->nl_n = -1;  // radii or r_max may differ: the next step builds its list afresh
    c->live_ok = false;  // and writes its grids whole
    return GIC_OK;
}

gic_status gic_destroy(gic_ctx *c)
{
    if (!c) return GIC_E_ARG;
    hipError_t e = hipDeviceSynchronize();
    (void)hipFree(c->sort.kA);
    (void)hipFree(c->sort.kB);
    (void)hipFree(c->sort.skeys[0]);
    (void)hipFree(c->sort.skeys[1]);
    (void)hipFree(c->sort.chg);
    (void)hipFree(c->sort.chg_s);
    (void)hipFree(c->sort.chg_p);
    (void)hipFree(c->sort.ctl);
    (void)hipFree(c->sort.vA);
    (void)hipFree(c->sort.vB);
    (void)hipFree(c->sort.rowtot);
    (void)hipFree(c->sort.tcnt);
    (void)hipFree(c->sort.sums);
    (void)hipFree(c->sort.cnt);
    (void)hipFree(c->err);
    (void)hipFree(c->part);
    (void)hipFree(c->bricks.list);
    (void)hipFree(c->bricks.count);
    (void)hipFree(c->bricks.sums);
    (void)hipFree(c->bricks.slot_of);
    (void)hipFree(c->p2gs.esc);
    (void)hipFree(c->p2gs.tiles);
    (void)hipFree(const_cast<int32_t *>(c->p2gs.cover));
    (void)hipFree(c->p2gs.live);
    (void)hipFree(c->esc_n2);
    (void)hipFree(c->shell.dev);
    (void)hipHostFree(c->shell.host);
    (void)hipFree(c->brick_n.dev);
    (void)hipHostFree(c->brick_n.host);
    if (c->tm_ev) {
        for (int i = 0; i < c->tm_cap * kStageEvents; ++i) (void)hipEventDestroy(c->tm_ev[i]);
        delete[] c->tm_ev;
    }
    (void)hipFree(c->fxs);
    (void)hipFree(c->fxp);
    (void)hipFree(c->nl.nbr);
    (void)hipFree(c->nl.cnt);
    (void)hipFree(c->nl.xref);
    (void)hipFree(c->nl.ctl);
    (void)hipFree(c->nl.dpart);
    delete c;
    return hip_status(e);
}

gic_status gic_get_error(gic_ctx *c, void *stream, int32_t *code, int64_t *index, int32_t clear)
{
    if (!c || !code || !index) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    int64_t h[2] = {0, -1};
    hipError_t e = hipMemcpyAsync(h, c->err, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return GIC_E_HIP;
    *code = (int32_t)h[0];
    *index = h[0] ? h[1] : -1;
    if (clear) {
        e = hipMemsetAsync(c->err, 0, sizeof(int64_t) * 2, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    return hip_status(e);
}

gic_status gic_neighbour_builds(gic_ctx *c, void *stream, int64_t *builds)
{
    if (!c || !builds) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    uint32_t h[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(h, c->nl.ctl, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return GIC_E_HIP;
    *builds = (int64_t)h[2];
    return GIC_OK;
}

gic_status gic_sort_cells(gic_ctx *c, int64_t n, const double *x, uint32_t *key, int32_t *order,
                          int32_t *cell_begin, int32_t *cell_end, void *stream)
{
    if (!n_ok(c, n) || !cell_begin || !cell_end || (n > 0 && (!x || !key || !order))) return GIC_E_ARG;
    c->nl_n = -1;  // the next gic_step cannot rely on this sort's keys for its neighbour list
    c->rng_ok = false;
    c->bl_pin = false;
    return hip_status(launch_sort_cells(c->dp, n, x, key, order, cell_begin, cell_end, c->K, c->sort, c->err,
                                        (hipStream_t)stream));
}

gic_status gic_brick_list(gic_ctx *c, const int32_t *cell_begin, const int32_t *cell_end, void *stream)
{
    if (!c || !cell_begin || !cell_end) return GIC_E_ARG;
    c->bl_pin = false;
    const hipError_t e = brick_list(c, cell_begin, cell_end, (hipStream_t)stream);
    if (e != hipSuccess) return GIC_E_HIP;
    if (!c->in_step) {
        c->bl_pin = true;
        c->bl_cb = cell_begin;
        c->bl_ce = cell_end;
    }
    return GIC_OK;
}

gic_status gic_reorder(gic_ctx *c, int64_t n, const int32_t *order, const double *x, const double *v,
                       const double *r, const int32_t *id, double *x_out, double *v_out, double *r_out,
                       int32_t *id_out, void *stream)
{
    if (!n_ok(c, n)) return GIC_E_ARG;
    if (n > 0 && (!order || !x || !v || !r || !x_out || !v_out || !r_out)) return GIC_E_ARG;
    if ((id == nullptr) != (id_out == nullptr)) return GIC_E_ARG;
    if (n > 0 && (x_out == x || v_out == v || r_out == r || (id && id_out == id))) return GIC_E_ARG;
    return hip_status(launch_reorder(n, order, x, v, r, id, x_out, v_out, r_out, id_out, (hipStream_t)stream));
}

// Neighbour list (built when force is set or the sort asked for it) and the
// contact forces from it.
static gic_status contact_impl(gic_ctx *c, int64_t n, const double *x, const double *v, const double *r,
                               const int32_t *cell_begin, const int32_t *cell_end, void *f_contact,
                               int32_t *n_contacts, int32_t *pair_ids, int32_t pair_cap, int force, hipStream_t s)
{
    if (!pair_ids && (!c->in_step || !(c->nl.thr2 > 0.0f))) {
        // a list that would serve this call only (a stage call outside the
        // stepping path, or no skin: cells of exactly 2 r_max, so the
        // stepping path would rebuild it every step): the forces come
        // straight from the cells (same partner order, same bits)
        if (fp32(c))
            return hip_status(launch_contact<float>(c->dp, n, x, v, r, cell_begin, cell_end, c->bricks, nullptr,
                                                    nullptr, (float *)f_contact, n_contacts, c->err, s, &c->shell));
        return hip_status(launch_contact<double>(c->dp, n, x, v, r, cell_begin, cell_end, c->bricks, nullptr,
                                                 nullptr, (double *)f_contact, n_contacts, c->err, s, &c->shell));
    }
    if (launch_nbr_build(c->dp, n, x, r, cell_begin, cell_end, c->bricks, c->nl, force, c->err, s) != hipSuccess)
        return GIC_E_HIP;
    if (fp32(c))
        return hip_status(launch_contact_list<float>(c->dp, n, x, v, r, cell_begin, cell_end, c->nl,
                                                     (float *)f_contact, n_contacts, pair_ids, pair_cap, c->err, s));
    return hip_status(launch_contact_list<double>(c->dp, n, x, v, r, cell_begin, cell_end, c->nl,
                                                  (double *)f_contact, n_contacts, pair_ids, pair_cap, c->err, s));
}

gic_status gic_contact_forces(gic_ctx *c, int64_t n, const double *x, const double *v, const double *r,
                              const int32_t *cell_begin, const int32_t *cell_end, void *f_contact,
                              int32_t *n_contacts, int32_t *pair_ids, int32_t pair_cap, void *stream)
{
    if (!n_ok(c, n) || pair_cap < 0 || (pair_cap > 0 && !pair_ids)) return GIC_E_ARG;
    if (n > 0 && (!x || !v || !r || !cell_begin || !cell_end || !f_contact)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return GIC_OK;
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    c->nl_n = -1;  // the list now belongs to these arrays, not to the stepping path
    return contact_impl(c, n, x, v, r, cell_begin, cell_end, f_contact, n_contacts, pair_cap > 0 ? pair_ids : nullptr,
                        pair_cap, 1, s);
}

gic_status gic_contact_capillary_forces(gic_ctx *c, int64_t n, const double *x, const double *v, const double *r,
                                        const void *sr, const double *held, const int32_t *cell_begin,
                                        const int32_t *cell_end, void *f_contact, int32_t *n_contacts, void *stream)
{
    if (!n_ok(c, n)) return GIC_E_ARG;
    if (!(c->p.sigma > 0.0)) return GIC_E_ARG;
    if (n > 0 && (!x || !v || !r || !sr || !cell_begin || !cell_end || !f_contact)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return GIC_OK;
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    if (fp32(c))
        return hip_status(launch_contact<float>(c->dp, n, x, v, r, cell_begin, cell_end, c->bricks,
                                                (const float *)sr, held, (float *)f_contact, n_contacts, c->err,
                                                s, &c->shell));
    return hip_status(launch_contact<double>(c->dp, n, x, v, r, cell_begin, cell_end, c->bricks,
                                             (const double *)sr, held, (double *)f_contact, n_contacts, c->err, s,
                                             &c->shell));
}

gic_status gic_moisture_ratio(gic_ctx *c, int64_t n, const double *held, const void *alpha_f, void *sr,
                              void *stream)
{
    if (!n_ok(c, n)) return GIC_E_ARG;
    if (n > 0 && (!held || !alpha_f || !sr)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (fp32(c))
        return hip_status(launch_moisture_ratio<float>(n, held, (const float *)alpha_f, (float *)sr, s));
    return hip_status(launch_moisture_ratio<double>(n, held, (const double *)alpha_f, (double *)sr, s));
}

gic_status gic_g2p(gic_ctx *c, int64_t n, const double *x, const void *u, const int64_t *alpha_fx,
                   const double *alpha_real, void *u_at, void *alpha_f, void *stream)
{
    if (!n_ok(c, n) || ((alpha_fx == nullptr) == (alpha_real == nullptr))) return GIC_E_ARG;
    if (n > 0 && (!x || !u || !u_at || !alpha_f)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (fp32(c))
        return hip_status(launch_g2p<float>(c->dp, n, x, (const float *)u, alpha_fx, alpha_real, (float *)u_at,
                                            (float *)alpha_f, s));
    return hip_status(launch_g2p<double>(c->dp, n, x, (const double *)u, alpha_fx, alpha_real, (double *)u_at,
                                         (double *)alpha_f, s));
}

gic_status gic_drag(gic_ctx *c, int64_t n, const double *r, const double *v, const void *u_at, const void *alpha_f,
                    void *f_drag, void *stream)
{
    if (!n_ok(c, n)) return GIC_E_ARG;
    if (n > 0 && (!r || !v || !u_at || !alpha_f || !f_drag)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (fp32(c))
        return hip_status(launch_drag<float>(c->dp, n, r, v, (const float *)u_at, (const float *)alpha_f,
                                             (float *)f_drag, s));
    return hip_status(launch_drag<double>(c->dp, n, r, v, (const double *)u_at, (const double *)alpha_f,
                                          (double *)f_drag, s));
}

gic_status gic_integrate(gic_ctx *c, int64_t n, const double *r, const void *f_contact, const void *f_drag,
                         double *x, double *v, void *stream)
{
    if (!n_ok(c, n)) return GIC_E_ARG;
    if (n > 0 && (!r || !f_contact || !x || !v)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (fp32(c))
        return hip_status(launch_integrate<float>(c->dp, n, r, (const float *)f_contact, (const float *)f_drag, x,
                                                  v, s));
    return hip_status(
        launch_integrate<double>(c->dp, n, r, (const double *)f_contact, (const double *)f_drag, x, v, s));
}

// A call writes len int64 from p: the live flags no longer describe the
// stepping path's grids if p overlaps them.
static void grids_written(gic_ctx *c, const int64_t *p, int64_t len)
{
    if (!c->live_ok || !p) return;
    const int64_t G = c->dp.G;
    auto overlaps = [&](const int64_t *q, int64_t m) { return p < q + m && q < p + len; };
    if (overlaps(c->live_a, G) || overlaps(c->live_m, 3 * G)) c->live_ok = false;
}

gic_status gic_p2g(gic_ctx *c, int64_t n, const double *x, const double *v, const double *r,
                   const int32_t *cell_begin, const int32_t *cell_end, int64_t *alpha_fx, int64_t *mom_fx,
                   int32_t accumulate, void *stream)
{
    if (!n_ok(c, n) || !alpha_fx) return GIC_E_ARG;
    if (n > 0 && (!x || !r || !cell_begin || !cell_end || (mom_fx && !v))) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t G = c->dp.G;
    grids_written(c, alpha_fx, G);
    grids_written(c, mom_fx, 3 * G);
    if (!accumulate) {
        hipError_t e = launch_fill_i64(alpha_fx, G, s);
        if (e == hipSuccess && mom_fx) e = launch_fill_i64(mom_fx, 3 * G, s);
        if (e != hipSuccess) return GIC_E_HIP;
    }
    if (n == 0) return GIC_OK;
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    return hip_status(
        launch_p2g_fixed(c->dp, n, c->K, x, v, r, cell_begin, cell_end, c->bricks, alpha_fx, mom_fx, c->err, s));
}

gic_status gic_p2g_real(gic_ctx *c, int64_t n, const double *x, const double *v, const double *r,
                        const int32_t *cell_begin, const int32_t *cell_end, double *alpha, double *mom,
                        int32_t accumulate, void *stream)
{
    if (!n_ok(c, n) || (!alpha && !mom)) return GIC_E_ARG;
    if (n > 0 && (!x || !r || !cell_begin || !cell_end || (mom && !v))) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n > 0 && brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    return hip_status(launch_p2g_real(c->dp, n, c->K, x, v, r, cell_begin, cell_end, c->bricks, alpha, mom,
                                      accumulate ? 1 : 0, c->fxs, c->fxp, s));
}

gic_status gic_gather_g2p_drag(gic_ctx *c, int64_t n, const int32_t *order, const double *x, const double *v,
                               const double *r, const int32_t *id, double *x_out, double *v_out, double *r_out,
                               int32_t *id_out, const void *u, const int64_t *alpha_fx, const int32_t *cell_begin,
                               const int32_t *cell_end, void *f_drag, void *u_at, void *alpha_f, void *stream)
{
    if (!n_ok(c, n) || !cell_begin || !cell_end) return GIC_E_ARG;
    if (n > 0 && (!order || !x || !v || !r || !x_out || !v_out || !r_out || !u || !alpha_fx || !f_drag))
        return GIC_E_ARG;
    if ((id == nullptr) != (id_out == nullptr) || (u_at == nullptr) != (alpha_f == nullptr)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return GIC_OK;
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    if (fp32(c))
        return hip_status(launch_gather_g2p_drag<float>(c->dp, n, c->K, order, x, v, r, id, x_out, v_out, r_out,
                                                        id_out, (const float *)u, alpha_fx, cell_begin, cell_end,
                                                        c->bricks, (float *)f_drag, (float *)u_at, (float *)alpha_f,
                                                        s));
    return hip_status(launch_gather_g2p_drag<double>(c->dp, n, c->K, order, x, v, r, id, x_out, v_out, r_out, id_out,
                                                     (const double *)u, alpha_fx, cell_begin, cell_end, c->bricks,
                                                     (double *)f_drag, (double *)u_at, (double *)alpha_f, s));
}

static gic_status integrate_p2g_impl(gic_ctx *c, int64_t n, double *x, double *v, const double *r,
                                     const double *held, const void *f_contact, const void *f_drag,
                                     const int32_t *cell_begin, const int32_t *cell_end, int64_t *alpha_fx,
                                     int64_t *mom_fx, int32_t accumulate, void *stream)
{
    if (!n_ok(c, n) || !alpha_fx || !mom_fx || !cell_begin || !cell_end) return GIC_E_ARG;
    if (n > 0 && (!x || !v || !r || !f_contact || !f_drag)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    grids_written(c, alpha_fx, c->dp.G);
    grids_written(c, mom_fx, 3 * c->dp.G);
    if (!accumulate) {
        hipError_t e = launch_fill_i64(alpha_fx, c->dp.G, s);
        if (e == hipSuccess) e = launch_fill_i64(mom_fx, 3 * c->dp.G, s);
        if (e != hipSuccess) return GIC_E_HIP;
    }
    if (n == 0) return GIC_OK;
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    if (fp32(c))
        return hip_status(launch_integrate_p2g<float>(c->dp, n, c->K, x, v, r, (const float *)f_contact,
                                                      (const float *)f_drag, cell_begin, cell_end, c->bricks,
                                                      alpha_fx, mom_fx, c->err, s, held));
    return hip_status(launch_integrate_p2g<double>(c->dp, n, c->K, x, v, r, (const double *)f_contact,
                                                   (const double *)f_drag, cell_begin, cell_end, c->bricks, alpha_fx,
                                                   mom_fx, c->err, s, held));
}

gic_status gic_integrate_p2g(gic_ctx *c, int64_t n, double *x, double *v, const double *r, const void *f_contact,
                             const void *f_drag, const int32_t *cell_begin, const int32_t *cell_end,
                             int64_t *alpha_fx, int64_t *mom_fx, int32_t accumulate, void *stream)
{
    return integrate_p2g_impl(c, n, x, v, r, nullptr, f_contact, f_drag, cell_begin, cell_end, alpha_fx, mom_fx,
                              accumulate, stream);
}

gic_status gic_integrate_p2g_wet(gic_ctx *c, int64_t n, double *x, double *v, const double *r, const double *held,
                                 const void *f_contact, const void *f_drag, const int32_t *cell_begin,
                                 const int32_t *cell_end, int64_t *alpha_fx, int64_t *mom_fx, int32_t accumulate,
                                 void *stream)
{
    if (n > 0 && !held) return GIC_E_ARG;
    return integrate_p2g_impl(c, n, x, v, r, held, f_contact, f_drag, cell_begin, cell_end, alpha_fx, mom_fx,
                              accumulate, stream);
}

// The stepping path's integrate + P2G into freshly written grids: stored
// tiles assembled node by node (no clearing, no grid atomics) when the
// context holds tile storage, else cleared grids and atomics.
static void stage_mark(gic_ctx *c, int k, hipStream_t s);

// Integrate + P2G of the stepping paths, between the stage events 5
// (integrate + P2G) and 7: with tiles, the tile kernel, event 6, then the
// assembly of the grids; otherwise the grid fills, event 5, the atomic
// deposit, event 6 (no assembly).
static gic_status step_integrate_p2g(gic_ctx *c, int64_t n, double *x, double *v, const double *r,
                                     const void *f_contact, const void *f_force, const int32_t *cell_begin,
                                     const int32_t *cell_end, int64_t *alpha_fx, int64_t *mom_fx, hipStream_t s)
{
    if (!c->p2gs.tiles || n == 0) {
        c->live_ok = false;
        if (launch_fill_i64(alpha_fx, c->dp.G, s) != hipSuccess || launch_fill_i64(mom_fx, 3 * c->dp.G, s) != hipSuccess)
            return GIC_E_HIP;
        stage_mark(c, 5, s);
        const gic_status st =
            gic_integrate_p2g(c, n, x, v, r, f_contact, f_force, cell_begin, cell_end, alpha_fx, mom_fx, 1, s);
        stage_mark(c, 6, s);
        return st;
    }
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    stage_mark(c, 5, s);
    P2GStore st = c->p2gs;
    st.full = c->live_ok && c->live_a == alpha_fx && c->live_m == mom_fx ? 0 : 1;
    st.esc_n = c->esc_n2 + c->esc_par;
    uint32_t *next = c->esc_n2 + (c->esc_par ^ 1);
    c->esc_par ^= 1;
    hipError_t e;
    if (fp32(c))
        e = launch_integrate_p2g_store<float>(c->dp, n, c->K, x, v, r, (const float *)f_contact,
                                              (const float *)f_force, cell_begin, cell_end, c->bricks, c->err, s, st,
                                              &c->brick_n);
    else
        e = launch_integrate_p2g_store<double>(c->dp, n, c->K, x, v, r, (const double *)f_contact,
                                               (const double *)f_force, cell_begin, cell_end, c->bricks, c->err, s,
                                               st, &c->brick_n);
    if (e != hipSuccess) return hip_status(e);
    stage_mark(c, 6, s);
    e = launch_p2g_assemble(c->dp, n, x, v, r, c->bricks, alpha_fx, mom_fx, c->err, s, st, next);
    c->live_ok = e == hipSuccess && st.live;
    c->live_a = alpha_fx;
    c->live_m = mom_fx;
    return hip_status(e);
}

// Stage event k of the current timed step (no-op unless timing is on and
// the event buffer has room).
static void stage_mark(gic_ctx *c, int k, hipStream_t s)
{
    if (c->tm_used < c->tm_cap) (void)hipEventRecord(c->tm_ev[c->tm_used * kStageEvents + k], s);
}

static void stage_done(gic_ctx *c)
{
    if (c->tm_used < c->tm_cap) ++c->tm_used;
}

gic_status gic_stage_timing(gic_ctx *c, int32_t max_steps)
{
    if (!c || max_steps < 0) return GIC_E_ARG;
    if (c->tm_ev) {
        (void)hipDeviceSynchronize();
        for (int i = 0; i < c->tm_cap * kStageEvents; ++i) (void)hipEventDestroy(c->tm_ev[i]);
        delete[] c->tm_ev;
    }
    c->tm_ev = nullptr;
    c->tm_cap = c->tm_used = 0;
    if (max_steps == 0) return GIC_OK;
    c->tm_ev = new hipEvent_t[(size_t)max_steps * kStageEvents];
    for (int i = 0; i < max_steps * kStageEvents; ++i)
        if (hipEventCreate(&c->tm_ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->tm_ev[j]);
            delete[] c->tm_ev;
            c->tm_ev = nullptr;
            return GIC_E_HIP;
        }
    c->tm_cap = max_steps;
    return GIC_OK;
}

gic_status gic_stage_times(gic_ctx *c, void *stream, double *ms, int32_t *steps)
{
    if (!c || !ms || !steps) return GIC_E_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return GIC_E_HIP;
    for (int k = 0; k < kStageEvents - 1; ++k) ms[k] = 0.0;
    for (int t = 0; t < c->tm_used; ++t)
        for (int k = 0; k < kStageEvents - 1; ++k) {
            float e = 0.0f;
            if (hipEventElapsedTime(&e, c->tm_ev[t * kStageEvents + k], c->tm_ev[t * kStageEvents + k + 1]) !=
                hipSuccess)
                return GIC_E_HIP;
            ms[k] += (double)e;
        }
    *steps = c->tm_used;
    c->tm_used = 0;
    return GIC_OK;
}

gic_status gic_step(gic_ctx *c, int64_t n, const double *x_cur, const double *v_cur, const double *r_cur,
                    const int32_t *id_cur, double *x_nxt, double *v_nxt, double *r_nxt, int32_t *id_nxt,
                    const void *u, int64_t *alpha_fx, int64_t *mom_fx, uint32_t *key, int32_t *order,
                    int32_t *cell_begin, int32_t *cell_end, void *f_contact, void *f_drag, void *u_at,
                    void *alpha_f, void *stream)
{
    if (!n_ok(c, n) || !alpha_fx || !mom_fx || !cell_begin || !cell_end) return GIC_E_ARG;
    if (n > 0 && (!x_cur || !v_cur || !r_cur || !x_nxt || !v_nxt || !r_nxt || !u || !key || !order ||
                  !f_contact || !f_drag))
        return GIC_E_ARG;
    if ((id_cur == nullptr) != (id_nxt == nullptr) || (u_at == nullptr) != (alpha_f == nullptr)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    // the neighbour list of the last step is kept when this step continues
    // that step's state (the sort then checks order and displacement)
    const int force = !(c->nl_n == n && c->nl_x == x_cur && c->sort.last_n == n);
    c->nl_n = -1;
    stage_mark(c, 0, s);
    if (step_sort(c, n, x_cur, key, order, cell_begin, cell_end, force, s) != hipSuccess) return GIC_E_HIP;
    stage_mark(c, 1, s);
    c->in_step = true;  // the stages below share this brick list
    // alpha_fx was deposited at the current positions and is read by node,
    // so the gather into sorted order does not change it
    gic_status st = gic_gather_g2p_drag(c, n, order, x_cur, v_cur, r_cur, id_cur, x_nxt, v_nxt, r_nxt, id_nxt, u,
                                        alpha_fx, cell_begin, cell_end, f_drag, u_at, alpha_f, stream);
    stage_mark(c, 2, s);
    if (st == GIC_OK && n > 0)
        st = contact_impl(c, n, x_nxt, v_nxt, r_nxt, cell_begin, cell_end, f_contact, nullptr, nullptr, 0, force, s);
    stage_mark(c, 3, s);
    stage_mark(c, 4, s);  // no exchange deposit in this step
    if (st == GIC_OK)
        st = step_integrate_p2g(c, n, x_nxt, v_nxt, r_nxt, f_contact, f_drag, cell_begin, cell_end, alpha_fx, mom_fx,
                                s);
    stage_mark(c, 7, s);
    stage_done(c);
    c->in_step = false;
    if (st == GIC_OK) {
        c->nl_n = n;  // the list holds the sorted order of the state now in x_nxt
        c->nl_x = x_nxt;
    }
    return st;
}

/* ---- remaining interphase forces and the sand step ----------------------- */

gic_status gic_gather_g2p_fluid(gic_ctx *c, int64_t n, const int32_t *order, const double *x, const double *v,
                                const double *r, const int32_t *id, double *x_out, double *v_out, double *r_out,
                                int32_t *id_out, const void *u, const int64_t *alpha_fx, const void *grad_p,
                                const void *acc_f, const int32_t *cell_begin, const int32_t *cell_end,
                                void *f_fluid, const double *held, double *held_out, void *stream)
{
    if (!n_ok(c, n) || !cell_begin || !cell_end) return GIC_E_ARG;
    if (n > 0 && (!order || !x || !v || !r || !x_out || !v_out || !r_out || !u || !alpha_fx || !f_fluid))
        return GIC_E_ARG;
    if ((id == nullptr) != (id_out == nullptr) || (held == nullptr) != (held_out == nullptr)) return GIC_E_ARG;
    if (n > 0 && (x_out == x || v_out == v || r_out == r || (id && id_out == id) || (held && held_out == held)))
        return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return GIC_OK;
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    if (fp32(c))
        return hip_status(launch_gather_g2p_fluid<float>(
            c->dp, n, c->K, order, x, v, r, id, x_out, v_out, r_out, id_out, (const float *)u, alpha_fx,
            (const float *)grad_p, (const float *)acc_f, cell_begin, cell_end, c->bricks, (float *)f_fluid, s, held,
            held_out));
    return hip_status(launch_gather_g2p_fluid<double>(
        c->dp, n, c->K, order, x, v, r, id, x_out, v_out, r_out, id_out, (const double *)u, alpha_fx,
        (const double *)grad_p, (const double *)acc_f, cell_begin, cell_end, c->bricks, (double *)f_fluid, s, held,
        held_out));
}

gic_status gic_exchange_p2g(gic_ctx *c, int64_t n, const double *x, const double *r, const void *f_contact,
                            const void *f_fluid, const int32_t *cell_begin, const int32_t *cell_end, double weight,
                            int64_t *fs_fx, const double *held, void *stream)
{
    if (!n_ok(c, n) || !cell_begin || !cell_end || !fs_fx) return GIC_E_ARG;
    if (n > 0 && (!x || !r || !f_contact || !f_fluid)) return GIC_E_ARG;
    if (!(c->p.f_unit > 0.0) || !isfinite(weight)) return GIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    grids_written(c, fs_fx, 3 * c->dp.G);
    if (n == 0) return GIC_OK;
    if (brick_list(c, cell_begin, cell_end, s) != hipSuccess) return GIC_E_HIP;
    const double exsc = -weight / c->p.f_unit;
    if (fp32(c))
        return hip_status(launch_exchange_p2g<float>(c->dp, n, c->K, x, r, (const float *)f_contact,
                                                     (const float *)f_fluid, cell_begin, cell_end, c->bricks, exsc,
                                                     fs_fx, c->err, s, held));
    return hip_status(launch_exchange_p2g<double>(c->dp, n, c->K, x, r, (const double *)f_contact,
                                                  (const double *)f_fluid, cell_begin, cell_end, c->bricks, exsc,
                                                  fs_fx, c->err, s, held));
}

gic_status gic_sand_step(gic_ctx *c, int64_t n, double Dt, double *x_a, double *v_a, double *r_a, int32_t *id_a,
                         double *x_b, double *v_b, double *r_b, int32_t *id_b, const void *u, const void *grad_p,
                         const void *acc_f, int64_t *alpha_fx, int64_t *mom_fx, int64_t *fs_fx, uint32_t *key,
                         int32_t *order, int32_t *cell_begin, int32_t *cell_end, void *f_contact, void *f_fluid,
                         int32_t *nsub, int32_t *which, void *stream)
{
    if (!n_ok(c, n) || !alpha_fx || !mom_fx || !cell_begin || !cell_end || !nsub || !which) return GIC_E_ARG;
    if (!(Dt > 0.0) || !isfinite(Dt)) return GIC_E_ARG;
    if (n > 0 && (!x_a || !v_a || !r_a || !x_b || !v_b || !r_b || !u || !key || !order || !f_contact || !f_fluid))
        return GIC_E_ARG;
    if ((id_a == nullptr) != (id_b == nullptr)) return GIC_E_ARG;
    if (fs_fx && !(c->p.f_unit > 0.0)) return GIC_E_ARG;
    const double q = ceil(Dt / c->p.dt);
    if (!(q < 2147483647.0)) return GIC_E_ARG;
    const int32_t N = q < 1.0 ? 1 : (int32_t)q;
    const double dt_sub = Dt / (double)N;
    const double weight = dt_sub / Dt;
    hipStream_t s = (hipStream_t)stream;
    const double dt_keep = c->dp.dt;
    c->dp.dt = dt_sub;  // the sub-steps' length, captured by value at each launch
    gic_status st = GIC_OK;
    for (int32_t i = 0; i < N && st == GIC_OK; ++i) {
        const bool even = (i & 1) == 0;
        double *xc = even ? x_a : x_b, *vc = even ? v_a : v_b, *rc = even ? r_a : r_b;
        double *xn = even ? x_b : x_a, *vn = even ? v_b : v_a, *rn = even ? r_b : r_a;
        int32_t *ic = even ? id_a : id_b, *in = even ? id_b : id_a;
        const int force = !(c->nl_n == n && c->nl_x == xc && c->sort.last_n == n);
        c->nl_n = -1;
        stage_mark(c, 0, s);
        if (step_sort(c, n, xc, key, order, cell_begin, cell_end, force, s) != hipSuccess) {
            st = GIC_E_HIP;
            break;
        }
        stage_mark(c, 1, s);
        c->in_step = true;  // the stages below share this brick list
        st = gic_gather_g2p_fluid(c, n, order, xc, vc, rc, ic, xn, vn, rn, in, u, alpha_fx, grad_p, acc_f,
                                  cell_begin, cell_end, f_fluid, nullptr, nullptr, stream);
        stage_mark(c, 2, s);
        if (st == GIC_OK && n > 0)
            st = contact_impl(c, n, xn, vn, rn, cell_begin, cell_end, f_contact, nullptr, nullptr, 0, force, s);
        stage_mark(c, 3, s);
        if (st == GIC_OK && fs_fx)
            st = gic_exchange_p2g(c, n, xn, rn, f_contact, f_fluid, cell_begin, cell_end, weight, fs_fx, nullptr,
                                  stream);
        stage_mark(c, 4, s);
        if (st == GIC_OK)
            st = step_integrate_p2g(c, n, xn, vn, rn, f_contact, f_fluid, cell_begin, cell_end, alpha_fx, mom_fx, s);
        stage_mark(c, 7, s);
        stage_done(c);
        c->in_step = false;
        if (st == GIC_OK) {
            c->nl_n = n;
            c->nl_x = xn;
        }
    }
    c->dp.dt = dt_keep;
    *nsub = N;
    *which = N & 1;
    return st;
}

/* ---- adjoint form (double) ---------------------------------------------- */

gic_status gic_contact_forces_vjp(gic_ctx *c, int64_t n, const double *x, const double *v, const double *r,
                                  const int32_t *cell_begin, const int32_t *cell_end, const double *g_f, double *g_x,
                                  double *g_v, double *g_mu, void *stream)
{
    if (c && (c->p.drag_model != 0 || c->p.vmass != 0)) return GIC_E_ARG;  // the adjoint covers the linear drag only
    if (!n_ok(c, n) || fp32(c)) return GIC_E_ARG;
    if (n > 0 && (!x || !v || !r || !cell_begin || !cell_end || !g_f || !g_x || !g_v || !g_mu)) return GIC_E_ARG;
    return hip_status(launch_contact_vjp(c->dp, n, x, v, r, cell_begin, cell_end, g_f, g_x, g_v, g_mu,
                                         (hipStream_t)stream));
}

gic_status gic_drag_vjp(gic_ctx *c, int64_t n, const double *r, const double *v, const double *u_at,
                        const double *alpha_f, const double *g_f, double *g_v, double *g_u_at, double *g_alpha_f,
                        double *g_cdrag, void *stream)
{
    if (c && (c->p.drag_model != 0 || c->p.vmass != 0)) return GIC_E_ARG;  // the adjoint covers the linear drag only
    if (!n_ok(c, n) || fp32(c)) return GIC_E_ARG;
    if (n > 0 && (!r || !v || !u_at || !alpha_f || !g_f || !g_v || !g_u_at || !g_alpha_f || !g_cdrag))
        return GIC_E_ARG;
    return hip_status(
        launch_drag_vjp(c->dp, n, r, v, u_at, alpha_f, g_f, g_v, g_u_at, g_alpha_f, g_cdrag, (hipStream_t)stream));
}

gic_status gic_integrate_vjp(gic_ctx *c, int64_t n, const double *r, const double *g_x, double *g_v, double *g_f,
                             void *stream)
{
    if (c && (c->p.drag_model != 0 || c->p.vmass != 0)) return GIC_E_ARG;  // the adjoint covers the linear drag only
    if (!n_ok(c, n) || fp32(c)) return GIC_E_ARG;
    if (n > 0 && (!r || !g_x || !g_v || !g_f)) return GIC_E_ARG;
    return hip_status(launch_integrate_vjp(c->dp, n, r, g_x, g_v, g_f, (hipStream_t)stream));
}

gic_status gic_g2p_vjp(gic_ctx *c, int64_t n, const double *x, const double *u, const double *alpha_real,
                       const double *g_u_at, const double *g_alpha_f, const int32_t *cell_begin,
                       const int32_t *cell_end, double *g_x, double *g_alpha, void *stream)
{
    if (c && (c->p.drag_model != 0 || c->p.vmass != 0)) return GIC_E_ARG;  // the adjoint covers the linear drag only
    if (!n_ok(c, n) || fp32(c)) return GIC_E_ARG;
    if (n > 0 && (!x || !u || !alpha_real || !g_u_at || !g_alpha_f || !g_x)) return GIC_E_ARG;
    if (n > 0 && g_alpha && (!cell_begin || !cell_end)) return GIC_E_ARG;
    if (n > 0 && g_alpha && brick_list(c, cell_begin, cell_end, (hipStream_t)stream) != hipSuccess)
        return GIC_E_HIP;
    return hip_status(launch_g2p_vjp(c->dp, n, c->K, x, u, alpha_real, g_u_at, g_alpha_f, cell_begin, cell_end,
                                     c->bricks, g_x, g_alpha, c->fxs, c->fxp, (hipStream_t)stream));
}

gic_status gic_p2g_vjp(gic_ctx *c, int64_t n, const double *x, const double *v, const double *r,
                       const double *g_alpha, const double *g_mom, double *g_x, double *g_v, void *stream)
{
    if (c && (c->p.drag_model != 0 || c->p.vmass != 0)) return GIC_E_ARG;  // the adjoint covers the linear drag only
    if (!n_ok(c, n)) return GIC_E_ARG;
    if (n > 0 && (!x || !r || !g_x || (g_mom && (!v || !g_v)) || (!g_alpha && !g_mom))) return GIC_E_ARG;
    return hip_status(launch_p2g_vjp(c->dp, n, x, v, r, g_alpha, g_mom, g_x, g_v, (hipStream_t)stream));
}

gic_status gic_sum(gic_ctx *c, int64_t n, const double *a, const double *b, double *out, int32_t accumulate,
                   void *stream)
{
    if (!c || n < 0 || !out || (n > 0 && !a)) return GIC_E_ARG;
    return hip_status(launch_sum(a, b, n, c->part, kSumParts, out, accumulate ? 1 : 0, (hipStream_t)stream));
}

// Partial sums of gic_sum_noalloc: a fixed array per device, so that the
// call needs neither a context nor an allocation.  Host code uses the
// per-device address from hipGetSymbolAddress, never the symbol itself.
static __device__ __align__(256) double scratch[kSumParts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices];  // address of `scratch` on each device, once looked up

// Address of this device's scratch array (looked up on the first call on the
// device, with it current), or NULL on failure.
double *device_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

gic_status gic_sum_noalloc(int64_t n, const double *a, const double *b, double *out, int32_t accumulate,
                           void *stream)
{
    if (n < 0 || !out || (n > 0 && !a)) return GIC_E_ARG;
    if (n > kSumNoallocMax) return GIC_E_ARG;
    double *part = device_scratch();
    if (!part) return GIC_E_HIP;
    return hip_status(launch_sum(a, b, n, part, kSumParts, out, accumulate ? 1 : 0, (hipStream_t)stream));
}

gic_status gic_scale(gic_ctx *c, int64_t n, const double *a, const double *s, double factor, double *out,
                     void *stream)
{
    if (!c || n < 0 || (n > 0 && (!a || !s || !out)) || !isfinite(factor)) return GIC_E_ARG;
    return hip_status(launch_scale(n, a, s, factor, out, (hipStream_t)stream));
}

gic_status gic_permute(gic_ctx *c, int64_t n, int32_t comps, const int32_t *order, const double *in, double *out,
                       int32_t scatter, void *stream)
{
    if (!n_ok(c, n) || comps < 1 || comps > 6) return GIC_E_ARG;
    if (n > 0 && (!order || !in || !out || in == out)) return GIC_E_ARG;
    return hip_status(launch_permute(n, comps, order, in, out, scatter ? 1 : 0, (hipStream_t)stream));
}

int64_t gic_idp_workspace_bytes(const gic_ctx *c)
{
    if (!c) return -1;
    return idp_work_bytes(idp_dims(c->dp));
}

gic_status gic_idp_setup(gic_ctx *c, const int64_t *alpha_fx, const double *alpha_star, const uint8_t *label,
                         double *alpha_t, double *rhs, void *stream)
{
    if (!c || !alpha_fx || !alpha_star || !label || !alpha_t || !rhs) return GIC_E_ARG;
    return hip_status(launch_idp_setup(idp_dims(c->dp), c->dp.alpha_max, alpha_fx, alpha_star, label, alpha_t, rhs,
                                       c->err, (hipStream_t)stream));
}

gic_status gic_idp_apply(gic_ctx *c, const double *alpha_t, const uint8_t *label, const double *q, double *out,
                         void *stream)
{
    if (!c || !alpha_t || !label || !q || !out || out == q) return GIC_E_ARG;
    return hip_status(launch_idp_apply(idp_dims(c->dp), alpha_t, label, q, out, (hipStream_t)stream));
}

gic_status gic_idp_solve(gic_ctx *c, const double *alpha_t, const uint8_t *label, const double *rhs, double *q,
                         void *work, int32_t max_iter, double tol, int32_t check_every, int32_t precond,
                         int32_t *iters, double *relres, void *stream)
{
    if (!c || !alpha_t || !label || !rhs || !q || !work || max_iter < 0 || check_every < 1) return GIC_E_ARG;
    if (!(tol >= 0.0) || !isfinite(tol) || (precond != 0 && precond != 1)) return GIC_E_ARG;
    double *at_w, *s_w;
    const IdpWork W = idp_carve(work, idp_dims(c->dp), precond, &at_w, &s_w);
    return idp_cg(c, alpha_t, label, rhs, q, W, max_iter, tol, check_every, iters, relres, (hipStream_t)stream);
}

gic_status gic_idp_displacement(gic_ctx *c, const double *q, const uint8_t *label, double *fx, double *fy,
                                double *fz, void *stream)
{
    if (!c || !q || !label || !fx || !fy || !fz) return GIC_E_ARG;
    return hip_status(launch_idp_faces(idp_dims(c->dp), c->p.dx, q, label, fx, fy, fz, (hipStream_t)stream));
}

gic_status gic_density_projection(gic_ctx *c, const int64_t *alpha_fx, const double *alpha_star,
                                  const uint8_t *label, double *q, double *fx, double *fy, double *fz, void *work,
                                  int32_t max_iter, double tol, int32_t check_every, int32_t precond,
                                  int32_t *iters, double *relres, void *stream)
{
    if (!c || !alpha_fx || !alpha_star || !label || !q || !fx || !fy || !fz || !work) return GIC_E_ARG;
    if (max_iter < 0 || check_every < 1 || !(tol >= 0.0) || !isfinite(tol)) return GIC_E_ARG;
    if (precond != 0 && precond != 1) return GIC_E_ARG;
    const IdpDims D = idp_dims(c->dp);
    hipStream_t s = (hipStream_t)stream;
    double *at, *rhs;
    const IdpWork W = idp_carve(work, D, precond, &at, &rhs);
    if (launch_idp_setup(D, c->dp.alpha_max, alpha_fx, alpha_star, label, at, rhs, c->err, s) != hipSuccess)
        return GIC_E_HIP;
    const gic_status st = idp_cg(c, at, label, rhs, q, W, max_iter, tol, check_every, iters, relres, s);
    if (st != GIC_OK) return st;
    return hip_status(launch_idp_faces(D, c->p.dx, q, label, fx, fy, fz, s));
}

}  // extern "C"
