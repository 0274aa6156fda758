// Device-side definitions shared by the gfx950 kernels of the granule path.
//
// Paper: Tang, Zhu, Ni, Chen, "The Granule-In-Cell Method for Simulating
// Sand-Water Mixtures", ACM TOG 44(6) 2025 (arXiv 2504.00745).
//
// Everything that decides an integer (cell keys, the contact test, B-spline
// weights that feed fixed-point rounding) is written with FMA contraction off,
// one rounding per operation in the order written, so that these decisions
// are reproducible operation by operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gic {

#define GIC_PI 3.14159265358979323846
#define GIC_C43PI (4.0 * GIC_PI / 3.0)
#define GIC_C12PI (12.0 * GIC_PI)
#define GIC_TWO32 4294967296.0
#define GIC_TWOM32 (1.0 / 4294967296.0)
constexpr int kBrick = 4;                 // cells per brick edge in the key
constexpr int kBrickCells = kBrick * kBrick * kBrick;

// Workgroups are handed to the 8 XCDs round robin (workgroup b runs on XCD
// b mod 8), and each XCD has its own L2.  Kernels whose neighbouring
// workgroups read overlapping data remap their workgroup index so that each
// XCD runs one contiguous eighth of the logical workgroups.  Launch with
// xcd_grid(nlogical) workgroups; xcd_block returns the logical index or -1.
constexpr int kXcds = 8;

inline unsigned xcd_grid(int64_t nlogical)
{
    const int64_t per = (nlogical + kXcds - 1) / kXcds;
    return (unsigned)(per * kXcds > 0 ? per * kXcds : kXcds);
}

__device__ inline int64_t xcd_block(int64_t nlogical)
{
    const int64_t per = (nlogical + kXcds - 1) / kXcds;
    const int64_t b = blockIdx.x;
    const int64_t l = (b % kXcds) * per + b / kXcds;
    return l < nlogical ? l : -1;
}

// Brick kernels run over the list of occupied bricks, in brick order (a bed
// often fills only part of the box); each XCD takes one contiguous eighth
// of the list, so the load is even and neighbouring bricks, which read
// overlapping cells and nodes, mostly share an L2.  Launch with
// brick_grid(nbricks) workgroups (an upper bound of the list length);
// brick_of_block returns the brick or -1.
inline unsigned brick_grid(int64_t nbricks) { return xcd_grid(nbricks); }

__device__ inline int64_t brick_of_block(const int32_t *__restrict__ list, const int32_t *__restrict__ count)
{
    const int64_t nocc = *count;
    const int64_t per = (nocc + kXcds - 1) / kXcds;  // list entries per XCD
    const int64_t b = blockIdx.x;
    const int64_t j = b / kXcds;  // slot on the XCD; the grid has slots to spare
    const int64_t l = (b % kXcds) * per + j;
    return j < per && l < nocc ? list[l] : -1;
}

// Brick kernels that loop: workgroup b takes the entries j = b / kXcds +
// it * (gridDim.x / kXcds), it = 0, 1, ..., of its XCD's eighth of the list
// (the same split as brick_of_block); -1 when it has no more.  The grid is
// brick_loop_grid(nbricks) workgroups (a multiple of kXcds).
constexpr int64_t kBrickLoopGrid = 2048;
inline unsigned brick_loop_grid(int64_t nbricks)
{
    const unsigned g = xcd_grid(nbricks);
    return g < (unsigned)kBrickLoopGrid ? g : (unsigned)kBrickLoopGrid;
}

__device__ inline int64_t brick_at(const int32_t *__restrict__ list, const int32_t *__restrict__ count, int64_t it)
{
    const int64_t nocc = *count;
    const int64_t per = (nocc + kXcds - 1) / kXcds;
    const int64_t j = (int64_t)blockIdx.x / kXcds + it * ((int64_t)gridDim.x / kXcds);
    const int64_t l = ((int64_t)blockIdx.x % kXcds) * per + j;
    return j < per && l < nocc ? list[l] : -1;
}

// brick_of_block that also gives the brick's position in the list.
__device__ inline int64_t brick_slot_of_block(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                                              int64_t &slot)
{
    const int64_t nocc = *count;
    const int64_t per = (nocc + kXcds - 1) / kXcds;
    const int64_t b = blockIdx.x;
    const int64_t j = b / kXcds;
    slot = (b % kXcds) * per + j;
    return j < per && slot < nocc ? list[slot] : -1;
}

// A range [b, e) of sorted positions read from caller-given cell ranges,
// clipped to [0, n]: ranges that do not match the positions give wrong
// results (and, where detected, a latched error) but never an access
// outside the arrays.
__device__ inline void clip_range(int64_t n, int32_t &b, int32_t &e)
{
    b = b < 0 ? 0 : (b > n ? (int32_t)n : b);
    e = e < b ? b : (e > n ? (int32_t)n : e);
}

// Latched error codes (same values as gic_status).
constexpr int kErrDomain = 4;
constexpr int kErrNonFinite = 5;
constexpr int kErrRange = 6;

// Parameters as the kernels use them: derived constants precomputed on the
// host once per context.
struct DevParams {
    int32_t n[3];       // grid nodes per axis
    int32_t nc[3];      // neighbour cells per axis
    int32_t nb[3];      // bricks per axis
    int32_t tile;       // P2G LDS tile edge (nodes)
    int64_t G;          // nodes
    double dx, inv_dx, inv_vcell;
    double cell, inv_cell;
    double L[3];        // box edges n_a dx
    double kn, zeta, kt_ratio, mu;
    double rho_s, cdrag;  // cdrag = c_drag 6 pi eta_f
    double c_drag, cdrag_unit;  // C_d and 6 pi eta_f separately (adjoint)
    double alpha_max;   // clamp of alpha_s: 0.740, times (1 + r_max) when granules absorb water (Sec. 5.3)
    double g[3], dt;
    double r_max, search_scale;
    uint32_t walls;
    // remaining interphase forces (Sec. 3.3 Eq. 5a-5c, Sec. 5.2 Eq. 9)
    double rho_f, half_rho_f;  // fluid density and rho_f / 2 (virtual mass per volume)
    double c_quad;             // coefficient of the quadratic drag
    int32_t drag_model;        // 0: linear Stokes form x alpha_f; 1: quadratic of Eq. 5b
    int32_t vmass;             // 1: virtual mass, effective mass m + rho_f V / 2
    // capillary (concentration-gradient) pair force, Sec. 5.4
    double sigma, vbridge, sr_peak;  // surface tension, bridge volume / granule volume, peak of Gamma
    double dr_max;                   // rupture distance of the largest pair (search reach)
};

// Latch the first error: code and granule index.
__device__ inline void raise_error(int64_t *err, int code, int64_t idx)
{
    unsigned long long *e = reinterpret_cast<unsigned long long *>(err);
    if (atomicCAS(e, 0ull, (unsigned long long)code) == 0ull) atomicExch(e + 1, (unsigned long long)idx);
}

__device__ inline double volume_of(double r)
{
#pragma clang fp contract(off)
    return ((GIC_C43PI * r) * r) * r;
}

__device__ inline double mass_of(const DevParams &P, double r) { return P.rho_s * volume_of(r); }

// Mass of a wet granule that holds water of `held` times its own volume
// (Sec. 5.3, Eq. 19): V (rho_s + held rho_f).
__device__ inline double wet_mass(const DevParams &P, double r, double held)
{
#pragma clang fp contract(off)
    return volume_of(r) * (P.rho_s + held * P.rho_f);
}

// Volume the fluid sees of a wet granule (Sec. 5.3: the absorbed water
// counts as extra volume): V (1 + held), V exactly when held = 0.
__device__ inline double wet_volume(double r, double held)
{
#pragma clang fp contract(off)
    const double V = volume_of(r);
    return held != 0.0 ? V + V * held : V;
}

// clamp(floor(x / cell), 0, nc - 1); NaN -> 0.
__device__ inline int32_t cell_coord(double x, double inv_cell, int32_t nc)
{
#pragma clang fp contract(off)
    double t = floor(x * inv_cell);
    if (!(t >= 0.0)) return 0;
    if (t > (double)(nc - 1)) return nc - 1;
    return (int32_t)t;
}

__device__ inline uint32_t key_of_cell(const DevParams &P, int32_t cx, int32_t cy, int32_t cz)
{
    uint32_t brick = (uint32_t)(((cz / kBrick) * P.nb[1] + (cy / kBrick)) * P.nb[0] + (cx / kBrick));
    uint32_t local = (uint32_t)(((cz % kBrick) * kBrick + (cy % kBrick)) * kBrick + (cx % kBrick));
    return brick * (uint32_t)kBrickCells + local;
}

// Quadratic B-spline stencil on cell-centred nodes.  base = floor(t - 1),
// f = (t - base) - 1/2 in [1/2, 3/2) is the distance to the first node;
// weights N(f), N(f-1), N(2-f).  Node indices are folded into [0, n-1].
struct Stencil {
    int32_t node[3][3];
    double w[3][3];
};

__device__ inline void stencil_of(const DevParams &P, const double xa[3], Stencil &s)
{
#pragma clang fp contract(off)
    for (int a = 0; a < 3; ++a) {
        double t = xa[a] * P.inv_dx;
        double fb = floor(t - 1.0);
        double f = (t - fb) - 0.5;
        double c0 = 1.5 - f, c1 = f - 1.0, c2 = f - 0.5;
        s.w[a][0] = 0.5 * (c0 * c0);
        s.w[a][1] = 0.75 - c1 * c1;
        s.w[a][2] = 0.5 * (c2 * c2);
        double hi = (double)P.n[a];
        if (!(fb >= -2.0)) fb = -2.0;
        if (fb > hi) fb = hi;
        int32_t b = (int32_t)fb;
        for (int k = 0; k < 3; ++k) {
            int32_t id = b + k;
            id = id < 0 ? 0 : id;
            id = id > P.n[a] - 1 ? P.n[a] - 1 : id;
            s.node[a][k] = id;
        }
    }
}

// Derivative of the 1-D weights with respect to x (per metre).
__device__ inline void stencil_dw(const DevParams &P, const double xa[3], double dw[3][3])
{
    for (int a = 0; a < 3; ++a) {
        double t = xa[a] * P.inv_dx;
        double fb = floor(t - 1.0);
        double f = (t - fb) - 0.5;
        dw[a][0] = -(1.5 - f) * P.inv_dx;
        dw[a][1] = (-2.0 * (f - 1.0)) * P.inv_dx;
        dw[a][2] = (f - 0.5) * P.inv_dx;
    }
}

__device__ inline int64_t node_index(const DevParams &P, int32_t i, int32_t j, int32_t k)
{
    return (int64_t)i + (int64_t)P.n[0] * ((int64_t)j + (int64_t)P.n[1] * k);
}

// rint (round half to even) to int64 for |v| < 2^51: adding 1.5 * 2^52 puts
// the value in [2^52, 2^53) where the unit in the last place is 1, so the
// add itself rounds to an integer; the integer is then the difference of the
// bit patterns.
__device__ inline int64_t rint_i64(double v)
{
#pragma clang fp contract(off)
    const double M = 6755399441055744.0;
    double y = v + M;
    return __double_as_longlong(y) - __double_as_longlong(M);
}

// Sampled fluid velocity and fluid fraction at a granule (Sec. 5.2; clamp of
// Sec. 5.1): u_at = sum_k w_k u_k, alpha_f = 1 - sum_k w_k min(alpha_k,
// alpha_max) over the 27 stencil nodes, weights and sums in T.  fetch(i, j,
// k, u[3], al) supplies node (i, j, k)'s velocity and its clamped solid
// fraction; the same summation order serves every caller.
// extra(w) runs after each fetch with that node's weight (further channels
// sampled with the same weights, e.g. by the fluid gather).
struct NoExtra {
    template <typename T>
    __device__ void operator()(T) const {}
};

template <typename T, typename Fetch, typename Extra = NoExtra>
__device__ inline void g2p_sample_st(const Stencil &s, Fetch &&fetch, T uat[3], T &af, Extra &&extra = Extra())
{
    T acc[3] = {(T)0, (T)0, (T)0};
    T as = (T)0;
    // the z-planes' weights and nodes rotate through registers: a stencil
    // indexed with the loop counter would be placed in scratch memory
    double wz = s.w[2][0], wz1 = s.w[2][1], wz2 = s.w[2][2];
    int32_t nz = s.node[2][0], nz1 = s.node[2][1], nz2 = s.node[2][2];
#pragma unroll 1
    for (int cz = 0; cz < 3; ++cz) {  // one node plane at a time keeps few loads in flight per lane
        for (int cy = 0; cy < 3; ++cy) {
            const double wyz = s.w[1][cy] * wz;
            for (int cx = 0; cx < 3; ++cx) {
                const T w = (T)(s.w[0][cx] * wyz);
                T u[3], al;
                fetch(s.node[0][cx], s.node[1][cy], nz, u, al);
                acc[0] += w * u[0];
                acc[1] += w * u[1];
                acc[2] += w * u[2];
                as += w * al;
                extra(w);
            }
        }
        wz = wz1;
        wz1 = wz2;
        nz = nz1;
        nz1 = nz2;
    }
    uat[0] = acc[0];
    uat[1] = acc[1];
    uat[2] = acc[2];
    af = (T)1 - as;
}

template <typename T, typename Fetch>
__device__ inline void g2p_sample(const DevParams &P, const double xa[3], Fetch &&fetch, T uat[3], T &af)
{
    Stencil s;
    stencil_of(P, xa, s);
    g2p_sample_st<T>(s, fetch, uat, af);
}

// Solid fraction of a node for G2P: fixed point to cell volumes, clamped.
__device__ inline double node_alpha(const DevParams &P, int64_t afx)
{
    const double al = (double)afx * GIC_TWOM32;
    return al > P.alpha_max ? P.alpha_max : al;
}
__device__ inline double node_alpha_real(const DevParams &P, double a) { return a > P.alpha_max ? P.alpha_max : a; }

// Drag.  Linear (drag_model 0): Eq. (5b) in the Stokes form of App. A,
// scaled by the fluid fraction, F_d = C_d 6 pi eta_f r alpha_f (u_at - v).
// Quadratic (drag_model 1): Eq. (5b) as printed, F_d = 12 pi r^2 rho_f C
// |u_at - v| (u_at - v) with C the dimensionless coefficient c_quad.
template <typename T>
__device__ inline void drag_one(const DevParams &P, double r, const double v[3], const T uat[3], T af, T Fd[3])
{
#pragma clang fp contract(off)  // one rounding per operation in every kernel that inlines it
    if (P.drag_model == 1) {
        T w[3];
        for (int a = 0; a < 3; ++a) w[a] = uat[a] - (T)v[a];
        const T s2 = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
        T sp;
        if constexpr (sizeof(T) == sizeof(float))
            sp = __builtin_amdgcn_sqrtf(s2);
        else
            sp = sqrt(s2);
        const T coef = (T)((((GIC_C12PI * r) * r) * P.rho_f) * P.c_quad);
        for (int a = 0; a < 3; ++a) Fd[a] = (coef * sp) * w[a];
        return;
    }
    const T beta = (T)(P.cdrag * r) * af;
    for (int a = 0; a < 3; ++a) Fd[a] = beta * (uat[a] - (T)v[a]);
}

// Semi-implicit Euler (Sec. 4): v += dt ((F_c + F_d) / m + g), then x += dt v.
// With virtual mass (Eq. 9) the effective mass is m + rho_f V / 2 and
// gravity acts on m: v += dt ((F_c + F_d) + m g) / (m + rho_f V / 2).
// m: the granule's mass (rho_s V, or the wet mass of Eq. 19); vol: the
// volume of the virtual mass (V, or V (1 + held) for a wet granule).
template <typename T>
__device__ inline void integrate_one_m(const DevParams &P, double vol, double m, const T Fc[3], const T *Fd,
                                       double x[3], double v[3])
{
#pragma clang fp contract(off)  // one rounding per operation in every kernel that inlines it
    if (P.vmass) {
        const double me = m + P.half_rho_f * vol;
        for (int a = 0; a < 3; ++a) {
            double f = (double)Fc[a];
            if (Fd) f += (double)Fd[a];
            const double vn = v[a] + P.dt * ((f + m * P.g[a]) / me);
            v[a] = vn;
            x[a] = x[a] + P.dt * vn;
        }
        return;
    }
    const double inv_m = 1.0 / m;
    for (int a = 0; a < 3; ++a) {
        double f = (double)Fc[a];
        if (Fd) f += (double)Fd[a];
        const double vn = v[a] + P.dt * (f * inv_m + P.g[a]);
        v[a] = vn;
        x[a] = x[a] + P.dt * vn;
    }
}

template <typename T>
__device__ inline void integrate_one(const DevParams &P, double r, const T Fc[3], const T *Fd, double x[3],
                                     double v[3])
{
    integrate_one_m<T>(P, volume_of(r), mass_of(P, r), Fc, Fd, x, v);
}

// Moisture curve Gamma of the capillary force (Sec. 5.4): zero when dry
// (sr <= 0) and when saturated (sr >= 1), one at sr_peak, a quadratic Bezier
// arc on each side with a level tangent at the peak.
__device__ inline double gamma_of(const DevParams &P, double sr)
{
    if (!(sr > 0.0) || !(sr < 1.0)) return 0.0;
    if (sr <= P.sr_peak) {
        const double u = sr / P.sr_peak;
        return u * (2.0 - u);
    }
    const double u = (sr - P.sr_peak) / (1.0 - P.sr_peak);
    return 1.0 - u * u;
}

// Capillary force of the liquid bridge between granules i and j (Sec. 5.4)
// added to acc: with s = d - (r_i + r_j), the pair's mean radius rb, the
// bridge volume V* = vbridge (4/3) pi rb^3 and rupture distance d_r = V*^(1/3)
// + 0.1 V*^(2/3), for 0 < s < d_r the force on i is -Gamma((sr_i + sr_j) / 2)
// F^st (x_i - x_j) / d with F^st = -2 pi sigma rb ((1 + 2 V* / (pi rb s^2))^(-1/2)
// - 1) > 0: an attraction.  dx = x_i - x_j, d2 = |dx|^2.  Double arithmetic
// (s is a small difference of nearly equal lengths); returns 1 if bridged.
template <typename T>
__device__ inline int capillary_pair(const DevParams &P, const double dx[3], double d2, double ri, double rj, T sri,
                                     T srj, T acc[3])
{
#pragma clang fp contract(off)
    const double d = sqrt(d2);
    const double s = d - (ri + rj);
    const double rb = 0.5 * (ri + rj);
    const double V = P.vbridge * volume_of(rb);
    const double t = cbrt(V);
    const double dr = t + 0.1 * (t * t);
    if (!(s > 0.0) || !(s < dr)) return 0;
    const double g = gamma_of(P, 0.5 * ((double)sri + (double)srj));
    const double q = 1.0 + (2.0 * V) / ((GIC_PI * rb) * (s * s));
    const double fst = -(2.0 * GIC_PI * P.sigma * rb) * (1.0 / sqrt(q) - 1.0);
    const double f = -(g * fst);
    for (int a = 0; a < 3; ++a) acc[a] += (T)(f * (dx[a] / d));
    return 1;
}

// Origin of a brick's node tile: one node below the brick's first node per
// axis.  The tile (P.tile nodes per edge) holds the stencils of all granules
// whose cell lies in the brick.
__device__ inline void tile_origin(const DevParams &P, int64_t b, int32_t o[3])
{
    const int64_t bc[3] = {b % P.nb[0], (b / P.nb[0]) % P.nb[1], b / ((int64_t)P.nb[0] * P.nb[1])};
    // the brick's lower face in node units; the tolerance keeps a face that
    // lies on a node boundary from rounding to the node below
    for (int a = 0; a < 3; ++a) o[a] = (int32_t)floor((double)(bc[a] * kBrick) * P.cell * P.inv_dx + 1e-7) - 1;
}

// Bit pattern of v + 1.5 * 2^52, i.e. rint(v) plus kRintBias, for |v| < 2^51.
// Sums of such patterns, taken modulo 2^64 and corrected by the count times
// kRintBias, are sums of rint values.
constexpr uint64_t kRintBias = 0x4338000000000000ull;  // bits of 1.5 * 2^52
__device__ inline uint64_t rint_biased(double v)
{
#pragma clang fp contract(off)
    const double M = 6755399441055744.0;
    return (uint64_t)__double_as_longlong(v + M);
}

// Bit pattern of the nearest integer (ties to even) to the exact product
// a b, plus kRintBias, for |a b| < 2^51: a b + 1.5 * 2^52 lies where the
// doubles are the integers, so the one rounding of the fused multiply-add
// rounds a b itself (a fixed-point contribution w S is rounded once).
__device__ inline uint64_t rint_product_biased(double a, double b)
{
    return (uint64_t)__double_as_longlong(__builtin_fma(a, b, 6755399441055744.0));
}

constexpr double kFixLimit = 2251799813685248.0;  // 2^51

// Pair (or wall) force of Eq. (1a)-(1c) with the dashpot reading, in real
// type T.  nh: unit normal from the partner to this granule; delta: overlap;
// w: relative velocity; meff: effective mass.  Returns 1 if capped.
// Square root and quotient of the pair law: correctly rounded in double; in
// float the hardware square root and reciprocal (about 1 ulp), far inside
// the FP32 form's 1e-5 tolerance.
__device__ inline double law_sqrt(double a) { return sqrt(a); }
__device__ inline float law_sqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ inline double law_div(double a, double b) { return a / b; }
__device__ inline float law_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

template <typename T>
__device__ inline int pair_force(const DevParams &P, const T nh[3], T delta, const T w[3], T meff, T F[3])
{
    const T kn = (T)P.kn;
    T gam = (T)2 * (T)P.zeta * law_sqrt(meff * kn);
    T kt = (T)P.kt_ratio * gam;
    T vn = (w[0] * nh[0] + w[1] * nh[1]) + w[2] * nh[2];
    T fn = kn * delta - gam * vn;
    T ft[3];
    for (int a = 0; a < 3; ++a) ft[a] = -kt * (w[a] - vn * nh[a]);
    T fts = law_sqrt((ft[0] * ft[0] + ft[1] * ft[1]) + ft[2] * ft[2]);
    T cap = (T)P.mu * (kn * delta);
    int slide = fts > cap;
    T s = slide ? law_div(cap, fts) : (T)1;
    for (int a = 0; a < 3; ++a) F[a] = fn * nh[a] + ft[a] * s;
    return slide;
}

}  // namespace gic
