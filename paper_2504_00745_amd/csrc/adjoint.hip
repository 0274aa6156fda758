// a9: adjoint (vector-Jacobian products) of the granule step on gfx950, in
// double.  Forward definitions (Sec. 3.1 Eq. 1a-c; Sec. 3.3 Eq. 5b with the
// App. A relaxation drag; Sec. 5.1 Eq. 7a; Sec. 5.2 G2P; Sec. 4 symplectic
// Euler), unquantised transfers:
//   A = P2G_alpha(x);  (u_at, alpha_f) = G2P(x; u, A);
//   F_d = C_d 6 pi eta r alpha_f (u_at - v);  F_c = contact(x, v; mu);
//   v' = v + dt ((F_c + F_d)/m + g);  x' = x + dt v'.
// Every kernel reads its forward inputs and recomputes what it needs; the
// contact pullback is a gather (granule i collects, for each touching
// partner j, the pair term with cotangent g_i - g_j), so no atomics are used
// except in the grid scatter of the G2P pullback, which sums integers
// (contributions rounded at the scale of the largest one; transfer.hip), so
// every result is the same bits in every run.
#include "gic_launch.hpp"

namespace gic {

namespace {

constexpr int kAdjPartners = 16;

// Reverse of pair_force in double.  gbar: cotangent of the force on the
// first partner; gmu: cotangent used for the derivative in mu.  Adds to
// nbar, *dbar (overlap), wbar (relative velocity), *mubar.
__device__ inline void pair_force_vjp(const DevParams &P, const double nh[3], double delta, const double w[3],
                                      double meff, const double gbar[3], const double gmu[3], double nbar[3],
                                      double &dbar, double wbar[3], double &mubar)
{
    const double gam = 2.0 * P.zeta * sqrt(meff * P.kn);
    const double kt = P.kt_ratio * gam;
    const double vn = (w[0] * nh[0] + w[1] * nh[1]) + w[2] * nh[2];
    const double fn = P.kn * delta - gam * vn;
    double ft[3];
    for (int a = 0; a < 3; ++a) ft[a] = -kt * (w[a] - vn * nh[a]);
    const double s = sqrt((ft[0] * ft[0] + ft[1] * ft[1]) + ft[2] * ft[2]);
    const double cap = P.mu * (P.kn * delta);
    const bool slide = s > cap;
    const double fnbar = (gbar[0] * nh[0] + gbar[1] * nh[1]) + gbar[2] * nh[2];
    for (int a = 0; a < 3; ++a) nbar[a] += fn * gbar[a];
    double ftbar[3];
    if (slide) {
        const double fh[3] = {ft[0] / s, ft[1] / s, ft[2] / s};
        const double gdotf = (gbar[0] * fh[0] + gbar[1] * fh[1]) + gbar[2] * fh[2];
        for (int a = 0; a < 3; ++a) ftbar[a] = (cap / s) * (gbar[a] - gdotf * fh[a]);
        dbar += gdotf * P.mu * P.kn;
        const double gmudotf = (gmu[0] * fh[0] + gmu[1] * fh[1]) + gmu[2] * fh[2];
        mubar += gmudotf * P.kn * delta;
    } else {
        for (int a = 0; a < 3; ++a) ftbar[a] = gbar[a];
    }
    double tbar[3];
    for (int a = 0; a < 3; ++a) tbar[a] = -kt * ftbar[a];
    double vnbar = -((tbar[0] * nh[0] + tbar[1] * nh[1]) + tbar[2] * nh[2]);
    for (int a = 0; a < 3; ++a) {
        wbar[a] += tbar[a];
        nbar[a] += -vn * tbar[a];
    }
    dbar += P.kn * fnbar;
    vnbar += -gam * fnbar;
    for (int a = 0; a < 3; ++a) {
        wbar[a] += vnbar * nh[a];
        nbar[a] += vnbar * w[a];
    }
}

__device__ inline void search_range_adj(const DevParams &P, double xa, double R, int32_t nc, int32_t &lo,
                                        int32_t &hi)
{
    int32_t c = cell_coord(xa, P.inv_cell, nc);
    int32_t l = cell_coord(xa - R, P.inv_cell, nc);
    int32_t h = cell_coord(xa + R, P.inv_cell, nc);
    lo = l > c - 1 ? l : c - 1;
    hi = h < c + 1 ? h : c + 1;
}

__device__ inline bool touching_adj(double d0, double d1, double d2c, double R, double &d2)
{
#pragma clang fp contract(off)
    d2 = (d0 * d0 + d1 * d1) + d2c * d2c;
    return d2 < R * R;
}

__global__ void __launch_bounds__(256) k_contact_vjp(DevParams P, int64_t n, const double *__restrict__ x,
                                                     const double *__restrict__ v, const double *__restrict__ r,
                                                     const int32_t *__restrict__ cb, const int32_t *__restrict__ ce,
                                                     const double *__restrict__ gF, double *__restrict__ gx,
                                                     double *__restrict__ gv, double *__restrict__ gmu)
{
    __shared__ int32_t plist[kAdjPartners * 256];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int tid = threadIdx.x;
    const double xi[3] = {x[q], x[n + q], x[2 * n + q]};
    const double vi[3] = {v[q], v[n + q], v[2 * n + q]};
    const double gi[3] = {gF[q], gF[n + q], gF[2 * n + q]};
    const double ri = r[q];
    const double mi = mass_of(P, ri);
    const double Rs = (ri + P.r_max) * P.search_scale;
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) search_range_adj(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
    double gxi[3] = {0, 0, 0}, gvi[3] = {0, 0, 0}, mu_acc = 0.0;
    auto pair = [&](int32_t j) {
        const double d0 = xi[0] - x[j], d1 = xi[1] - x[n + j], d2c = xi[2] - x[2 * n + j];
        const double rj = r[j];
        double d2;
        touching_adj(d0, d1, d2c, ri + rj, d2);
        const double d = sqrt(d2);
        const double nh[3] = {d0 / d, d1 / d, d2c / d};
        const double delta = (ri + rj) - d;
        const double w[3] = {vi[0] - v[j], vi[1] - v[n + j], vi[2] - v[2 * n + j]};
        const double mj = mass_of(P, rj);
        const double meff = (mi * mj) / (mi + mj);
        const double gbar[3] = {gi[0] - gF[j], gi[1] - gF[n + j], gi[2] - gF[2 * n + j]};
        double nbar[3] = {0, 0, 0}, wbar[3] = {0, 0, 0}, dbar = 0.0, mubar = 0.0;
        pair_force_vjp(P, nh, delta, w, meff, gbar, gi, nbar, dbar, wbar, mubar);
        const double nn = (nbar[0] * nh[0] + nbar[1] * nh[1]) + nbar[2] * nh[2];
        for (int a = 0; a < 3; ++a) {
            gxi[a] += (nbar[a] - nn * nh[a]) / d - dbar * nh[a];
            gvi[a] += wbar[a];
        }
        mu_acc += mubar;
    };
    int32_t cnt = 0;
    for (int32_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int32_t cy = lo[1]; cy <= hi[1]; ++cy) {
            int32_t cx = lo[0];
            while (cx <= hi[0]) {
                const int32_t brick_end = (cx & ~(kBrick - 1)) + (kBrick - 1);
                const int32_t cend = hi[0] < brick_end ? hi[0] : brick_end;
                const uint32_t k0 = key_of_cell(P, cx, cy, cz);
                int32_t jb = cb[k0], je = ce[k0 + (uint32_t)(cend - cx)];
                clip_range(n, jb, je);
                for (int32_t j = jb; j < je; ++j) {
                    double d2;
                    if (!touching_adj(xi[0] - x[j], xi[1] - x[n + j], xi[2] - x[2 * n + j], ri + r[j], d2) ||
                        d2 == 0.0)
                        continue;
                    if (cnt < kAdjPartners)
                        plist[cnt * 256 + tid] = j;
                    else
                        pair(j);
                    ++cnt;
                }
                cx = cend + 1;
            }
        }
    const int listed = cnt < kAdjPartners ? cnt : kAdjPartners;
    for (int k = 0; k < listed; ++k) pair(plist[k * 256 + tid]);
    if (P.walls)
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side) {
                if (!(P.walls & (1u << (2 * a + side)))) continue;
                const double dist = side == 0 ? xi[a] : P.L[a] - xi[a];
                const double delta = ri - dist;
                if (!(delta > 0.0)) continue;
                double nh[3] = {0.0, 0.0, 0.0};
                nh[a] = side == 0 ? 1.0 : -1.0;
                double nbar[3] = {0, 0, 0}, wbar[3] = {0, 0, 0}, dbar = 0.0, mubar = 0.0;
                pair_force_vjp(P, nh, delta, vi, mi, gi, gi, nbar, dbar, wbar, mubar);
                gxi[a] += side == 0 ? -dbar : dbar;
                for (int b = 0; b < 3; ++b) gvi[b] += wbar[b];
                mu_acc += mubar;
            }
    for (int a = 0; a < 3; ++a) {
        gx[a * n + q] += gxi[a];
        gv[a * n + q] += gvi[a];
    }
    gmu[q] = mu_acc;
}

__global__ void __launch_bounds__(256) k_drag_vjp(DevParams P, int64_t n, const double *__restrict__ r,
                                                  const double *__restrict__ v, const double *__restrict__ uat,
                                                  const double *__restrict__ af, const double *__restrict__ gF,
                                                  double *__restrict__ gv, double *__restrict__ guat,
                                                  double *__restrict__ gaf, double *__restrict__ gcd)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double c = P.cdrag_unit * r[q];   // 6 pi eta r
    const double beta = P.c_drag * c;
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double g = gF[a * n + q];
        gv[a * n + q] += -beta * af[q] * g;
        guat[a * n + q] = beta * af[q] * g;
        s += (uat[a * n + q] - v[a * n + q]) * g;
    }
    gaf[q] = beta * s;
    gcd[q] = c * af[q] * s;
}

// dL/dx^{n+1} = gx, dL/dv^{n+1} = gv on entry.  v^{n+1} feeds x^{n+1}, so
// its total adjoint is gv + dt gx (written back to gv: this is also the
// adjoint of v^n through the identity term); gF = dt/m of it.
__global__ void __launch_bounds__(256) k_integrate_vjp(DevParams P, int64_t n, const double *__restrict__ r,
                                                       const double *__restrict__ gx, double *__restrict__ gv,
                                                       double *__restrict__ gF)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double s = P.dt / mass_of(P, r[q]);
    for (int a = 0; a < 3; ++a) {
        const double t = gv[a * n + q] + P.dt * gx[a * n + q];
        gv[a * n + q] = t;
        gF[a * n + q] = s * t;
    }
}

// Granule part of the G2P pullback: gx += sum_k grad w_k (u_k . guat -
// min(A_k, alpha_max) gaf).
__global__ void __launch_bounds__(256) k_g2p_vjp_x(DevParams P, int64_t n, const double *__restrict__ x,
                                                   const double *__restrict__ u, const double *__restrict__ A,
                                                   const double *__restrict__ guat, const double *__restrict__ gaf,
                                                   double *__restrict__ gx)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double xa[3] = {x[q], x[n + q], x[2 * n + q]};
    Stencil s;
    stencil_of(P, xa, s);
    double dw[3][3];
    stencil_dw(P, xa, dw);
    const int64_t G = P.G;
    const double gu[3] = {guat[q], guat[n + q], guat[2 * n + q]};
    const double ga = gaf[q];
    double acc[3] = {0, 0, 0};
    for (int cz = 0; cz < 3; ++cz)
        for (int cy = 0; cy < 3; ++cy)
            for (int cx = 0; cx < 3; ++cx) {
                const int64_t k = node_index(P, s.node[0][cx], s.node[1][cy], s.node[2][cz]);
                const double ul = (u[k] * gu[0] + u[G + k] * gu[1]) + u[2 * G + k] * gu[2];
                const double al = A[k] < P.alpha_max ? A[k] : P.alpha_max;
                const double coef = ul - al * ga;
                acc[0] += (dw[0][cx] * s.w[1][cy]) * s.w[2][cz] * coef;
                acc[1] += (s.w[0][cx] * dw[1][cy]) * s.w[2][cz] * coef;
                acc[2] += (s.w[0][cx] * s.w[1][cy]) * dw[2][cz] * coef;
            }
    for (int a = 0; a < 3; ++a) gx[a * n + q] += acc[a];
}

// P2G pullback (gather): gx += frac sum_k gA_k grad w_k + m sum_k (gP_k . v)
// grad w_k;  gv += m sum_k w_k gP_k.
__global__ void __launch_bounds__(256) k_p2g_vjp(DevParams P, int64_t n, const double *__restrict__ x,
                                                 const double *__restrict__ v, const double *__restrict__ r,
                                                 const double *__restrict__ gA, const double *__restrict__ gP,
                                                 double *__restrict__ gx, double *__restrict__ gv)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double xa[3] = {x[q], x[n + q], x[2 * n + q]};
    Stencil s;
    stencil_of(P, xa, s);
    double dw[3][3];
    stencil_dw(P, xa, dw);
    const int64_t G = P.G;
    const double frac = volume_of(r[q]) * P.inv_vcell;
    const double m = mass_of(P, r[q]);
    const double vq[3] = {v[q], v[n + q], v[2 * n + q]};
    double ax[3] = {0, 0, 0}, av[3] = {0, 0, 0};
    for (int cz = 0; cz < 3; ++cz)
        for (int cy = 0; cy < 3; ++cy)
            for (int cx = 0; cx < 3; ++cx) {
                const int64_t k = node_index(P, s.node[0][cx], s.node[1][cy], s.node[2][cz]);
                const double w = (s.w[0][cx] * s.w[1][cy]) * s.w[2][cz];
                double coef = 0.0;
                if (gA) coef += gA[k] * frac;
                if (gP) {
                    const double g3[3] = {gP[k], gP[G + k], gP[2 * G + k]};
                    coef += m * ((g3[0] * vq[0] + g3[1] * vq[1]) + g3[2] * vq[2]);
                    for (int a = 0; a < 3; ++a) av[a] += m * w * g3[a];
                }
                ax[0] += (dw[0][cx] * s.w[1][cy]) * s.w[2][cz] * coef;
                ax[1] += (s.w[0][cx] * dw[1][cy]) * s.w[2][cz] * coef;
                ax[2] += (s.w[0][cx] * s.w[1][cy]) * dw[2][cz] * coef;
            }
    for (int a = 0; a < 3; ++a) {
        gx[a * n + q] += ax[a];
        gv[a * n + q] += av[a];
    }
}

// Deterministic sum: fixed per-workgroup partial sums (wave shuffles, then
// LDS), then one workgroup adds the partials in index order.
__global__ void __launch_bounds__(256) k_partial_sums(const double *__restrict__ a, const double *__restrict__ b,
                                                      int64_t n, int64_t per, double *__restrict__ part)
{
    __shared__ double w[4];
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += b ? a[i] * b[i] : a[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((w[0] + w[1]) + w[2]) + w[3];
}

__global__ void __launch_bounds__(256) k_final_sum(const double *__restrict__ part, int nb, double *out, int acc)
{
    __shared__ double w[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = ((w[0] + w[1]) + w[2]) + w[3];
        *out = acc ? *out + t : t;
    }
}

// out = (factor s[0]) a, s a device scalar (a cotangent that stays on the
// device).
__global__ void __launch_bounds__(256) k_scale(int64_t n, const double *__restrict__ a, const double *__restrict__ sp,
                                               double factor, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (factor * sp[0]) * a[i];
}

__global__ void __launch_bounds__(256) k_permute(int64_t n, int comps, const int32_t *__restrict__ order,
                                                 const double *__restrict__ in, double *__restrict__ out, int scatter)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t i = order[q];
    if ((uint64_t)i >= (uint64_t)n) return;  // not a permutation of [0, n): left untouched
    for (int c = 0; c < comps; ++c) {
        if (scatter)
            out[c * n + i] = in[c * n + q];
        else
            out[c * n + q] = in[c * n + i];
    }
}

}  // namespace

hipError_t launch_contact_vjp(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                              const int32_t *cb, const int32_t *ce, const double *gF, double *gx, double *gv,
                              double *gmu, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_contact_vjp<<<grid_for(n, 256), 256, 0, s>>>(P, n, x, v, r, cb, ce, gF, gx, gv, gmu);
    return hipGetLastError();
}

hipError_t launch_drag_vjp(const DevParams &P, int64_t n, const double *r, const double *v, const double *uat,
                           const double *af, const double *gF, double *gv, double *guat, double *gaf, double *gcd,
                           hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_drag_vjp<<<grid_for(n, 256), 256, 0, s>>>(P, n, r, v, uat, af, gF, gv, guat, gaf, gcd);
    return hipGetLastError();
}

hipError_t launch_integrate_vjp(const DevParams &P, int64_t n, const double *r, const double *gx, double *gv,
                                double *gF, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_integrate_vjp<<<grid_for(n, 256), 256, 0, s>>>(P, n, r, gx, gv, gF);
    return hipGetLastError();
}

hipError_t launch_g2p_vjp(const DevParams &P, int64_t n, int64_t K, const double *x, const double *u,
                          const double *A, const double *guat, const double *gaf, const int32_t *cb,
                          const int32_t *ce, const BrickList &B, double *gx, double *gA, int64_t *fx, double *part,
                          hipStream_t s)
{
    if (n > 0) k_g2p_vjp_x<<<grid_for(n, 256), 256, 0, s>>>(P, n, x, u, A, guat, gaf, gx);
    if (gA) return launch_g2p_vjp_grid(P, n, K, x, A, gaf, cb, ce, B, gA, fx, part, s);
    return hipGetLastError();
}

hipError_t launch_p2g_vjp(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                          const double *gA, const double *gP, double *gx, double *gv, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_p2g_vjp<<<grid_for(n, 256), 256, 0, s>>>(P, n, x, v, r, gA, gP, gx, gv);
    return hipGetLastError();
}

hipError_t launch_sum(const double *a, const double *b, int64_t n, double *part, int nparts, double *out, int acc,
                      hipStream_t s)
{
    const int64_t per = n > 0 ? (n + nparts - 1) / nparts : 1;
    const int nb = (int)(n > 0 ? (n + per - 1) / per : 0);
    if (nb > 0) k_partial_sums<<<nb, 256, 0, s>>>(a, b, n, per, part);
    k_final_sum<<<1, 256, 0, s>>>(part, nb, out, acc);
    return hipGetLastError();
}

hipError_t launch_scale(int64_t n, const double *a, const double *sp, double factor, double *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_scale<<<grid_for(n, 256), 256, 0, s>>>(n, a, sp, factor, out);
    return hipGetLastError();
}

hipError_t launch_permute(int64_t n, int comps, const int32_t *order, const double *in, double *out, int scatter,
                          hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_permute<<<grid_for(n, 256), 256, 0, s>>>(n, comps, order, in, out, scatter);
    return hipGetLastError();
}

}  // namespace gic
