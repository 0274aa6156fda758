// a2 + a3: neighbour candidates and contact forces (Sec. 3.1, Eq. 1a-c) on
// gfx950.
//
// One thread per granule in sorted order.  Each granule visits only the
// neighbour cells its search box [x - (r_i + r_max), x + (r_i + r_max)]
// overlaps (at most 27, typically 8 when the cell is twice the largest
// diameter); candidates of a cell are contiguous in sorted order, so a wave's
// candidate loads fall in a few cache lines.  The contact test, the overlap
// and the normal are double in both forms (the overlap is a small difference
// of nearly equal distances); the pair law and the per-granule sum run in T.
#include "gic_launch.hpp"

namespace gic {

namespace {

// Cell range to visit along one axis: the cells overlapped by the search box,
// clipped to the 3 cells around the granule's own cell.
__device__ inline void search_range(const DevParams &P, double xa, double R, int32_t nc, int32_t &lo,
                                    int32_t &hi)
{
    int32_t c = cell_coord(xa, P.inv_cell, nc);
    int32_t l = cell_coord(xa - R, P.inv_cell, nc);
    int32_t h = cell_coord(xa + R, P.inv_cell, nc);
    lo = l > c - 1 ? l : c - 1;
    hi = h < c + 1 ? h : c + 1;
}

// Contact test of Sec. 3.1 with the reading 2r -> r_i + r_j: strict, on
// squared distances, one rounding per operation.
__device__ inline bool touching(double dx0, double dx1, double dx2, double R, double &d2)
{
#pragma clang fp contract(off)
    d2 = (dx0 * dx0 + dx1 * dx1) + dx2 * dx2;
    return d2 < R * R;
}

template <typename T>
__global__ void __launch_bounds__(256) k_contact(DevParams P, int64_t n, const double *__restrict__ x,
                                                 const double *__restrict__ v, const double *__restrict__ r,
                                                 const int32_t *__restrict__ cb, const int32_t *__restrict__ ce,
                                                 T *__restrict__ F, int32_t *__restrict__ ncont, int64_t *err)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double xi[3] = {x[q], x[n + q], x[2 * n + q]};
    const double vi[3] = {v[q], v[n + q], v[2 * n + q]};
    const double ri = r[q];
    if (ri > P.r_max) raise_error(err, kErrRange, q);
    const double mi = mass_of(P, ri);
    const double Rs = (ri + P.r_max) * P.search_scale;
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) search_range(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
    T acc[3] = {(T)0, (T)0, (T)0};
    int32_t cnt = 0;
    for (int32_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int32_t cy = lo[1]; cy <= hi[1]; ++cy)
            for (int32_t cx = lo[0]; cx <= hi[0]; ++cx) {
                const uint32_t key = key_of_cell(P, cx, cy, cz);
                const int32_t e = ce[key];
                for (int32_t j = cb[key]; j < e; ++j) {
                    if (j == q) continue;
                    const double d0 = xi[0] - x[j], d1 = xi[1] - x[n + j], d2c = xi[2] - x[2 * n + j];
                    const double rj = r[j];
                    const double R = ri + rj;
                    double d2;
                    if (!touching(d0, d1, d2c, R, d2) || d2 == 0.0) continue;
                    const double d = sqrt(d2);
                    const double inv_d = 1.0 / d;
                    const T nh[3] = {(T)(d0 * inv_d), (T)(d1 * inv_d), (T)(d2c * inv_d)};
                    const T delta = (T)(R - d);
                    const T w[3] = {(T)(vi[0] - v[j]), (T)(vi[1] - v[n + j]), (T)(vi[2] - v[2 * n + j])};
                    const double mj = mass_of(P, rj);
                    const T meff = (T)((mi * mj) / (mi + mj));
                    T Fp[3];
                    pair_force<T>(P, nh, delta, w, meff, Fp);
                    acc[0] += Fp[0];
                    acc[1] += Fp[1];
                    acc[2] += Fp[2];
                    ++cnt;
                }
            }
    if (P.walls) {
        const T wv[3] = {(T)vi[0], (T)vi[1], (T)vi[2]};
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side) {
                if (!(P.walls & (1u << (2 * a + side)))) continue;
                const double dist = side == 0 ? xi[a] : P.L[a] - xi[a];
                const double delta = ri - dist;
                if (!(delta > 0.0)) continue;
                T nh[3] = {(T)0, (T)0, (T)0};
                nh[a] = side == 0 ? (T)1 : (T)-1;
                T Fp[3];
                pair_force<T>(P, nh, (T)delta, wv, (T)mi, Fp);
                acc[0] += Fp[0];
                acc[1] += Fp[1];
                acc[2] += Fp[2];
                ++cnt;
            }
    }
    F[q] = acc[0];
    F[n + q] = acc[1];
    F[2 * n + q] = acc[2];
    if (ncont) ncont[q] = cnt;
}

__global__ void __launch_bounds__(256) k_contact_pairs(DevParams P, int64_t n, const double *__restrict__ x,
                                                       const double *__restrict__ r,
                                                       const int32_t *__restrict__ cb,
                                                       const int32_t *__restrict__ ce, int32_t *pairs, int64_t cap,
                                                       unsigned long long *count)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double xi[3] = {x[q], x[n + q], x[2 * n + q]};
    const double ri = r[q];
    const double Rs = (ri + P.r_max) * P.search_scale;
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) search_range(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
    for (int32_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int32_t cy = lo[1]; cy <= hi[1]; ++cy)
            for (int32_t cx = lo[0]; cx <= hi[0]; ++cx) {
                const uint32_t key = key_of_cell(P, cx, cy, cz);
                const int32_t e = ce[key];
                for (int32_t j = cb[key]; j < e; ++j) {
                    if (j <= q) continue;
                    double d2;
                    if (!touching(xi[0] - x[j], xi[1] - x[n + j], xi[2] - x[2 * n + j], ri + r[j], d2)) continue;
                    unsigned long long k = atomicAdd(count, 1ull);
                    if ((int64_t)k < cap) {
                        pairs[2 * k] = (int32_t)q;
                        pairs[2 * k + 1] = j;
                    }
                }
            }
}

__global__ void k_zero_count(unsigned long long *c) { *c = 0ull; }

}  // namespace

template <typename T>
hipError_t launch_contact(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                          const int32_t *cb, const int32_t *ce, T *F, int32_t *ncont, int64_t *err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_contact<T><<<grid_for(n, 256), 256, 0, s>>>(P, n, x, v, r, cb, ce, F, ncont, err);
    return hipGetLastError();
}

template hipError_t launch_contact<float>(const DevParams &, int64_t, const double *, const double *,
                                          const double *, const int32_t *, const int32_t *, float *, int32_t *,
                                          int64_t *, hipStream_t);
template hipError_t launch_contact<double>(const DevParams &, int64_t, const double *, const double *,
                                           const double *, const int32_t *, const int32_t *, double *, int32_t *,
                                           int64_t *, hipStream_t);

hipError_t launch_contact_pairs(const DevParams &P, int64_t n, const double *x, const double *r,
                                const int32_t *cb, const int32_t *ce, int32_t *pairs, int64_t cap,
                                int64_t *count, hipStream_t s)
{
    unsigned long long *c = reinterpret_cast<unsigned long long *>(count);
    k_zero_count<<<1, 1, 0, s>>>(c);
    if (n > 0) k_contact_pairs<<<grid_for(n, 256), 256, 0, s>>>(P, n, x, r, cb, ce, pairs, cap, c);
    return hipGetLastError();
}

}  // namespace gic
