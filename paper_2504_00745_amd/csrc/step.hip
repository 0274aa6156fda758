// Fused stages of one sub-step (Alg. 2) on gfx950: the gather into sorted
// order together with G2P (Sec. 5.2) and the drag (Sec. 3.3 Eq. 5b, App. A),
// one workgroup per brick of 4x4x4 cells.  The brick's node tile of fluid
// velocity and clamped solid fraction is copied into LDS once, so each
// granule's 27 node reads come from LDS instead of 4 x 27 global loads.
// Results are bit-identical to the separate reorder, G2P and drag kernels:
// the arithmetic is the same device functions in the same order.
#include "gic_launch.hpp"

namespace gic {

namespace {

// Node tile entry of the drag gather: u and the clamped solid fraction of a
// node, read with one LDS access.
template <typename T>
struct Node4;
template <>
struct Node4<float> {
    using type = float4;
};
template <>
struct Node4<double> {
    using type = double4;
};

// g2p_sample_st for a stencil that lies inside the tile: the same weights,
// products and summation order, the node read from the tile at
// lz[cz] + ly[cy] + lx[cx].
template <typename T, typename V4>
__device__ inline void g2p_sample_tile(const Stencil &s, const V4 *__restrict__ tile, const int lx[3],
                                       const int ly[3], const int lz[3], T uat[3], T &af)
{
    T acc[3] = {(T)0, (T)0, (T)0};
    T as = (T)0;
#pragma unroll
    for (int cz = 0; cz < 3; ++cz) {
        const double wz = s.w[2][cz];
#pragma unroll
        for (int cy = 0; cy < 3; ++cy) {
            const double wyz = s.w[1][cy] * wz;
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) {
                const T w = (T)(s.w[0][cx] * wyz);
                const V4 q = tile[lz[cz] + ly[cy] + lx[cx]];
                acc[0] += w * q.x;
                acc[1] += w * q.y;
                acc[2] += w * q.z;
                as += w * q.w;
            }
        }
    }
    uat[0] = acc[0];
    uat[1] = acc[1];
    uat[2] = acc[2];
    af = (T)1 - as;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gather_g2p_drag(DevParams P, int64_t n, const int32_t *__restrict__ bl,
                                                         const int32_t *__restrict__ bcnt,
                                                         const int32_t *__restrict__ order,
                                                         const double *__restrict__ x, const double *__restrict__ v,
                                                         const double *__restrict__ r, const int32_t *__restrict__ id,
                                                         double *__restrict__ xo, double *__restrict__ vo,
                                                         double *__restrict__ ro, int32_t *__restrict__ ido,
                                                         const T *__restrict__ u, const int64_t *__restrict__ afx,
                                                         const int32_t *__restrict__ cb, const int32_t *__restrict__ ce,
                                                         T *__restrict__ Fd, T *__restrict__ uat, T *__restrict__ af)
{
    using V4 = typename Node4<T>::type;
    extern __shared__ double smem_d[];
    const int64_t b = brick_of_block(bl, bcnt);
    if (b < 0) return;
    int32_t gb = cb[b * kBrickCells], ge = ce[b * kBrickCells + kBrickCells - 1];
    clip_range(n, gb, ge);
    if (ge <= gb) return;
    const int E = P.tile, E3 = E * E * E;
    V4 *su = reinterpret_cast<V4 *>(smem_d);  // [E3]: u_x, u_y, u_z, clamped alpha
    int32_t o[3];
    tile_origin(P, b, o);
    const int64_t G = P.G;
    // the first granule's state is fetched before the tile, so the two
    // loads' latencies overlap
    int64_t s = -1;
    double xa[3] = {0.0, 0.0, 0.0}, va[3] = {0.0, 0.0, 0.0}, rq = 0.0;
    int32_t idq = 0;
    auto fetch = [&](int64_t q) {
        s = order[q];
        if ((uint64_t)s >= (uint64_t)n) return;
        for (int a = 0; a < 3; ++a) {
            xa[a] = x[a * n + s];
            va[a] = v[a * n + s];
        }
        rq = r[s];
        if (ido) idq = id[s];
    };
    const int64_t q0 = gb + threadIdx.x;
    if (q0 < ge) fetch(q0);
    for (int k = threadIdx.x; k < E3; k += 256) {
        const int32_t i = o[0] + k % E, j = o[1] + (k / E) % E, l = o[2] + k / (E * E);
        if (i < 0 || j < 0 || l < 0 || i >= P.n[0] || j >= P.n[1] || l >= P.n[2]) continue;  // never referenced
        const int64_t idx = node_index(P, i, j, l);
        V4 q;
        q.x = u[idx];
        q.y = u[G + idx];
        q.z = u[2 * G + idx];
        q.w = (T)node_alpha(P, afx[idx]);
        su[k] = q;
    }
    __syncthreads();
    for (int64_t q = q0; q < ge; q += 256) {
        if (q != q0) fetch(q);
        if ((uint64_t)s >= (uint64_t)n) continue;  // not a permutation of [0, n): position q left untouched
        for (int a = 0; a < 3; ++a) {
            xo[a * n + q] = xa[a];
            vo[a * n + q] = va[a];
        }
        ro[q] = rq;
        if (ido) ido[q] = idq;
        Stencil st;
        stencil_of(P, xa, st);
        // tile offsets of the stencil's nodes; every node inside the tile is
        // the rule (a granule outside its brick's tile only if its cell is
        // clamped)
        int lx[3], ly[3], lz[3];
        bool inside = true;
        for (int k = 0; k < 3; ++k) {
            const int ax = st.node[0][k] - o[0], ay = st.node[1][k] - o[1], az = st.node[2][k] - o[2];
            inside &= ax >= 0 && ay >= 0 && az >= 0 && ax < E && ay < E && az < E;
            lx[k] = ax;
            ly[k] = ay * E;
            lz[k] = az * E * E;
        }
        T ua[3], a;
        if (inside) {
            g2p_sample_tile<T>(st, su, lx, ly, lz, ua, a);
        } else {
            g2p_sample_st<T>(st, [&](int32_t i, int32_t j, int32_t k, T uu[3], T &al) {
                const int32_t li = i - o[0], lj = j - o[1], lk = k - o[2];
                if (li >= 0 && lj >= 0 && lk >= 0 && li < E && lj < E && lk < E) {
                    const V4 t = su[(lk * E + lj) * E + li];
                    uu[0] = t.x;
                    uu[1] = t.y;
                    uu[2] = t.z;
                    al = t.w;
                } else {
                    const int64_t idx = node_index(P, i, j, k);
                    uu[0] = u[idx];
                    uu[1] = u[G + idx];
                    uu[2] = u[2 * G + idx];
                    al = (T)node_alpha(P, afx[idx]);
                }
            }, ua, a);
        }
        T f[3];
        drag_one<T>(P, rq, va, ua, a, f);
        for (int c = 0; c < 3; ++c) Fd[c * n + q] = f[c];
        if (uat) {
            uat[q] = ua[0];
            uat[n + q] = ua[1];
            uat[2 * n + q] = ua[2];
        }
        if (af) af[q] = a;
    }
}

// The same gather and G2P with the remaining interphase forces (Sec. 3.3
// Eq. 5a-5c): the node tile also holds grad p (gp) and the fluid
// acceleration (fa) when given, and each granule's fluid force is the drag
// of the drag model, plus -V grad p at the granule, plus (rho_f V / 2) a_f
// under virtual mass (the a_s part of the virtual-mass force sits in the
// effective mass of the integrator).  Both extra terms are V times the
// interpolation of one node field, e = -grad p + (rho_f / 2) a_f, so the
// tile holds e (three channels) instead of grad p and a_f (six).  The
// interpolation of u and alpha is the same function as in the drag-only
// kernel; e is sampled in the same pass over the 27 nodes with the same
// weights.  For wet granules (held given, in the input order)
// V = (4/3) pi r^3 (1 + held): the absorbed water counts as volume
// (Sec. 5.3); held is gathered into heldo with the rest of the state.
template <typename T>
__global__ void __launch_bounds__(256) k_gather_g2p_fluid(DevParams P, int64_t n, const int32_t *__restrict__ bl,
                                                          const int32_t *__restrict__ bcnt,
                                                          const int32_t *__restrict__ order,
                                                          const double *__restrict__ x, const double *__restrict__ v,
                                                          const double *__restrict__ r,
                                                          const int32_t *__restrict__ id, double *__restrict__ xo,
                                                          double *__restrict__ vo, double *__restrict__ ro,
                                                          int32_t *__restrict__ ido, const T *__restrict__ u,
                                                          const int64_t *__restrict__ afx, const T *__restrict__ gp,
                                                          const T *__restrict__ fa, const int32_t *__restrict__ cb,
                                                          const int32_t *__restrict__ ce, T *__restrict__ Ff,
                                                          const double *__restrict__ held,
                                                          double *__restrict__ heldo)
{
    extern __shared__ double smem_d[];
    const int64_t b = brick_of_block(bl, bcnt);
    if (b < 0) return;
    int32_t gb = cb[b * kBrickCells], ge = ce[b * kBrickCells + kBrickCells - 1];
    clip_range(n, gb, ge);
    if (ge <= gb) return;
    const bool vm_acc = P.vmass && fa != nullptr;
    const T half_rho_f = (T)P.half_rho_f;
    // e = -grad p + (rho_f / 2) a_f at grid node idx, component c
    auto extra_field = [&](int c, int64_t idx) {
        T e = gp ? -gp[c * P.G + idx] : (T)0;
        if (vm_acc) e = e + half_rho_f * fa[c * P.G + idx];
        return e;
    };
    const int E = P.tile, E3 = E * E * E;
    T *su = reinterpret_cast<T *>(smem_d);  // [7][E3]: u_x, u_y, u_z, clamped alpha, e (3)
    int32_t o[3];
    tile_origin(P, b, o);
    const int64_t G = P.G;
    for (int k = threadIdx.x; k < E3; k += 256) {
        const int32_t i = o[0] + k % E, j = o[1] + (k / E) % E, l = o[2] + k / (E * E);
        if (i < 0 || j < 0 || l < 0 || i >= P.n[0] || j >= P.n[1] || l >= P.n[2]) continue;  // never referenced
        const int64_t idx = node_index(P, i, j, l);
        for (int c = 0; c < 3; ++c) su[c * E3 + k] = u[c * G + idx];
        su[3 * E3 + k] = (T)node_alpha(P, afx[idx]);
        for (int c = 0; c < 3; ++c) su[(4 + c) * E3 + k] = extra_field(c, idx);
    }
    __syncthreads();
    // node (i, j, k) as a tile slot, or -1 outside the tile (a granule whose
    // cell is clamped; its values then come from the grid)
    auto slot = [&](int32_t i, int32_t j, int32_t k) {
        const int32_t li = i - o[0], lj = j - o[1], lk = k - o[2];
        return (li >= 0 && lj >= 0 && lk >= 0 && li < E && lj < E && lk < E) ? (lk * E + lj) * E + li : -1;
    };
    for (int64_t q = gb + threadIdx.x; q < ge; q += 256) {
        const int64_t s = order[q];
        if ((uint64_t)s >= (uint64_t)n) continue;  // not a permutation of [0, n): position q left untouched
        const double xa[3] = {x[s], x[n + s], x[2 * n + s]};
        const double va[3] = {v[s], v[n + s], v[2 * n + s]};
        const double rq = r[s];
        for (int a = 0; a < 3; ++a) {
            xo[a * n + q] = xa[a];
            vo[a * n + q] = va[a];
        }
        ro[q] = rq;
        if (ido) ido[q] = id[s];
        const double hq = held ? held[s] : 0.0;
        if (heldo) heldo[q] = hq;
        Stencil st;
        stencil_of(P, xa, st);
        T ua[3], a;
        T ea[3] = {(T)0, (T)0, (T)0};
        int t = -1;          // tile slot of the node just fetched, -1 outside the tile
        int64_t gidx = 0;    // its grid index when outside
        const bool extra = gp || vm_acc;
        g2p_sample_st<T>(st, [&](int32_t i, int32_t j, int32_t k, T uu[3], T &al) {
            t = slot(i, j, k);
            if (t >= 0) {
                uu[0] = su[t];
                uu[1] = su[E3 + t];
                uu[2] = su[2 * E3 + t];
                al = su[3 * E3 + t];
            } else {
                gidx = node_index(P, i, j, k);
                uu[0] = u[gidx];
                uu[1] = u[G + gidx];
                uu[2] = u[2 * G + gidx];
                al = (T)node_alpha(P, afx[gidx]);
            }
        }, ua, a, [&](T w) {
            if (!extra) return;
            for (int c = 0; c < 3; ++c) ea[c] += w * (t >= 0 ? su[(4 + c) * E3 + t] : extra_field(c, gidx));
        });
        T f[3];
        drag_one<T>(P, rq, va, ua, a, f);
        if (extra) {
            const T tV = (T)wet_volume(rq, hq);
            for (int c = 0; c < 3; ++c) f[c] = f[c] + tV * ea[c];
        }
        for (int c = 0; c < 3; ++c) Ff[c * n + q] = f[c];
    }
}

}  // namespace

template <typename T>
hipError_t launch_gather_g2p_fluid(const DevParams &P, int64_t n, int64_t K, const int32_t *order, const double *x,
                                   const double *v, const double *r, const int32_t *id, double *xo, double *vo,
                                   double *ro, int32_t *ido, const T *u, const int64_t *afx, const T *gp,
                                   const T *fa, const int32_t *cb, const int32_t *ce, const BrickList &B, T *Ff,
                                   hipStream_t s, const double *held, double *heldo)
{
    if (n == 0) return hipSuccess;
    const int64_t bricks = K / kBrickCells;
    const int E = P.tile;
    const size_t lds = sizeof(T) * 7 * (size_t)E * E * E;
    k_gather_g2p_fluid<T><<<brick_grid(bricks), 256, lds, s>>>(P, n, B.list, B.count, order, x, v, r, id, xo, vo, ro,
                                                               ido, u, afx, gp, fa, cb, ce, Ff, held, heldo);
    return hipGetLastError();
}

template hipError_t launch_gather_g2p_fluid<float>(const DevParams &, int64_t, int64_t, const int32_t *,
                                                   const double *, const double *, const double *, const int32_t *,
                                                   double *, double *, double *, int32_t *, const float *,
                                                   const int64_t *, const float *, const float *, const int32_t *,
                                                   const int32_t *, const BrickList &, float *, hipStream_t,
                                                   const double *, double *);
template hipError_t launch_gather_g2p_fluid<double>(const DevParams &, int64_t, int64_t, const int32_t *,
                                                    const double *, const double *, const double *, const int32_t *,
                                                    double *, double *, double *, int32_t *, const double *,
                                                    const int64_t *, const double *, const double *, const int32_t *,
                                                    const int32_t *, const BrickList &, double *, hipStream_t,
                                                    const double *, double *);

template <typename T>
hipError_t launch_gather_g2p_drag(const DevParams &P, int64_t n, int64_t K, const int32_t *order, const double *x,
                                  const double *v, const double *r, const int32_t *id, double *xo, double *vo,
                                  double *ro, int32_t *ido, const T *u, const int64_t *afx, const int32_t *cb,
                                  const int32_t *ce, const BrickList &B, T *Fd, T *uat, T *af, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t bricks = K / kBrickCells;
    const int E = P.tile;
    const size_t lds = sizeof(typename Node4<T>::type) * (size_t)E * E * E;
    k_gather_g2p_drag<T><<<brick_grid(bricks), 256, lds, s>>>(P, n, B.list, B.count, order, x, v, r, id, xo, vo, ro,
                                                              ido, u, afx, cb, ce, Fd, uat, af);
    return hipGetLastError();
}

template hipError_t launch_gather_g2p_drag<float>(const DevParams &, int64_t, int64_t, const int32_t *,
                                                  const double *, const double *, const double *, const int32_t *,
                                                  double *, double *, double *, int32_t *, const float *,
                                                  const int64_t *, const int32_t *, const int32_t *,
                                                  const BrickList &, float *, float *, float *, hipStream_t);
template hipError_t launch_gather_g2p_drag<double>(const DevParams &, int64_t, int64_t, const int32_t *,
                                                   const double *, const double *, const double *, const int32_t *,
                                                   double *, double *, double *, int32_t *, const double *,
                                                   const int64_t *, const int32_t *, const int32_t *,
                                                   const BrickList &, double *, double *, double *, hipStream_t);

}  // namespace gic
