// f4: density projection of the fluid fraction (Sec. 5.1, Eq. 12b and 13;
// App. B discretisation on the MAC grid) on gfx950.
//
// Cells are the transfer grid's nodes (cell centres, x fastest).  With the
// scaled pressure q = (dt^2 / (rho_0 dx^2)) p_2, every fluid cell satisfies
//     (L q)_c = sum_j beta_cj (q_c - q_j) = alpha'_c (clamp(alpha*_c / alpha'_c, 0.5, 1.5) - 1),
// beta_cj = (alpha'_c + alpha'_j) / 2 over the six face neighbours that are
// not solid (an air neighbour is a Dirichlet neighbour with q_j = 0; a solid
// neighbour or the box boundary closes the face).  Non-fluid cells are
// identity rows with a zero right-hand side, so L is symmetric positive
// definite on the whole grid and the solution is zero off the fluid.
//
// The solve is conjugate gradients preconditioned by one multigrid V-cycle
// per iteration (the default; Jacobi as the alternative).  The iteration's
// kernels are streaming or blocked stencil passes over the cells (HBM
// bound), the coarse levels launch-latency bound.  Dot products are reduced
// without atomics: each block writes one partial per quantity, and every
// block of the consuming kernel sums all partials in the same fixed order,
// so the iteration is deterministic and needs no clearing between launches.
#include "idp_launch.hpp"

namespace gic {

namespace {

constexpr int kIdpThreads = 256;

__device__ inline double block_sum(double v, double *red)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Sum of the nb partials of a quantity, identical in every block.
__device__ inline double sum_partials(const double *__restrict__ part, int nb, double *red)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kIdpThreads) v += part[i];
    return block_sum(v, red);
}

struct Nbr {
    int64_t off;   // index offset of the neighbour
    bool inside;   // within the box
};

// Coordinates of cell c.  Below 2^31 cells the two divisions are a multiply
// by a reciprocal and a shift (the stencil kernels would otherwise spend
// most of their instructions on them); larger grids divide in 64 bits.
__device__ inline void coords(const IdpDims &D, int64_t c, int64_t &i, int64_t &j, int64_t &k)
{
    if (D.G <= 0x80000000ll) {
        const uint32_t cc = (uint32_t)c, nx = (uint32_t)D.nx, ny = (uint32_t)D.ny;
        const uint32_t row = (uint32_t)(((uint64_t)cc * D.mx) >> D.shx);
        i = cc - row * nx;
        const uint32_t kk = (uint32_t)(((uint64_t)row * D.my) >> D.shy);
        j = row - kk * ny;
        k = kk;
    } else {
        const int64_t row = c / D.nx;
        i = c - row * D.nx;
        k = row / D.ny;
        j = row - k * D.ny;
    }
}

// The six face neighbours of cell c = (i, j, k) in the fixed order -x, +x, -y, +y, -z, +z.
__device__ inline void neighbours(const IdpDims &D, int64_t i, int64_t j, int64_t k, Nbr nb[6])
{
    nb[0] = {-1, i > 0};
    nb[1] = {1, i < D.nx - 1};
    nb[2] = {-D.nx, j > 0};
    nb[3] = {D.nx, j < D.ny - 1};
    nb[4] = {-D.sxy, k > 0};
    nb[5] = {D.sxy, k < D.nz - 1};
}

__device__ inline void neighbours(const IdpDims &D, int64_t c, Nbr nb[6])
{
    int64_t i, j, k;
    coords(D, c, i, j, k);
    neighbours(D, i, j, k, nb);
}

// (L v)_c and the diagonal of L at c.
__device__ inline void apply_row(const IdpDims &D, int64_t c, const double *__restrict__ at,
                                 const uint8_t *__restrict__ lab, const double *__restrict__ v, double &Lv,
                                 double &diag)
{
#pragma clang fp contract(off)
    if (lab[c] != kIdpFluid) {
        Lv = v[c];
        diag = 1.0;
        return;
    }
    Nbr nb[6];
    neighbours(D, c, nb);
    const double ac = at[c], vc = v[c];
    double acc = 0.0, dg = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!nb[f].inside) continue;
        const int64_t n = c + nb[f].off;
        const uint8_t ln = lab[n];
        if (ln == kIdpSolid) continue;
        const double beta = (ac + at[n]) * 0.5;
        const double vn = ln == kIdpFluid ? v[n] : 0.0;
        acc += beta * (vc - vn);
        dg += beta;
    }
    Lv = acc;
    diag = dg;
}

// sum over the open faces of cell c = (i, j, k) of beta (v_c - v_n), from
// the signed coefficients ac (alpha_f' on fluid cells, -alpha_f' on air
// cells, 0 on solid cells): the six neighbours' coefficients and values are
// loaded without branches; a closed face gets beta = 0 and an air neighbour
// the value 0, so the sum is the operator's for any values v.  val(n, i, j, k)
// gives the value of cell n at (i, j, k).
template <typename V>
__device__ inline double face_sum_ac(const IdpDims &D, int64_t c, int64_t i, int64_t j, int64_t k,
                                     const double *__restrict__ ac, V val)
{
    const int64_t off[6] = {-1, 1, -D.nx, D.nx, -D.sxy, D.sxy};
    const bool in[6] = {i > 0, i < D.nx - 1, j > 0, j < D.ny - 1, k > 0, k < D.nz - 1};
    const int64_t di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
    const double a = ac[c], vc = val(c, i, j, k);
    double an[6], vn[6];
    // a neighbour outside the box reads the cell itself (so that every load is
    // issued without a branch, all before any is used) and gets an = 0: it
    // contributes nothing, whatever vn holds
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int64_t n = c + (in[f] ? off[f] : 0);
        an[f] = ac[n];
        vn[f] = val(n, in[f] ? i + di[f] : i, in[f] ? j + dj[f] : j, in[f] ? k + dk[f] : k);
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) an[f] = in[f] ? an[f] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const double beta = an[f] != 0.0 ? (a + fabs(an[f])) * 0.5 : 0.0;
        const double v = an[f] > 0.0 ? vn[f] : 0.0;
        acc += beta * (vc - v);
    }
    return acc;
}

__global__ void __launch_bounds__(kIdpThreads) k_idp_setup(IdpDims D, double alpha_max,
                                                           const int64_t *__restrict__ afx,
                                                           const double *__restrict__ astar,
                                                           const uint8_t *__restrict__ lab, double *__restrict__ at,
                                                           double *__restrict__ s, int64_t *err)
{
#pragma clang fp contract(off)
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        if (lab[c] > kIdpSolid) raise_error(err, kErrRange, c);
        double as = (double)afx[c] * 2.3283064365386963e-10;  // 2^-32
        as = as < alpha_max ? as : alpha_max;
        const double a = 1.0 - as;
        at[c] = a;
        double ratio = astar[c] / a;
        ratio = ratio < 0.5 ? 0.5 : (ratio > 1.5 ? 1.5 : ratio);
        s[c] = lab[c] == kIdpFluid ? a * (ratio - 1.0) : 0.0;
    }
}

__global__ void __launch_bounds__(kIdpThreads) k_idp_apply(IdpDims D, const double *__restrict__ at,
                                                           const uint8_t *__restrict__ lab,
                                                           const double *__restrict__ v, double *__restrict__ out)
{
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        double Lv, dg;
        apply_row(D, c, at, lab, v, Lv, dg);
        out[c] = Lv;
    }
}

// CG start: r = s - L q, z = r / diag, d = z, the signed coefficients ac
// (alpha_f' on fluid cells, -alpha_f' on air cells, 0 on solid cells) that
// the iteration kernels read instead of alpha_f' and the labels; partials of
// s.s, r.z, r.r.
__global__ void __launch_bounds__(kIdpThreads) k_cg_init(IdpDims D, const double *__restrict__ at,
                                                         const uint8_t *__restrict__ lab,
                                                         const double *__restrict__ s, const double *__restrict__ q,
                                                         double *__restrict__ r, double *__restrict__ d,
                                                         double *__restrict__ dinv, double *__restrict__ ac,
                                                         double *__restrict__ part, CgState *__restrict__ st,
                                                         int64_t *err)
{
    __shared__ double red[4];
    double rz = 0.0, rr = 0.0, ss = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        double Lq, dg;
        apply_row(D, c, at, lab, q, Lq, dg);
        const uint8_t lc = lab[c];
        // the signed coefficients need alpha_f' > 0 on fluid and air cells and a known label
        if (lc > kIdpSolid || (lc != kIdpSolid && !(at[c] > 0.0 && at[c] < INFINITY)))
            raise_error(err, kErrRange, c);
        ac[c] = lc == kIdpFluid ? at[c] : (lc == kIdpAir ? -at[c] : 0.0);
        const double sc = lab[c] == kIdpFluid ? s[c] : 0.0;
        const double rc = sc - Lq;
        const double di = dg > 0.0 ? 1.0 / dg : 0.0;  // a fluid cell walled in on all sides: singular row
        const double zc = rc * di;
        r[c] = rc;
        d[c] = zc;
        dinv[c] = di;
        rz += rc * zc;
        rr += rc * rc;
        ss += sc * sc;
    }
    const int nb = gridDim.x;
    rz = block_sum(rz, red);
    rr = block_sum(rr, red);
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = ss;
        part[nb + blockIdx.x] = rz;
        part[2 * nb + blockIdx.x] = rr;
        if (blockIdx.x == 0) st->done = -1;  // kernels of a previous solve may have left it set
    }
}

// Reduces the start partials into the scalar state (one block).
__global__ void __launch_bounds__(kIdpThreads) k_cg_start(int nb, const double *__restrict__ part, double tol,
                                                          CgState *__restrict__ st)
{
    __shared__ double red[4];
    const double ss = sum_partials(part, nb, red);
    const double rz = sum_partials(part + nb, nb, red);
    const double rr = sum_partials(part + 2 * nb, nb, red);
    if (threadIdx.x == 0) {
        st->rz[0] = rz;
        st->rz[1] = rz;
        st->ss = ss;
        st->thr = tol * tol * ss;
        st->rr = rr;
        st->done = rr <= tol * tol * ss ? 0 : -1;
        st->iters = 0;
    }
}

// Stencil passes blocked in 2.5D.
//   MODE 0, iteration k, part 1: w = L d, the partials of d.w in
//     part[block].
//   MODE 1, the multigrid post-sweep from the prolonged iterate d = u:
//     w = e = u + omega D^-1 (b - A u) on fluid cells, b elsewhere; the
//     partials of b.e in part[nblocks + block] when part is given.
//   MODE 2, the residual after the pre-sweep from zero, e1 = omega D^-1 b
//     (formed as each value is loaded): w = b - A e1 on fluid cells, 0
//     elsewhere, for the restriction.
// A block takes x-y tiles of kTileX x kTileY cells (each wave kTileRows rows)
// and a run of zlen planes.  It keeps its columns' coefficients and values for
// planes z - 1, z, z + 1 in registers and the tile of plane z with a one-cell
// halo in LDS, so that each operand is read from memory about once instead of
// once per neighbour; the next plane of each column and the next halo are
// loaded one step ahead, within the run.  The face sum is face_sum_ac's, term
// by term in the same order (cells outside the box hold coefficient 0 and
// value 0).  Items (tile, run of planes) are dealt to the blocks; the block
// count is the other iteration kernels', whose partial sums these kernels'
// must match.
constexpr double kOmega = 2.0 / 3.0;  // damping of the multigrid's Jacobi sweeps
constexpr int kTileRows = 2;  // tile rows per wave (rows row and row + 4 of the tile)
constexpr int kTileX = 64, kTileY = kIdpThreads / 64 * kTileRows;

template <int MODE>
__global__ void __launch_bounds__(kIdpThreads) k_stencil_tiled(IdpDims D, int ntx, int nty, int zlen,
                                                               const double *__restrict__ ac,
                                                               const double *__restrict__ d,
                                                               const double *__restrict__ b,
                                                               const double *__restrict__ dinv, double scale,
                                                               double *__restrict__ w, double *__restrict__ part,
                                                               const CgState *__restrict__ st)
{
    constexpr int kWaves = kIdpThreads / 64;
    __shared__ double red[4];
    __shared__ double sa[kTileY + 2][kTileX + 2], sv[kTileY + 2][kTileX + 2];
    if (st->done >= 0) return;
    // the value a cell contributes: d, or the pre-sweep iterate w D^-1 b of the residual pass
    auto val = [&](int64_t n) { return MODE == 2 ? kOmega * dinv[n] * b[n] : d[n]; };
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6, t = threadIdx.x;
    const int64_t nx = D.nx, ny = D.ny, nz = D.nz;
    const int64_t tiles = (int64_t)ntx * nty, nzc = (nz + zlen - 1) / zlen, items = tiles * nzc;
    // halo slot of this thread: rows below and above the tile (t < 128), columns left and right (t < 144)
    int hr = -1, hc = -1, hdi = 0, hdj = 0;
    if (t < kTileX) { hr = 0; hc = t + 1; hdi = t; hdj = -1; }
    else if (t < 2 * kTileX) { hr = kTileY + 1; hc = t - kTileX + 1; hdi = t - kTileX; hdj = kTileY; }
    else if (t < 2 * kTileX + kTileY) { hr = t - 2 * kTileX + 1; hc = 0; hdi = -1; hdj = t - 2 * kTileX; }
    else if (t < 2 * kTileX + 2 * kTileY) { hr = t - 2 * kTileX - kTileY + 1; hc = kTileX + 1; hdi = kTileX; hdj = t - 2 * kTileX - kTileY; }
    // items in tile order within a run of planes; workgroups are dealt to the
    // eight XCDs in turn, so block b starts at item (b % 8) nb/8 + b/8 and each
    // XCD takes a contiguous eighth (y-adjacent tiles share its L2)
    const int64_t nb = gridDim.x;
    const int64_t first = nb % 8 ? (int64_t)blockIdx.x : (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    double dw = 0.0;
    for (int64_t it = first; it < items; it += nb) {
        const int64_t tile = it % tiles, z0 = (it / tiles) * zlen;
        const int64_t z1 = z0 + zlen < nz ? z0 + zlen : nz;
        const int64_t i0 = (tile % ntx) * kTileX, j0 = (tile / ntx) * kTileY;
        const int64_t i = i0 + lane;
        bool own[kTileRows];
        int64_t col[kTileRows];  // cell index of (i, j, 0) for the thread's rows
#pragma unroll
        for (int q = 0; q < kTileRows; ++q) {
            const int64_t j = j0 + row + q * kWaves;
            own[q] = i < nx && j < ny;
            col[q] = j * nx + i;
        }
        const int64_t hi = i0 + hdi, hj = j0 + hdj;
        const bool hown = hr >= 0 && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
        const int64_t hcol = hj * nx + hi;
        // columns: m = z - 1, 0 = z, p = z + 1; halo of plane z
        double am[kTileRows], vm[kTileRows], a0[kTileRows], v0[kTileRows], ap[kTileRows], vp[kTileRows];
        double b0[kTileRows], di0[kTileRows];  // right-hand side and 1/diag of plane z (sweep)
        double ha = 0.0, hv = 0.0;
#pragma unroll
        for (int q = 0; q < kTileRows; ++q) {
            am[q] = vm[q] = a0[q] = v0[q] = ap[q] = vp[q] = b0[q] = di0[q] = 0.0;
            if (MODE != 0 && own[q]) b0[q] = b[col[q] + z0 * D.sxy];
            if (MODE == 1 && own[q]) di0[q] = dinv[col[q] + z0 * D.sxy];
            if (own[q] && z0 > 0) { am[q] = ac[col[q] + (z0 - 1) * D.sxy]; vm[q] = val(col[q] + (z0 - 1) * D.sxy); }
            if (own[q]) { a0[q] = ac[col[q] + z0 * D.sxy]; v0[q] = val(col[q] + z0 * D.sxy); }
            if (own[q] && z0 + 1 < nz) { ap[q] = ac[col[q] + (z0 + 1) * D.sxy]; vp[q] = val(col[q] + (z0 + 1) * D.sxy); }
        }
        if (hown) { ha = ac[hcol + z0 * D.sxy]; hv = val(hcol + z0 * D.sxy); }
        for (int64_t z = z0; z < z1; ++z) {
            // one step ahead: the columns' plane z + 2 and the halo of plane z + 1
            double a2[kTileRows], v2[kTileRows], b1[kTileRows], di1[kTileRows], ha1 = 0.0, hv1 = 0.0;
#pragma unroll
            for (int q = 0; q < kTileRows; ++q) {
                a2[q] = v2[q] = b1[q] = di1[q] = 0.0;
                if (MODE != 0 && own[q] && z + 1 < z1) b1[q] = b[col[q] + (z + 1) * D.sxy];
                if (MODE == 1 && own[q] && z + 1 < z1) di1[q] = dinv[col[q] + (z + 1) * D.sxy];
                // plane z1 is the last one the run reads (the +z neighbour of its last plane)
                if (own[q] && z + 2 <= z1 && z + 2 < nz) {
                    a2[q] = ac[col[q] + (z + 2) * D.sxy];
                    v2[q] = val(col[q] + (z + 2) * D.sxy);
                }
            }
            if (hown && z + 1 < z1) { ha1 = ac[hcol + (z + 1) * D.sxy]; hv1 = val(hcol + (z + 1) * D.sxy); }
            __syncthreads();  // the previous plane's reads of the tile are done
#pragma unroll
            for (int q = 0; q < kTileRows; ++q) {
                sa[row + q * kWaves + 1][lane + 1] = a0[q];
                sv[row + q * kWaves + 1][lane + 1] = v0[q];
            }
            if (hr >= 0) { sa[hr][hc] = ha; sv[hr][hc] = hv; }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kTileRows; ++q) {
                if (!own[q]) continue;
                const int r = row + q * kWaves + 1;  // the cell's row in the tile
                const double an[6] = {sa[r][lane], sa[r][lane + 2], sa[r - 1][lane + 1], sa[r + 1][lane + 1], am[q], ap[q]};
                const double vn[6] = {sv[r][lane], sv[r][lane + 2], sv[r - 1][lane + 1], sv[r + 1][lane + 1], vm[q], vp[q]};
                double acc = 0.0;
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const double beta = an[f] != 0.0 ? (a0[q] + fabs(an[f])) * 0.5 : 0.0;
                    const double v = an[f] > 0.0 ? vn[f] : 0.0;
                    acc += beta * (v0[q] - v);
                }
                if (MODE == 2) {
                    w[col[q] + z * D.sxy] = a0[q] > 0.0 ? b0[q] - scale * acc : 0.0;
                } else if (MODE == 1) {
                    const double Au = scale * acc;
                    const double e = a0[q] > 0.0 ? v0[q] + kOmega * di0[q] * (b0[q] - Au) : b0[q];
                    w[col[q] + z * D.sxy] = e;
                    dw += b0[q] * e;
                } else {
                    const double Lv = a0[q] > 0.0 ? acc : v0[q];  // identity row off the fluid
                    w[col[q] + z * D.sxy] = Lv;
                    dw += v0[q] * Lv;
                }
            }
#pragma unroll
            for (int q = 0; q < kTileRows; ++q) {
                am[q] = a0[q]; vm[q] = v0[q]; a0[q] = ap[q]; v0[q] = vp[q]; ap[q] = a2[q]; vp[q] = v2[q];
                b0[q] = b1[q]; di0[q] = di1[q];
            }
            ha = ha1; hv = hv1;
        }
    }
    if (MODE == 0 || (MODE == 1 && part)) {
        dw = block_sum(dw, red);
        if (threadIdx.x == 0) part[(MODE == 1 ? nb : 0) + blockIdx.x] = dw;
    }
}

template <bool JAC>
__global__ void __launch_bounds__(kIdpThreads) k_cg_update(IdpDims D, int k, const double *__restrict__ d,
                                                           const double *__restrict__ w,
                                                           const double *__restrict__ dinv, double *__restrict__ q,
                                                           double *__restrict__ r, double *__restrict__ part,
                                                           const CgState *__restrict__ st)
{
    __shared__ double red[4];
    if (st->done >= 0) return;
    const int nb = gridDim.x;
    const double dw = sum_partials(part, nb, red);
    const double alpha = st->rz[k & 1] / dw;
    double rz = 0.0, rr = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        q[c] += alpha * d[c];
        const double rc = r[c] - alpha * w[c];
        r[c] = rc;
        if (JAC) rz += rc * (rc * dinv[c]);
        rr += rc * rc;
    }
    if (JAC) rz = block_sum(rz, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        if (JAC) part[nb + blockIdx.x] = rz;  // with multigrid the V-cycle writes r.z
        part[2 * nb + blockIdx.x] = rr;
    }
}

// Iteration k, part 3: rz_{k+1}, r.r; stop at r.r <= tol^2 s.s, else
// d = z + (rz_{k+1} / rz_k) d.  Block 0 records the state for iteration k + 1
// in the other rz slot (the current one is still read by other blocks).
template <bool JAC>
__global__ void __launch_bounds__(kIdpThreads) k_cg_direction(IdpDims D, int k, const double *__restrict__ r,
                                                              const double *__restrict__ dinv,
                                                              const double *__restrict__ z, double *__restrict__ d,
                                                              const double *__restrict__ part,
                                                              CgState *__restrict__ st)
{
    __shared__ double red[4];
    __shared__ int64_t s_done;
    // block 0 of this kernel may set done while others start: read it once per block
    if (threadIdx.x == 0) s_done = st->done;
    __syncthreads();
    if (s_done >= 0) return;
    const int nb = gridDim.x;
    const double rz1 = sum_partials(part + nb, nb, red);
    const double rr = sum_partials(part + 2 * nb, nb, red);
    const bool conv = rr <= st->thr;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rz[(k + 1) & 1] = rz1;
        st->rr = rr;
        st->iters = k + 1;
        if (conv) st->done = k + 1;
    }
    if (conv) return;
    const double beta = rz1 / st->rz[k & 1];
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < D.G;
         c += (int64_t)gridDim.x * kIdpThreads)
        d[c] = (JAC ? r[c] * dinv[c] : z[c]) + beta * d[c];
}

// Face displacements (Eq. 13): for the face from cell c to its +axis
// neighbour j, dx (q_c - q_j) with air sides at q = 0, where one side is fluid
// and neither is solid, clamped to [-dx, dx]; faces on the box boundary are
// zero.  The thread of cell c writes the three faces above it and, on the
// lower box faces, the boundary face below it.
__global__ void __launch_bounds__(kIdpThreads) k_idp_faces(IdpDims D, double dx, const double *__restrict__ q,
                                                           const uint8_t *__restrict__ lab, double *__restrict__ fx,
                                                           double *__restrict__ fy, double *__restrict__ fz)
{
#pragma clang fp contract(off)
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        int64_t i, j, k;
        coords(D, c, i, j, k);
        const uint8_t lc = lab[c];
        const double qc = lc == kIdpFluid ? q[c] : 0.0;
        const bool up[3] = {i < D.nx - 1, j < D.ny - 1, k < D.nz - 1};
        const int64_t off[3] = {1, D.nx, D.sxy};
        double *const F[3] = {fx, fy, fz};
        // face index of the face above c along each axis
        const int64_t fi[3] = {(k * D.ny + j) * (D.nx + 1) + i + 1, (k * (D.ny + 1) + j + 1) * D.nx + i,
                               ((k + 1) * D.ny + j) * D.nx + i};
        const int64_t step[3] = {1, D.nx, D.sxy};  // face-index distance to the face below c
        const bool low[3] = {i == 0, j == 0, k == 0};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double val = 0.0;
            if (up[a]) {
                const uint8_t ln = lab[c + off[a]];
                const bool live =
                    (lc == kIdpFluid || ln == kIdpFluid) && lc != kIdpSolid && ln != kIdpSolid;
                if (live) {
                    const double qn = ln == kIdpFluid ? q[c + off[a]] : 0.0;
                    val = dx * (qc - qn);
                    val = val > -dx ? val : -dx;
                    val = val < dx ? val : dx;
                }
            }
            F[a][fi[a]] = val;
            if (low[a]) F[a][fi[a] - step[a]] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Multigrid preconditioner: one symmetric V-cycle per CG iteration.  Level
// l + 1 halves level l per axis (rounding up); a coarse cell is air if any of
// its children is air, else fluid if any child is fluid, else solid, and its
// alpha_f' is the mean over its children that are not solid.  The level
// operator is A_l = 4^l L(alpha_f'_l, labels_l), which for constant
// coefficients is the Galerkin product R A_{l-1} P of piecewise-constant
// prolongation P (a fluid coarse cell's correction added to its fluid
// children) and R = P^T (the sum of the fluid children's residuals).
// Smoothing: one damped Jacobi sweep (omega = 2/3) before and one after the
// coarse correction; the pre-sweep from zero, w D^-1 b, is formed on the fly
// where it is used.  A small level costs two passes (restriction; correction
// and post-sweep); a level of at least kMgSplitCells cells four (residual into
// t, restriction of t, prolongation into t, post-sweep).  The coarsest level (at most 256 cells) takes 48 sweeps in
// LDS.  Equal pre- and post-sweeps and R = P^T keep the preconditioner
// symmetric.  Non-fluid rows of the finest level are identity rows and get
// z = r.  Levels carry the signed coefficients (see face_sum_ac).
constexpr int kCoarseSweeps = 48;

// uniform per block: read the solver state once
__device__ inline bool cg_done(const CgState *st)
{
    __shared__ int64_t s_done;
    if (threadIdx.x == 0) s_done = st->done;
    __syncthreads();
    return s_done >= 0;
}

__global__ void __launch_bounds__(kIdpThreads) k_mg_coarsen(MgLevel F, MgLevel Cl)
{
    for (int64_t C = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; C < Cl.D.G;
         C += (int64_t)gridDim.x * kIdpThreads) {
        int64_t I, J, K;
        coords(Cl.D, C, I, J, K);
        bool air = false, fluid = false;
        double sum = 0.0;
        int cnt = 0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    const int64_t i = 2 * I + a, j = 2 * J + b, k = 2 * K + c;
                    if (i >= F.D.nx || j >= F.D.ny || k >= F.D.nz) continue;
                    const double v = F.ac[(k * F.D.ny + j) * F.D.nx + i];
                    air |= v < 0.0;
                    fluid |= v > 0.0;
                    if (v != 0.0) {
                        sum += fabs(v);
                        ++cnt;
                    }
                }
        const double mean = cnt ? sum / cnt : 0.0;
        Cl.ac[C] = air ? -mean : (fluid ? mean : 0.0);
    }
}

__global__ void __launch_bounds__(kIdpThreads) k_mg_diag(MgLevel L)
{
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < L.D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        double di = 1.0;
        if (L.ac[c] > 0.0) {
            int64_t i, j, k;
            coords(L.D, c, i, j, k);
            // the face sum of v = 1 on c and 0 on every neighbour is the diagonal
            const double dg =
                face_sum_ac(L.D, c, i, j, k, L.ac, [&](int64_t n, int64_t, int64_t, int64_t) { return n == c ? 1.0 : 0.0; });
            di = dg > 0.0 ? 1.0 / (L.scale * dg) : 0.0;
        }
        L.dinv[c] = di;
    }
}

// Restriction after one pre-smoothing sweep from zero, e1 = w D^-1 b (formed
// on the fly): the coarse right-hand side is the sum of the fluid children's
// residuals b - A e1.  Eight adjacent lanes take the eight children of one
// coarse cell (lane bits: x, y, z offset) and add their residuals with three
// butterfly shuffles, the same order in every group.
__global__ void __launch_bounds__(kIdpThreads) k_mg_restrict(MgLevel F, MgLevel Cl, const double *__restrict__ r1,
                                                            const CgState *__restrict__ st)
{
    if (cg_done(st)) return;
    auto e1 = [&](int64_t n, int64_t, int64_t, int64_t) { return kOmega * F.dinv[n] * F.b[n]; };
    const int64_t total = 8 * Cl.D.G;  // a multiple of 8: the lanes of a group leave the loop together
    for (int64_t t = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * kIdpThreads) {
        const int64_t C = t >> 3;
        const int ch = (int)(t & 7);
        double v = 0.0;
        if (Cl.ac[C] > 0.0) {
            int64_t I, J, K;
            coords(Cl.D, C, I, J, K);
            const int64_t i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
            if (i < F.D.nx && j < F.D.ny && k < F.D.nz) {
                const int64_t f = (k * F.D.ny + j) * F.D.nx + i;
                if (r1)
                    v = r1[f];  // the residual pass's value: zero off the fluid
                else if (F.ac[f] > 0.0)
                    v = F.b[f] - F.scale * face_sum_ac(F.D, f, i, j, k, F.ac, e1);
            }
        }
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        if (ch == 0) Cl.b[C] = v;
    }
}

// Restriction of stored residuals r1 (zero off the fluid): one thread per
// coarse cell adds its eight children in the order of k_mg_restrict's
// butterfly, ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7)) with child
// bits (x, y, z), so the coarse right-hand side is the same bit for bit.
__global__ void __launch_bounds__(kIdpThreads) k_mg_restrict_sum(MgLevel F, MgLevel Cl,
                                                                const double *__restrict__ r1,
                                                                const CgState *__restrict__ st)
{
    if (cg_done(st)) return;
    for (int64_t C = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; C < Cl.D.G;
         C += (int64_t)gridDim.x * kIdpThreads) {
        double v = 0.0;
        if (Cl.ac[C] > 0.0) {
            int64_t I, J, K;
            coords(Cl.D, C, I, J, K);
            double c[8];
#pragma unroll
            for (int ch = 0; ch < 8; ++ch) {
                const int64_t i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
                c[ch] = i < F.D.nx && j < F.D.ny && k < F.D.nz ? r1[(k * F.D.ny + j) * F.D.nx + i] : 0.0;
            }
            v = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
        }
        Cl.b[C] = v;
    }
}

// Coarse correction alone: u = e1 + P E on fluid cells (0 elsewhere) into t,
// for the larger levels, where the post-sweep then reads u once per
// neighbour.
__global__ void __launch_bounds__(kIdpThreads) k_mg_prolong(MgLevel F, MgLevel Cl, const CgState *__restrict__ st)
{
    if (cg_done(st)) return;
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < F.D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        double u = 0.0;
        if (F.ac[c] > 0.0) {
            int64_t i, j, k;
            coords(F.D, c, i, j, k);
            const int64_t p = ((k >> 1) * Cl.D.ny + (j >> 1)) * Cl.D.nx + (i >> 1);
            u = kOmega * F.dinv[c] * F.b[c];
            if (Cl.ac[p] > 0.0) u += Cl.e[p];
        }
        F.t[c] = u;
    }
}

// Coarse correction and one post-smoothing sweep: u = e1 + P E, e = u + w D^-1
// (b - A u) (e = b on non-fluid rows); on the finest level also the partials
// of b.e (= r.z of the CG iteration).
__global__ void __launch_bounds__(kIdpThreads) k_mg_post(MgLevel F, MgLevel Cl, double *__restrict__ part,
                                                         const CgState *__restrict__ st)
{
    __shared__ double red[4];
    if (cg_done(st)) return;
    auto u = [&](int64_t n, int64_t i, int64_t j, int64_t k) {
        const int64_t p = ((k >> 1) * Cl.D.ny + (j >> 1)) * Cl.D.nx + (i >> 1);
        const double e1 = kOmega * F.dinv[n] * F.b[n];
        return Cl.ac[p] > 0.0 ? e1 + Cl.e[p] : e1;
    };
    double rz = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kIdpThreads + threadIdx.x; c < F.D.G;
         c += (int64_t)gridDim.x * kIdpThreads) {
        double z = F.b[c];
        if (F.ac[c] > 0.0) {
            int64_t i, j, k;
            coords(F.D, c, i, j, k);
            const double Au = F.scale * face_sum_ac(F.D, c, i, j, k, F.ac, u);
            z = u(c, i, j, k) + kOmega * F.dinv[c] * (F.b[c] - Au);
        }
        F.e[c] = z;
        rz += F.b[c] * z;
    }
    if (part) {
        rz = block_sum(rz, red);
        if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = rz;
    }
}

// The coarsest level (at most 256 cells) in one block: kCoarseSweeps damped
// Jacobi sweeps from zero, in LDS.
__global__ void __launch_bounds__(kIdpThreads) k_mg_coarsest(MgLevel L, const CgState *__restrict__ st)
{
    __shared__ double se[2][kIdpThreads], sb[kIdpThreads], sdi[kIdpThreads], sac[kIdpThreads];
    if (cg_done(st)) return;
    const int c = threadIdx.x;
    const bool live = c < L.D.G;
    sb[c] = live ? L.b[c] : 0.0;
    sdi[c] = live ? L.dinv[c] : 0.0;
    sac[c] = live ? L.ac[c] : 0.0;
    se[0][c] = 0.0;
    int64_t i = 0, j = 0, k = 0;
    if (live) coords(L.D, c, i, j, k);
    __syncthreads();
    for (int s = 0; s < kCoarseSweeps; ++s) {
        const int cur = s & 1;
        double v = 0.0;
        if (live && sac[c] > 0.0) {
            const double Ae = L.scale * face_sum_ac(L.D, (int64_t)c, i, j, k, sac,
                                                    [&](int64_t n, int64_t, int64_t, int64_t) { return se[cur][n]; });
            v = se[cur][c] + kOmega * sdi[c] * (sb[c] - Ae);
        }
        se[cur ^ 1][c] = v;
        __syncthreads();
    }
    if (live) L.e[c] = se[kCoarseSweeps & 1][c];
}

unsigned idp_blocks(int64_t G)
{
    const int64_t b = (G + kIdpThreads - 1) / kIdpThreads;
    return (unsigned)(b < 1 ? 1 : (b > kIdpMaxBlocks ? kIdpMaxBlocks : b));
}

// One thread per cell for kernels that write no partials (grid-stride
// beyond 2^31 - 1 blocks).
unsigned idp_blocks_full(int64_t G)
{
    const int64_t b = (G + kIdpThreads - 1) / kIdpThreads;
    return (unsigned)(b < 1 ? 1 : (b > 0x7fffffffll ? 0x7fffffffll : b));
}

}  // namespace

// m = ceil(2^(31+s) / d) with 2^(s-1) < d <= 2^s: m < 2^32, and m d - 2^(31+s)
// < d <= 2^s, so floor(n m / 2^(31+s)) = floor(n / d) for every n < 2^31
// (the round-up reciprocal of Granlund and Montgomery, 1994).
static void div_constants(int64_t d, uint32_t &m, int32_t &sh)
{
    int s = 0;
    while ((int64_t(1) << s) < d) ++s;
    if (d < 1 || s > 31) {  // grids of 2^31 cells or more divide in 64 bits
        m = 0;
        sh = 0;
        return;
    }
    m = (uint32_t)(((uint64_t(1) << (31 + s)) + (uint64_t)d - 1) / (uint64_t)d);
    sh = 31 + s;
}

void idp_dims_finish(IdpDims &D)
{
    D.sxy = D.nx * D.ny;
    D.G = D.sxy * D.nz;
    div_constants(D.nx, D.mx, D.shx);
    div_constants(D.ny, D.my, D.shy);
}

IdpDims idp_dims(const DevParams &P)
{
    IdpDims D;
    D.nx = P.n[0];
    D.ny = P.n[1];
    D.nz = P.n[2];
    idp_dims_finish(D);
    return D;
}

hipError_t launch_idp_setup(const IdpDims &D, double alpha_max, const int64_t *afx, const double *astar,
                            const uint8_t *lab, double *at, double *s, int64_t *err, hipStream_t st)
{
    k_idp_setup<<<idp_blocks(D.G), kIdpThreads, 0, st>>>(D, alpha_max, afx, astar, lab, at, s, err);
    return hipGetLastError();
}

hipError_t launch_idp_apply(const IdpDims &D, const double *at, const uint8_t *lab, const double *v, double *out,
                            hipStream_t st)
{
    k_idp_apply<<<idp_blocks(D.G), kIdpThreads, 0, st>>>(D, at, lab, v, out);
    return hipGetLastError();
}

hipError_t launch_idp_faces(const IdpDims &D, double dx, const double *q, const uint8_t *lab, double *fx,
                            double *fy, double *fz, hipStream_t st)
{
    k_idp_faces<<<idp_blocks(D.G), kIdpThreads, 0, st>>>(D, dx, q, lab, fx, fy, fz);
    return hipGetLastError();
}

// z = M^-1 r by one V-cycle over the levels of W (level 0 works on r and z).
// Levels with at least this many cells prolong in a pass of their own and
// then sweep; smaller levels do both in one pass (launch latency dominates).
constexpr int64_t kMgSplitCells = 1 << 18;

// Tiles of a blocked stencil pass over D and the planes per item: about one
// item per block of nb.
static void stencil_items(const IdpDims &D, unsigned nb, int &ntx, int &nty, int &zlen)
{
    ntx = (int)((D.nx + kTileX - 1) / kTileX);
    nty = (int)((D.ny + kTileY - 1) / kTileY);
    const int64_t zl = (D.nz * ntx * nty + nb - 1) / nb;
    zlen = (int)(zl < 1 ? 1 : (zl > D.nz ? D.nz : zl));
}

static void launch_vcycle(const IdpWork &W, hipStream_t st)
{
    const int L = W.nlev;
    for (int l = 0; l + 1 < L; ++l) {
        const MgLevel &F = W.lev[l];
        const double *r1 = nullptr;
        if (F.D.G >= kMgSplitCells) {  // the fine residual by the blocked pass, into t (free until prolongation)
            const unsigned nb = idp_blocks(F.D.G);
            int ntx, nty, zlen;
            stencil_items(F.D, nb, ntx, nty, zlen);
            k_stencil_tiled<2><<<nb, kIdpThreads, 0, st>>>(F.D, ntx, nty, zlen, F.ac, nullptr, F.b, F.dinv, F.scale,
                                                           F.t, nullptr, W.state);
            r1 = F.t;
        }
        if (r1)
            k_mg_restrict_sum<<<idp_blocks_full(W.lev[l + 1].D.G), kIdpThreads, 0, st>>>(F, W.lev[l + 1], r1,
                                                                                      W.state);
        else
            k_mg_restrict<<<idp_blocks_full(8 * W.lev[l + 1].D.G), kIdpThreads, 0, st>>>(F, W.lev[l + 1], nullptr,
                                                                                         W.state);
    }
    k_mg_coarsest<<<1, kIdpThreads, 0, st>>>(W.lev[L - 1], W.state);
    for (int l = L - 2; l >= 0; --l) {
        const unsigned nb = idp_blocks(W.lev[l].D.G);
        double *part = l == 0 ? W.part : nullptr;
        if (W.lev[l].D.G >= kMgSplitCells) {
            k_mg_prolong<<<idp_blocks_full(W.lev[l].D.G), kIdpThreads, 0, st>>>(W.lev[l], W.lev[l + 1], W.state);
            const MgLevel &F = W.lev[l];
            int ntx, nty, zlen;
            stencil_items(F.D, nb, ntx, nty, zlen);
            k_stencil_tiled<1><<<nb, kIdpThreads, 0, st>>>(F.D, ntx, nty, zlen, F.ac, F.t, F.b, F.dinv, F.scale,
                                                               F.e, part, W.state);
        } else {
            k_mg_post<<<nb, kIdpThreads, 0, st>>>(W.lev[l], W.lev[l + 1], part, W.state);
        }
    }
}

hipError_t launch_cg_start(const IdpDims &D, const double *at, const uint8_t *lab, const double *s, const double *q,
                           const IdpWork &W, double tol, int64_t *err, hipStream_t st)
{
    const unsigned nb = idp_blocks(D.G);
    k_cg_init<<<nb, kIdpThreads, 0, st>>>(D, at, lab, s, q, W.r, W.d, W.dinv, W.lev[0].ac, W.part, W.state, err);
    if (W.nlev > 1) {
        for (int l = 0; l + 1 < W.nlev; ++l) {
            k_mg_coarsen<<<idp_blocks(W.lev[l + 1].D.G), kIdpThreads, 0, st>>>(W.lev[l], W.lev[l + 1]);
            k_mg_diag<<<idp_blocks(W.lev[l + 1].D.G), kIdpThreads, 0, st>>>(W.lev[l + 1]);
        }
        launch_vcycle(W, st);
        hipError_t e = hipMemcpyAsync(W.d, W.lev[0].e, sizeof(double) * D.G, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    k_cg_start<<<1, kIdpThreads, 0, st>>>((int)nb, W.part, tol, W.state);
    return hipGetLastError();
}

hipError_t launch_cg_iterations(const IdpDims &D, const double *at, const uint8_t *lab, double *q,
                                const IdpWork &W, int k0, int count, hipStream_t st)
{
    const unsigned nb = idp_blocks(D.G);
    const bool mg = W.nlev > 1;
    int ntx, nty, zlen;
    stencil_items(D, nb, ntx, nty, zlen);
    for (int k = k0; k < k0 + count; ++k) {
        k_stencil_tiled<0><<<nb, kIdpThreads, 0, st>>>(D, ntx, nty, zlen, W.lev[0].ac, W.d, nullptr, nullptr,
                                                            1.0, W.w, W.part, W.state);
        if (mg) {
            k_cg_update<false><<<nb, kIdpThreads, 0, st>>>(D, k, W.d, W.w, W.dinv, q, W.r, W.part, W.state);
            launch_vcycle(W, st);
            k_cg_direction<false><<<nb, kIdpThreads, 0, st>>>(D, k, W.r, W.dinv, W.lev[0].e, W.d, W.part, W.state);
        } else {
            k_cg_update<true><<<nb, kIdpThreads, 0, st>>>(D, k, W.d, W.w, W.dinv, q, W.r, W.part, W.state);
            k_cg_direction<true><<<nb, kIdpThreads, 0, st>>>(D, k, W.r, W.dinv, nullptr, W.d, W.part, W.state);
        }
    }
    return hipGetLastError();
}

}  // namespace gic
