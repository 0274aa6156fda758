// a4 + a5: granule <-> grid transfers with the quadratic B-spline on
// cell-centred nodes (Sec. 5.1 Eq. 7a; Sec. 5.2 G2P) on gfx950.
//
// P2G: one workgroup per brick of 4x4x4 neighbour cells.  Granules of a brick
// are contiguous in sorted order and their stencils cover a small box of
// nodes, so their 27-node x 4-channel contributions are first summed in
// registers over runs of granules that share a stencil, then in an LDS tile
// with 64-bit LDS atomics, and then added to the grid with one global atomic
// per touched node and channel.  A contribution whose node falls
// outside the tile (a granule that moved after the sort) goes straight to a
// global atomic, so the result never depends on the order.  Fixed-point
// contributions are integers, so every accumulation order gives the same
// bits.
//
// G2P: one thread per granule, 27 node reads from L1/L2 (sorted granules
// read overlapping stencils).
//
// The unquantised transfers of the differentiable form (P2G and the grid
// part of the G2P pullback) round every contribution to an integer at a
// scale set by the largest contribution of the call and sum integers, so
// their grids are the same bits in every run.
#include "gic_launch.hpp"

namespace gic {

namespace {

constexpr int kP2GThreads = 256;

__global__ void __launch_bounds__(256) k_fill_i64(int64_t *a, int64_t len)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

__global__ void __launch_bounds__(256) k_fill_f64(double *a, int64_t len)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

// [begin, end) of brick b in sorted order, from the 64 cell ranges of the
// brick (each clipped to [0, n)); returned through LDS to the whole
// workgroup.
__device__ inline void brick_range(int64_t n, int64_t b, const int32_t *__restrict__ cb,
                                   const int32_t *__restrict__ ce, int32_t *s_range)
{
    if (threadIdx.x < 64) {
        const int64_t key = b * kBrickCells + threadIdx.x;
        int32_t bb = cb[key], ee = ce[key];
        clip_range(n, bb, ee);
        int32_t lo = ee > bb ? bb : 0x7fffffff;
        int32_t hi = ee > bb ? ee : 0;
        for (int off = 32; off > 0; off >>= 1) {
            int32_t olo = __shfl_xor(lo, off);
            int32_t ohi = __shfl_xor(hi, off);
            lo = olo < lo ? olo : lo;
            hi = ohi > hi ? ohi : hi;
        }
        if (threadIdx.x == 0) {
            s_range[0] = lo;
            s_range[1] = hi;
        }
    }
}

// Add an integer contribution to the LDS tile, or to the grid when its node
// lies outside the tile.  The two atomics carry different scopes so that
// they stay an LDS atomic and a global atomic.
__device__ inline void tile_add(unsigned long long *tile, unsigned long long *glob, bool in, int lidx,
                                int64_t gidx, int64_t val)
{
    if (val == 0) return;
    if (in)
        __hip_atomic_fetch_add(&tile[lidx], (unsigned long long)val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        __hip_atomic_fetch_add(&glob[gidx], (unsigned long long)val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup per brick, granules taken in batches.  Phase 1 (a thread per
// granule) stores the stencil base, the offsets f of the 1-D weights and the
// scaled totals S of each channel in LDS.  Consecutive sorted granules with
// the same stencil base form a run; they share all 27 nodes.  Phase 2 (a
// thread per run and channel) walks the run's granules, rounds each outer
// contribution w S (once, from the exact product: one fused multiply-add)
// and sums it in one of 26 register accumulators; the
// centre node gets the run's sum of Q = rint(S) minus the 26 sums, which is
// the sum over the run's granules of each granule's centre remainder (all
// integer, so the regrouping is exact).  A run then costs 27 LDS atomics per
// channel, not 27 per granule.
//
// INTEG: the move of Sec. 4 is applied first, in place (x, v advanced with
// the contact and drag forces Fc, Fd, as the integration kernel does), and
// the granule is deposited at its new position; each granule is read and
// written by one thread only.
//
// EXCH: the exchange deposit of a sub-step (Sec. 5.2) instead of alpha and
// momentum: three channels, S_c = (exsc f_c) 2^32 with f the whole fluid
// force on the granule (Fd, plus the virtual-mass part -(rho_f V / 2) a_s
// with a_s = ((Fc + Fd) + m g) / (m + rho_f V / 2)), exsc = -weight / f_unit,
// deposited at the granule's current position; alpha receives channel 0 and
// mom channels 1 and 2.  With held (not NULL) m and V are the wet mass and
// volume (Sec. 5.3).
//
// WET: granules hold water (held, per unit of their volume): the move takes
// the wet mass of Eq. 19 (and the wet volume in the virtual mass), alpha
// receives frac (1 + held) and momentum the wet mass's (Sec. 5.3).
// NT: threads per workgroup (128 serves beds whose bricks hold few granules).
template <bool MOM, typename T, bool INTEG, bool EXCH = false, bool WET = false, bool STORE = false,
          int NT = kP2GThreads>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_p2g_fixed(DevParams P, int64_t n, const int32_t *__restrict__ bl,
                                                           const int32_t *__restrict__ bcnt, int batch,
                                                           double *x, double *v, const double *__restrict__ r,
                                                           const T *__restrict__ Fc, const T *__restrict__ Fd,
                                                           const int32_t *__restrict__ cb,
                                                           const int32_t *__restrict__ ce,
                                                           unsigned long long *__restrict__ alpha,
                                                           unsigned long long *__restrict__ mom, int64_t *err,
                                                           double exsc, const double *__restrict__ held,
                                                           P2GStore st)
{
#pragma clang fp contract(off)
    static_assert(!(EXCH && (MOM || INTEG)), "the exchange deposit is a kind of its own");
    static_assert(!STORE || (MOM && !EXCH && !WET), "the stored tiles serve the dry alpha and momentum deposit");
    constexpr int NCH = EXCH ? 3 : (MOM ? 4 : 1);
    extern __shared__ unsigned long long tile[];
    __shared__ int32_t s_range[2];
    __shared__ int32_t s_wave[NT / 64];
    int64_t slot;
    if (STORE && st.nclr && blockIdx.x == 0 && threadIdx.x < kRecSlots) st.nclr[threadIdx.x] = 0;  // the next call's record
    const int64_t b = brick_slot_of_block(bl, bcnt, slot);
    if (b < 0) return;
    brick_range(n, b, cb, ce, s_range);
    __syncthreads();
    const int32_t beg = s_range[0], end = s_range[1];
    if (STORE && st.nrec && threadIdx.x == 0) st.nrec[record_flag(end - beg)] = 1;  // the brick's granules
    if (end <= beg && !STORE) return;  // (a stored tile is written even if empty)
    const int E = P.tile;
    const int E3 = E * E * E;
    const int bs = batch + 1;  // padded stride: the arrays start on different LDS banks
    double *sf = reinterpret_cast<double *>(tile + NCH * E3);   // [3][bs] weight offsets f
    double *sS = sf + 3 * bs;                                    // [NCH][bs] scaled totals
    int32_t *srun = reinterpret_cast<int32_t *>(sS + NCH * bs);   // [bs] run starts
    int16_t *sbase = reinterpret_cast<int16_t *>(srun + bs);      // [3][bs] stencil base (grid edges < 2^15 nodes)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < NCH * E3; k += NT) tile[k] = 0ull;
    int32_t o[3];
    tile_origin(P, b, o);
    // grid plane of channel c (computed, not an array indexed by c, which
    // would live in scratch memory): alpha, then the momentum (or exchange)
    // planes that follow mom
    auto glob_of = [&](int c) { return c == 0 ? alpha : mom + (int64_t)(c - 1) * P.G; };
    for (int64_t b0 = beg; b0 < end; b0 += batch) {
        const int m = (int)(end - b0 < batch ? end - b0 : batch);
        // ---- phase 1: per granule
        for (int i = tid; i < m; i += NT) {
            const int64_t q = b0 + i;
            double xa[3] = {x[q], x[n + q], x[2 * n + q]};
            double va[3] = {0.0, 0.0, 0.0};
            if (MOM || INTEG)
                for (int a = 0; a < 3; ++a) va[a] = v[a * n + q];
            if (INTEG) {
                const T fc[3] = {Fc[q], Fc[n + q], Fc[2 * n + q]};
                const T fd[3] = {Fd[q], Fd[n + q], Fd[2 * n + q]};
                if (WET)
                    integrate_one_m<T>(P, wet_volume(r[q], held[q]), wet_mass(P, r[q], held[q]), fc, fd, xa, va);
                else
                    integrate_one<T>(P, r[q], fc, fd, xa, va);
                for (int a = 0; a < 3; ++a) {
                    x[a * n + q] = xa[a];
                    v[a * n + q] = va[a];
                }
            }
            bool inside = true;  // all 27 stencil nodes (folded onto the edge) in the tile
            for (int a = 0; a < 3; ++a) {
                const double t = xa[a] * P.inv_dx;
                double fb = floor(t - 1.0);
                sf[a * bs + i] = (t - fb) - 0.5;
                if (!(fb >= -2.0)) fb = -2.0;
                if (fb > (double)P.n[a]) fb = (double)P.n[a];
                sbase[a * bs + i] = (int16_t)fb;
                if (STORE) {
                    const int32_t lo = (int32_t)fb < 0 ? 0 : (int32_t)fb;
                    const int32_t hi = (int32_t)fb + 2 > P.n[a] - 1 ? P.n[a] - 1 : (int32_t)fb + 2;
                    inside &= lo - o[a] >= 0 && hi - o[a] < E;
                }
            }
            if (STORE && !inside) {
                // deposited after the assembly (k_p2g_escapes); a run of zeros here
                const uint32_t k = atomicAdd(st.esc_n, 1u);
                if (k < (uint32_t)n) st.esc[k] = (int32_t)q;
                for (int a = 0; a < 3; ++a) sbase[a * bs + i] = (int16_t)(o[a] + 1);
            }
            double S[NCH];
            if constexpr (EXCH) {
                // wet granules (held given): the wet mass of Eq. 19 and the
                // volume with the held water (Sec. 5.3)
                const double rq = r[q];
                const double hq = held ? held[q] : 0.0;
                const double m = held ? wet_mass(P, rq, hq) : mass_of(P, rq);
                const double hv = P.half_rho_f * wet_volume(rq, hq);
                const double me = m + hv;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double f = (double)Fd[c * n + q];
                    if (P.vmass) {
                        const double as = (((double)Fc[c * n + q] + f) + m * P.g[c]) / me;
                        f = f - hv * as;
                    }
                    S[c] = (exsc * f) * GIC_TWO32;
                }
            } else {
                const double frac = volume_of(r[q]) * P.inv_vcell;
                // a wet granule's held water counts as volume in alpha_s
                // (Sec. 5.3): frac (1 + held), frac exactly when held = 0
                S[0] = (WET ? frac + frac * held[q] : frac) * GIC_TWO32;
                // momentum in rho_s dx^3 units: a wet granule (Eq. 19) carries
                // frac (rho_s + held rho_f) / rho_s = frac + frac held rho_f / rho_s
                // per unit velocity (held = 0 gives frac exactly)
                const double fm = WET ? frac + (frac * (held[q] * P.rho_f)) / P.rho_s : frac;
                if (MOM)
#pragma unroll
                    for (int c = 1; c < NCH; ++c) S[c] = (fm * va[c - 1]) * GIC_TWO32;
            }
            bool ok = true;
#pragma unroll
            for (int c = 0; c < NCH; ++c) ok &= fabs(S[c]) < kFixLimit;
            if (!ok) {
                double sum = 0.0;
#pragma unroll
                for (int c = 0; c < NCH; ++c) sum += S[c];
                raise_error(err, isfinite(sum) ? kErrRange : kErrNonFinite, q);
#pragma unroll
                for (int c = 0; c < NCH; ++c) S[c] = 0.0;
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) sS[c * bs + i] = STORE && !inside ? 0.0 : S[c];
        }
        __syncthreads();
        // ---- runs of equal stencil base
        int nruns = 0;
        for (int i0 = 0; i0 < m; i0 += NT) {
            const int i = i0 + tid;
            bool start = false;
            if (i < m) {
                start = i == 0;
                if (!start)
                    for (int a = 0; a < 3; ++a) start |= sbase[a * bs + i - 1] != sbase[a * bs + i];
            }
            const uint64_t smask = __ballot(start);
            if (lane == 0) s_wave[wave] = (int32_t)__popcll(smask);
            __syncthreads();
            int off = nruns, tot = nruns;
            for (int w = 0; w < NT / 64; ++w) {
                off += w < wave ? s_wave[w] : 0;
                tot += s_wave[w];
            }
            if (start) {
                const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
                srun[off + __popcll(smask & lt)] = i;
            }
            nruns = tot;
            __syncthreads();
        }
        if (tid == 0) srun[nruns] = m;
        __syncthreads();
        // ---- phase 2: per run and channel
        for (int task = tid; task < nruns * NCH; task += NT) {
            const int rr = task / NCH;
            const int c = task - rr * NCH;
            const int g0 = srun[rr], g1 = srun[rr + 1];
            // sums of rint_biased patterns (mod 2^64), started at minus the
            // run's bias so that they end as sums of rint values
            const uint64_t nbias = 0ull - (uint64_t)(g1 - g0) * kRintBias;
            uint64_t acc[27];
#pragma unroll
            for (int k = 0; k < 27; ++k) acc[k] = nbias;
            uint64_t qsum = nbias;
            for (int g = g0; g < g1; ++g) {
                const double S = sS[c * bs + g];
                double w[3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double f = sf[a * bs + g];
                    const double c0 = 1.5 - f, c1 = f - 1.0, c2 = f - 0.5;
                    w[a][0] = 0.5 * (c0 * c0);
                    w[a][1] = 0.75 - c1 * c1;
                    w[a][2] = 0.5 * (c2 * c2);
                }
                qsum += rint_biased(S);
#pragma unroll
                for (int cz = 0; cz < 3; ++cz)
#pragma unroll
                    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
                        for (int cx = 0; cx < 3; ++cx) {
                            if (cx == 1 && cy == 1 && cz == 1) continue;
                            const double ww = (w[0][cx] * w[1][cy]) * w[2][cz];
                            acc[(cz * 3 + cy) * 3 + cx] += rint_product_biased(ww, S);
                        }
            }
            uint64_t outer = 0;
#pragma unroll
            for (int k = 0; k < 27; ++k)
                if (k != 13) outer += acc[k];
            acc[13] = qsum - outer;
            // nodes of the run's stencil, folded onto the edge
            int32_t nd[3][3];
            bool inb[3][3];
            for (int a = 0; a < 3; ++a) {
                const int32_t b0a = sbase[a * bs + g0];
                for (int k = 0; k < 3; ++k) {
                    int32_t id = b0a + k;
                    id = id < 0 ? 0 : id;
                    id = id > P.n[a] - 1 ? P.n[a] - 1 : id;
                    nd[a][k] = id;
                    const int32_t l = id - o[a];
                    inb[a][k] = l >= 0 && l < E;
                }
            }
            unsigned long long *tl = tile + c * E3;
            if (STORE) {  // every node in the tile (phase 1 set aside the granules that were not)
#pragma unroll
                for (int cz = 0; cz < 3; ++cz)
#pragma unroll
                    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
                        for (int cx = 0; cx < 3; ++cx)
                            __hip_atomic_fetch_add(
                                &tl[((nd[2][cz] - o[2]) * E + (nd[1][cy] - o[1])) * E + (nd[0][cx] - o[0])],
                                (unsigned long long)acc[(cz * 3 + cy) * 3 + cx], __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
#pragma unroll
                for (int cz = 0; cz < 3; ++cz)
#pragma unroll
                    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
                        for (int cx = 0; cx < 3; ++cx) {
                            const bool in = inb[0][cx] && inb[1][cy] && inb[2][cz];
                            const int lidx =
                                ((nd[2][cz] - o[2]) * E + (nd[1][cy] - o[1])) * E + (nd[0][cx] - o[0]);
                            const int64_t gidx = node_index(P, nd[0][cx], nd[1][cy], nd[2][cz]);
                            tile_add(tl, glob_of(c), in, lidx, gidx, (int64_t)acc[(cz * 3 + cy) * 3 + cx]);
                        }
            }
        }
        __syncthreads();
    }
    if (STORE) {  // the whole tile, for k_p2g_assemble
        unsigned long long *dst = st.tiles + slot * (int64_t)(NCH * E3);
        for (int k = tid; k < NCH * E3; k += NT) dst[k] = tile[k];
        return;
    }
    for (int k = tid; k < NCH * E3; k += NT) {
        const unsigned long long val = tile[k];
        if (val == 0ull) continue;
        const int c = k / E3;
        const int l = k - c * E3;
        const int32_t ni = o[0] + l % E, nj = o[1] + (l / E) % E, nk = o[2] + l / (E * E);
        atomicAdd(&glob_of(c)[node_index(P, ni, nj, nk)], val);
    }
}

// Grid of the stored tiles (P2G in STORE mode): every node's alpha and
// momentum is the sum of the tile entries of the occupied bricks whose tile
// holds it (at most two bricks per axis, from the cover table), written
// once, so the grids need no clearing and see no global atomics.  Nodes that
// no occupied brick's tile holds get zero.  A workgroup takes x-rows of
// nodes: the y and z bricks of a row are the same for all its threads.
// With live flags (4-node segments of a row) and !full, a segment that no
// tile holds now and that was not live holds zeros from an earlier
// assembly and is left as it is: a bed that fills part of the box writes
// its own region (and the region it left) instead of the whole grids.
// (Giving each XCD a contiguous eighth of the rows, so that the rows reading
// one tile share an L2, was slower: a bed fills part of the box, so most
// tile reads then fell to a few XCDs.)
constexpr int kAsmRows = 4;  // node rows per workgroup pass, one per wave

__global__ void __launch_bounds__(256) k_p2g_assemble(DevParams P, const unsigned long long *__restrict__ tiles,
                                                      const int32_t *__restrict__ slot_of,
                                                      const int32_t *__restrict__ cover,
                                                      unsigned long long *__restrict__ alpha,
                                                      unsigned long long *__restrict__ mom,
                                                      uint8_t *__restrict__ live, int full)
{
    extern __shared__ int32_t s_slot[];  // [kAsmRows][4][nb0]: slots of each row's (z, y) brick pairs along x
    __shared__ int32_t s_any[kAsmRows];
    const int E = P.tile, E3 = E * E * E;
    const int64_t G = P.G;
    const int64_t rows = (int64_t)P.n[1] * P.n[2];
    const int32_t *cx = cover, *cy = cover + 4 * P.n[0], *cz = cover + 4 * (P.n[0] + P.n[1]);
    const int32_t nbx = P.nb[0];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t r0 = (int64_t)blockIdx.x * kAsmRows; r0 < rows; r0 += (int64_t)gridDim.x * kAsmRows) {
        // the brick slots of the pass's rows into LDS (all loads in flight
        // together), and whether any is occupied
        if (threadIdx.x < kAsmRows) s_any[threadIdx.x] = 0;
        __syncthreads();
        for (int t = threadIdx.x; t < kAsmRows * 4 * nbx; t += 256) {
            const int rr = t / (4 * nbx), rem = t - rr * (4 * nbx);
            const int p = rem / nbx, bx = rem - p * nbx;
            const int64_t row = r0 + rr;
            int32_t sl = -1;
            if (row < rows) {
                const int32_t j = (int32_t)(row % P.n[1]), k = (int32_t)(row / P.n[1]);
                const int32_t by = cy[4 * j + 2 * (p & 1)], bz = cz[4 * k + 2 * (p >> 1)];
                if (bz >= 0 && by >= 0) sl = slot_of[((int64_t)bz * P.nb[1] + by) * nbx + bx];
            }
            s_slot[t] = sl;
            if (sl >= 0) s_any[rr] = 1;
        }
        __syncthreads();
        const int64_t row = r0 + wave;  // each wave writes one row
        if (row < rows) {
            const int32_t j = (int32_t)(row % P.n[1]), k = (int32_t)(row / P.n[1]);
            const int32_t ly[2] = {cy[4 * j + 1], cy[4 * j + 3]};
            const int32_t lz[2] = {cz[4 * k + 1], cz[4 * k + 3]};
            const int occupied = s_any[wave];
            const int32_t *rs = s_slot + wave * 4 * nbx;
            uint8_t *lrow = live ? live + row * ((P.n[0] + 3) >> 2) : nullptr;
            for (int32_t i = lane; i < P.n[0]; i += 64) {
                unsigned long long s0 = 0, s1 = 0, s2 = 0, s3 = 0;
                bool has = false;  // a tile holds the node
                if (occupied) {
                    const int32_t bx[2] = {cx[4 * i], cx[4 * i + 2]}, lx[2] = {cx[4 * i + 1], cx[4 * i + 3]};
                    for (int p = 0; p < 4; ++p) {
                        const int off_yz = (lz[p >> 1] * E + ly[p & 1]) * E;
                        for (int ix = 0; ix < 2; ++ix) {
                            if (bx[ix] < 0) continue;
                            const int32_t sl = rs[p * nbx + bx[ix]];
                            if (sl < 0) continue;
                            has = true;
                            const unsigned long long *t = tiles + (int64_t)sl * (4 * E3) + off_yz + lx[ix];
                            s0 += t[0];
                            s1 += t[E3];
                            s2 += t[2 * E3];
                            s3 += t[3 * E3];
                        }
                    }
                }
                bool put = true;
                if (lrow) {
                    // segment i / 4 (lanes 4 (lane / 4) .. + 3 of this round):
                    // written when a tile holds one of its nodes now or when
                    // it was live; its flag becomes the former
                    const bool now = ((__ballot(has) >> (lane & ~3)) & 0xFull) != 0ull;
                    const uint8_t was = lrow[i >> 2];
                    put = full || now || was != 0;
                    if ((lane & 3) == 0 && was != (uint8_t)now) lrow[i >> 2] = (uint8_t)now;
                }
                if (put) {
                    const int64_t idx = row * P.n[0] + i;
                    alpha[idx] = s0;
                    mom[idx] = s1;
                    mom[G + idx] = s2;
                    mom[2 * G + idx] = s3;
                }
            }
        }
        __syncthreads();  // s_slot and s_any are rewritten by the next pass
    }
}

// The granules whose stencil left their brick's tile (listed by the P2G in
// STORE mode): each deposited straight to the assembled grids with the
// rounding of the tile path, w S rounded once on the 26 outer nodes and rint(S)
// minus their sum on the centre.  Also clears the other list counter, the
// one the next step's P2G appends to.
__global__ void __launch_bounds__(256) k_p2g_escapes(DevParams P, int64_t n, const int32_t *__restrict__ esc,
                                                     const uint32_t *__restrict__ esc_n, uint32_t *__restrict__ next_n,
                                                     const double *__restrict__ x, const double *__restrict__ v,
                                                     const double *__restrict__ r,
                                                     unsigned long long *__restrict__ alpha,
                                                     unsigned long long *__restrict__ mom,
                                                     uint8_t *__restrict__ live, int64_t *err)
{
#pragma clang fp contract(off)
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_n = 0u;
    const uint32_t cnt = *esc_n < (uint32_t)n ? *esc_n : (uint32_t)n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
        const int64_t q = esc[e];
        if ((uint64_t)q >= (uint64_t)n) continue;
        double w[3][3];
        int32_t nd[3][3];
        for (int a = 0; a < 3; ++a) {
            const double t = x[a * n + q] * P.inv_dx;
            double fb = floor(t - 1.0);
            const double f = (t - fb) - 0.5;
            if (!(fb >= -2.0)) fb = -2.0;
            if (fb > (double)P.n[a]) fb = (double)P.n[a];
            const double c0 = 1.5 - f, c1 = f - 1.0, c2 = f - 0.5;
            w[a][0] = 0.5 * (c0 * c0);
            w[a][1] = 0.75 - c1 * c1;
            w[a][2] = 0.5 * (c2 * c2);
            for (int k = 0; k < 3; ++k) {
                int32_t id = (int32_t)fb + k;
                id = id < 0 ? 0 : id;
                id = id > P.n[a] - 1 ? P.n[a] - 1 : id;
                nd[a][k] = id;
            }
        }
        const double frac = volume_of(r[q]) * P.inv_vcell;
        double S[4] = {frac * GIC_TWO32, 0.0, 0.0, 0.0};
        for (int c = 1; c < 4; ++c) S[c] = (frac * v[(c - 1) * n + q]) * GIC_TWO32;
        bool ok = true;
        for (int c = 0; c < 4; ++c) ok &= fabs(S[c]) < kFixLimit;
        if (!ok) {
            const double sum = ((S[0] + S[1]) + S[2]) + S[3];
            raise_error(err, isfinite(sum) ? kErrRange : kErrNonFinite, q);
            continue;
        }
        if (live) {  // the segments of the stencil's nodes are live from now on
            const int64_t nseg = (P.n[0] + 3) >> 2;
            for (int cz = 0; cz < 3; ++cz)
                for (int cy = 0; cy < 3; ++cy) {
                    uint8_t *lr = live + ((int64_t)nd[2][cz] * P.n[1] + nd[1][cy]) * nseg;
                    for (int cx = 0; cx < 3; ++cx) lr[nd[0][cx] >> 2] = 1;
                }
        }
        for (int c = 0; c < 4; ++c) {
            unsigned long long *g = c == 0 ? alpha : mom + (int64_t)(c - 1) * P.G;
            uint64_t outer = 0;
            for (int cz = 0; cz < 3; ++cz)
                for (int cy = 0; cy < 3; ++cy)
                    for (int cx = 0; cx < 3; ++cx) {
                        if (cx == 1 && cy == 1 && cz == 1) continue;
                        const uint64_t val =
                            rint_product_biased((w[0][cx] * w[1][cy]) * w[2][cz], S[c]) - kRintBias;
                        outer += val;
                        if (val) atomicAdd(&g[node_index(P, nd[0][cx], nd[1][cy], nd[2][cz])], val);
                    }
            const uint64_t centre = (rint_biased(S[c]) - kRintBias) - outer;
            if (centre) atomicAdd(&g[node_index(P, nd[0][1], nd[1][1], nd[2][1])], centre);
        }
    }
}

// Unquantised P2G of the differentiable form, deterministic: every
// contribution c of channel ch is rounded to the integer
// rint(c 2^(50 - e_ch)), 2^e_ch the power of two at or above the largest
// contribution bound of the channel in this call (frac_i for alpha,
// |m_i v_i,a| for momentum), and the integers are summed in LDS and grid
// atomics, exactly and in any order; k_fix_finish scales the sums back.  A
// contribution is then off by at most 2^(e_ch - 51), the rounding of one
// double addition at that magnitude, and a node's sum holds while fewer than
// 2^12 granules reach it (|sum| < 2^62).
constexpr int kFixParts = 1024;  // partial maxima per channel

// Clears len int64 of fx and writes each workgroup's largest per-granule
// bound of each channel to part[ch * kFixParts + block]: frac, |m v_x|,
// |m v_y|, |m v_z| (P2G) or |gaf| (the G2P pullback, gaf given).
__global__ void __launch_bounds__(256) k_fix_prep(DevParams P, int64_t n, int64_t per, const double *__restrict__ v,
                                                  const double *__restrict__ r, const double *__restrict__ gaf,
                                                  int64_t *__restrict__ fx, int64_t len, double *__restrict__ part)
{
    __shared__ double wm[4][4];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) fx[i] = 0;
    const int nch = gaf ? 1 : 4;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    for (int64_t q = lo + threadIdx.x; q < hi; q += 256) {
        if (gaf) {
            m[0] = fmax(m[0], fabs(gaf[q]));
        } else {
            const double rq = r[q];
            m[0] = fmax(m[0], volume_of(rq) * P.inv_vcell);
            const double mq = mass_of(P, rq);
            for (int c = 0; c < 3; ++c) m[c + 1] = fmax(m[c + 1], fabs(mq * v[c * n + q]));
        }
    }
    for (int c = 0; c < nch; ++c) {
        double t = m[c];
        for (int off = 32; off > 0; off >>= 1) t = fmax(t, __shfl_xor(t, off));
        if ((threadIdx.x & 63) == 0) wm[c][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < nch)
        part[threadIdx.x * kFixParts + blockIdx.x] =
            fmax(fmax(wm[threadIdx.x][0], wm[threadIdx.x][1]), fmax(wm[threadIdx.x][2], wm[threadIdx.x][3]));
}

// The scales of a call, after its nb partial maxima per channel:
// part[kFixScale + c] = 2^(50 - e), 2^e the power of two above channel c's
// largest bound (1 when all are zero), so contributions times it stay below
// 2^50; part[kFixScale + 4 + c] = its inverse.  One workgroup, once per call.
constexpr int kFixScale = 4 * kFixParts;

__global__ void __launch_bounds__(256) k_fix_scale(double *__restrict__ part, int nb, int nch)
{
    __shared__ double wm[4];
    for (int c = 0; c < nch; ++c) {
        double M = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) M = fmax(M, part[c * kFixParts + b]);
        for (int off = 32; off > 0; off >>= 1) M = fmax(M, __shfl_xor(M, off));
        if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = M;
        __syncthreads();
        if (threadIdx.x == 0) {
            M = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
            double sc = 1.0;
            if (M > 0.0) {
                int e;
                (void)frexp(M, &e);  // M = f 2^e, f in [0.5, 1)
                sc = ldexp(1.0, 50 - e);
            }
            part[kFixScale + c] = sc;
            part[kFixScale + 4 + c] = 1.0 / sc;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kP2GThreads) k_p2g_real(DevParams P, int64_t n, const int32_t *__restrict__ bl,
                                                          const int32_t *__restrict__ bcnt,
                                                          const double *__restrict__ x,
                                                          const double *__restrict__ v,
                                                          const double *__restrict__ r,
                                                          const int32_t *__restrict__ cb,
                                                          const int32_t *__restrict__ ce,
                                                          const double *__restrict__ part, int nch,
                                                          unsigned long long *__restrict__ fx)
{
    extern __shared__ unsigned long long itile[];
    __shared__ int32_t s_range[2];
    const int64_t b = brick_of_block(bl, bcnt);
    if (b < 0) return;
    brick_range(n, b, cb, ce, s_range);
    const int E = P.tile;
    const int E3 = E * E * E;
    for (int k = threadIdx.x; k < nch * E3; k += kP2GThreads) itile[k] = 0ull;
    __syncthreads();
    const int32_t beg = s_range[0], end = s_range[1];
    if (end <= beg) return;
    double sc[4];
    for (int c = 0; c < nch; ++c) sc[c] = part[kFixScale + c];
    int32_t o[3];
    tile_origin(P, b, o);
    const int64_t G = P.G;
    for (int64_t q = beg + (int64_t)threadIdx.x; q < end; q += kP2GThreads) {
        const double xa[3] = {x[q], x[n + q], x[2 * n + q]};
        Stencil s;
        stencil_of(P, xa, s);
        const double m = mass_of(P, r[q]);
        double S[4] = {volume_of(r[q]) * P.inv_vcell, 0.0, 0.0, 0.0};
        if (nch > 1)
            for (int c = 0; c < 3; ++c) S[c + 1] = m * v[c * n + q];
        for (int cz = 0; cz < 3; ++cz)
            for (int cy = 0; cy < 3; ++cy)
                for (int cx = 0; cx < 3; ++cx) {
                    const double w = (s.w[0][cx] * s.w[1][cy]) * s.w[2][cz];
                    const int32_t ni = s.node[0][cx], nj = s.node[1][cy], nk = s.node[2][cz];
                    const int32_t li = ni - o[0], lj = nj - o[1], lk = nk - o[2];
                    const bool in = li >= 0 && lj >= 0 && lk >= 0 && li < E && lj < E && lk < E;
                    const int lidx = (lk * E + lj) * E + li;
                    const int64_t gidx = node_index(P, ni, nj, nk);
                    for (int c = 0; c < nch; ++c)
                        tile_add(itile + c * E3, fx + c * G, in, lidx, gidx, rint_i64((w * S[c]) * sc[c]));
                }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nch * E3; k += kP2GThreads) {
        const unsigned long long val = itile[k];
        if (val == 0ull) continue;
        const int c = k / E3;
        const int l = k - c * E3;
        const int32_t ni = o[0] + l % E, nj = o[1] + (l / E) % E, nk = o[2] + l / (E * E);
        atomicAdd(&fx[c * G + node_index(P, ni, nj, nk)], val);
    }
}

// out[c] (= or +=) the integer sums of channel c scaled back: fx / scale_c.
__global__ void __launch_bounds__(256) k_fix_finish(int64_t G, int nch, const double *__restrict__ part,
                                                    const int64_t *__restrict__ fx, double *__restrict__ out0,
                                                    double *__restrict__ out1, int acc)
{
    __shared__ double inv[4];
    if (threadIdx.x < nch) inv[threadIdx.x] = part[kFixScale + 4 + threadIdx.x];
    __syncthreads();
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nch * G; k += (int64_t)gridDim.x * 256) {
        const int c = (int)(k / G);
        double *o = c == 0 ? (out0 ? out0 + k : nullptr) : (out1 ? out1 + (k - G) : nullptr);
        if (!o) continue;
        const double val = (double)fx[k] * inv[c];
        *o = acc ? *o + val : val;
    }
}

template <typename T, bool FIXED>
__global__ void __launch_bounds__(256) k_g2p(DevParams P, int64_t n, int64_t nblk, const double *__restrict__ x,
                                             const T *__restrict__ u, const int64_t *__restrict__ afx,
                                             const double *__restrict__ are, T *__restrict__ uat,
                                             T *__restrict__ af)
{
    const int64_t lb = xcd_block(nblk);
    if (lb < 0) return;
    const int64_t q = lb * 256 + threadIdx.x;
    if (q >= n) return;
    const double xa[3] = {x[q], x[n + q], x[2 * n + q]};
    const int64_t G = P.G;
    T ua[3], a;
    g2p_sample<T>(P, xa, [&](int32_t i, int32_t j, int32_t k, T uu[3], T &al) {
        const int64_t idx = node_index(P, i, j, k);
        uu[0] = u[idx];
        uu[1] = u[G + idx];
        uu[2] = u[2 * G + idx];
        al = (T)(FIXED ? node_alpha(P, afx[idx]) : node_alpha_real(P, are[idx]));
    }, ua, a);
    uat[q] = ua[0];
    uat[n + q] = ua[1];
    uat[2 * n + q] = ua[2];
    af[q] = a;
}

}  // namespace

hipError_t launch_fill_i64(int64_t *a, int64_t len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    unsigned g = grid_for(len, 256);
    if (g > 65536) g = 65536;
    k_fill_i64<<<g, 256, 0, s>>>(a, len);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *a, int64_t len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    unsigned g = grid_for(len, 256);
    if (g > 65536) g = 65536;
    k_fill_f64<<<g, 256, 0, s>>>(a, len);
    return hipGetLastError();
}

// LDS bytes of the fixed-point P2G: node tile plus per-granule batch data.
static size_t p2g_lds(int nch, int E3, int batch)
{
    return sizeof(unsigned long long) * (size_t)nch * E3 + (size_t)(batch + 1) * (3 * 8 + nch * 8 + 4 + 3 * 2);
}

template <typename T, bool INTEG, bool WET = false>
static hipError_t p2g_fixed_impl(const DevParams &P, int64_t n, int64_t K, double *x, double *v, const double *r,
                                 const T *Fc, const T *Fd, const int32_t *cb, const int32_t *ce, const BrickList &B,
                                 int64_t *alpha, int64_t *mom, int64_t *err, hipStream_t s,
                                 const double *held = nullptr)
{
    if (n == 0) return hipSuccess;
    const int64_t bricks = K / kBrickCells;
    const int E3 = P.tile * P.tile * P.tile;
    const int nch = mom ? 4 : 1;
    int batch = 512;  // a brick of 64 cells of 8 granules in one batch; 256 run-channel tasks
    while (batch > 64 && p2g_lds(nch, E3, batch) > 49152) batch /= 2;
    const size_t lds = p2g_lds(nch, E3, batch);
    unsigned long long *A = reinterpret_cast<unsigned long long *>(alpha);
    unsigned long long *M = reinterpret_cast<unsigned long long *>(mom);
    if (mom)
        k_p2g_fixed<true, T, INTEG, false, WET><<<brick_grid(bricks), kP2GThreads, lds, s>>>(
            P, n, B.list, B.count, batch, x, v, r, Fc, Fd, cb, ce, A, M, err, 0.0, held, P2GStore{});
    else
        k_p2g_fixed<false, T, INTEG, false, WET><<<brick_grid(bricks), kP2GThreads, lds, s>>>(
            P, n, B.list, B.count, batch, x, v, r, Fc, Fd, cb, ce, A, nullptr, err, 0.0, held, P2GStore{});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_exchange_p2g(const DevParams &P, int64_t n, int64_t K, const double *x, const double *r,
                               const T *Fc, const T *Ffl, const int32_t *cb, const int32_t *ce, const BrickList &B,
                               double exsc, int64_t *fs, int64_t *err, hipStream_t s, const double *held)
{
    if (n == 0) return hipSuccess;
    const int64_t bricks = K / kBrickCells;
    const int E3 = P.tile * P.tile * P.tile;
    int batch = 512;
    while (batch > 64 && p2g_lds(3, E3, batch) > 49152) batch /= 2;
    const size_t lds = p2g_lds(3, E3, batch);
    unsigned long long *F = reinterpret_cast<unsigned long long *>(fs);
    // x is only read on this path
    k_p2g_fixed<false, T, false, true><<<brick_grid(bricks), kP2GThreads, lds, s>>>(
        P, n, B.list, B.count, batch, const_cast<double *>(x), nullptr, r, Fc, Ffl, cb, ce, F, F + P.G, err, exsc,
        held, P2GStore{});
    return hipGetLastError();
}

template hipError_t launch_exchange_p2g<float>(const DevParams &, int64_t, int64_t, const double *, const double *,
                                               const float *, const float *, const int32_t *, const int32_t *,
                                               const BrickList &, double, int64_t *, int64_t *, hipStream_t,
                                               const double *);
template hipError_t launch_exchange_p2g<double>(const DevParams &, int64_t, int64_t, const double *,
                                                const double *, const double *, const double *, const int32_t *,
                                                const int32_t *, const BrickList &, double, int64_t *, int64_t *,
                                                hipStream_t, const double *);

hipError_t launch_p2g_fixed(const DevParams &P, int64_t n, int64_t K, const double *x, const double *v,
                            const double *r, const int32_t *cb, const int32_t *ce, const BrickList &B,
                            int64_t *alpha, int64_t *mom, int64_t *err, hipStream_t s)
{
    // x and v are only read on this path
    return p2g_fixed_impl<float, false>(P, n, K, const_cast<double *>(x), const_cast<double *>(v), r, nullptr,
                                        nullptr, cb, ce, B, alpha, mom, err, s);
}

template <typename T>
hipError_t launch_integrate_p2g(const DevParams &P, int64_t n, int64_t K, double *x, double *v, const double *r,
                                const T *Fc, const T *Fd, const int32_t *cb, const int32_t *ce, const BrickList &B,
                                int64_t *alpha, int64_t *mom, int64_t *err, hipStream_t s, const double *held)
{
    if (held)
        return p2g_fixed_impl<T, true, true>(P, n, K, x, v, r, Fc, Fd, cb, ce, B, alpha, mom, err, s, held);
    return p2g_fixed_impl<T, true>(P, n, K, x, v, r, Fc, Fd, cb, ce, B, alpha, mom, err, s);
}

template <typename T>
hipError_t launch_integrate_p2g_store(const DevParams &P, int64_t n, int64_t K, double *x, double *v,
                                      const double *r, const T *Fc, const T *Fd, const int32_t *cb,
                                      const int32_t *ce, const BrickList &B, int64_t *err, hipStream_t s,
                                      const P2GStore &st, SizeRecord *rec)
{
    const int64_t bricks = K / kBrickCells;
    const int E3 = P.tile * P.tile * P.tile;
    int batch = 512;
    while (batch > 64 && p2g_lds(4, E3, batch) > 49152) batch /= 2;
    // bricks of at most 128 granules at the last record: workgroups of 128
    // threads and batches of 128 (less LDS, twice the workgroups per CU); a
    // denser brick loops over batches, and the calls after take 256
    const int32_t seen = record_seen(rec);
    const bool small = seen > 0 && seen <= 128 && batch >= 128;
    if (small) batch = 128;
    const size_t lds = p2g_lds(4, E3, batch);
    P2GStore sr = st;
    const bool copy = n > 0 && record_copy(rec);  // only these calls record (the stores contend)
    sr.nrec = copy ? rec->dev + rec->par * kRecSlots : nullptr;
    sr.nclr = copy ? rec->dev + (rec->par ^ 1) * kRecSlots : nullptr;
    if (n > 0 && small)
        k_p2g_fixed<true, T, true, false, false, true, 128><<<brick_grid(bricks), 128, lds, s>>>(
            P, n, B.list, B.count, batch, x, v, r, Fc, Fd, cb, ce, nullptr, nullptr, err, 0.0, nullptr, sr);
    else if (n > 0)
        k_p2g_fixed<true, T, true, false, false, true><<<brick_grid(bricks), kP2GThreads, lds, s>>>(
            P, n, B.list, B.count, batch, x, v, r, Fc, Fd, cb, ce, nullptr, nullptr, err, 0.0, nullptr, sr);
    hipError_t e = hipGetLastError();
    if (copy) {
        rec->par ^= 1;
        if (e == hipSuccess) e = hipMemcpyAsync(rec->host, sr.nrec, sizeof(int32_t) * kRecSlots, hipMemcpyDeviceToHost, s);
    }
    return e;
}

template hipError_t launch_integrate_p2g_store<float>(const DevParams &, int64_t, int64_t, double *, double *,
                                                      const double *, const float *, const float *,
                                                      const int32_t *, const int32_t *, const BrickList &,
                                                      int64_t *, hipStream_t, const P2GStore &, SizeRecord *);
template hipError_t launch_integrate_p2g_store<double>(const DevParams &, int64_t, int64_t, double *, double *,
                                                       const double *, const double *, const double *,
                                                       const int32_t *, const int32_t *, const BrickList &,
                                                       int64_t *, hipStream_t, const P2GStore &, SizeRecord *);

hipError_t launch_p2g_assemble(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                               const BrickList &B, int64_t *alpha, int64_t *mom, int64_t *err, hipStream_t s,
                               const P2GStore &st, uint32_t *esc_next)
{
    unsigned long long *A = reinterpret_cast<unsigned long long *>(alpha);
    unsigned long long *M = reinterpret_cast<unsigned long long *>(mom);
    const int64_t passes = ((int64_t)P.n[1] * P.n[2] + kAsmRows - 1) / kAsmRows;
    k_p2g_assemble<<<(unsigned)(passes < 16384 ? passes : 16384), 256, sizeof(int32_t) * kAsmRows * 4 * P.nb[0],
                     s>>>(
        P, st.tiles, B.slot_of, st.cover, A, M, st.live, st.live ? st.full : 1);
    k_p2g_escapes<<<256, 256, 0, s>>>(P, n, st.esc, st.esc_n, esc_next, x, v, r, A, M, st.live, err);
    return hipGetLastError();
}

void p2g_cover_table(const DevParams &P, int32_t *out)
{
    int32_t *t = out;
    for (int a = 0; a < 3; ++a) {
        for (int32_t i = 0; i < P.n[a]; ++i, t += 4) {
            t[0] = t[1] = t[2] = t[3] = -1;
            int k = 0;
            // tiles start about 4 cell/dx apart and reach about one node past
            // their brick: the bricks near the node's own are the candidates
            const int32_t bc = (int32_t)floor((double)(i + 1) / ((double)kBrick * P.cell * P.inv_dx));
            const int32_t b0 = bc - 2 > 0 ? bc - 2 : 0;
            for (int32_t bx = b0; bx <= bc + 2 && bx < P.nb[a] && k < 2; ++bx) {
                // the tile origin of tile_origin
                const int32_t o = (int32_t)floor((double)(bx * kBrick) * P.cell * P.inv_dx + 1e-7) - 1;
                if (i >= o && i < o + P.tile) {
                    t[2 * k] = bx;
                    t[2 * k + 1] = i - o;
                    ++k;
                }
            }
        }
    }
}

template hipError_t launch_integrate_p2g<float>(const DevParams &, int64_t, int64_t, double *, double *,
                                                const double *, const float *, const float *, const int32_t *,
                                                const int32_t *, const BrickList &, int64_t *, int64_t *, int64_t *,
                                                hipStream_t, const double *);
template hipError_t launch_integrate_p2g<double>(const DevParams &, int64_t, int64_t, double *, double *,
                                                 const double *, const double *, const double *, const int32_t *,
                                                 const int32_t *, const BrickList &, int64_t *, int64_t *, int64_t *,
                                                 hipStream_t, const double *);

hipError_t launch_p2g_real(const DevParams &P, int64_t n, int64_t K, const double *x, const double *v,
                           const double *r, const int32_t *cb, const int32_t *ce, const BrickList &B,
                           double *alpha, double *mom, int acc, int64_t *fx, double *part, hipStream_t s)
{
    const int64_t G = P.G;
    const int nch = mom ? 4 : 1;  // alpha is computed with the momentum and written when asked for
    const int64_t per = n > 0 ? (n + kFixParts - 1) / kFixParts : 1;
    const int nb = (int)(n > 0 ? (n + per - 1) / per : 1);
    k_fix_prep<<<nb, 256, 0, s>>>(P, n, per, v, r, nullptr, fx, nch * G, part);
    k_fix_scale<<<1, 256, 0, s>>>(part, nb, nch);
    if (n > 0) {
        const int64_t bricks = K / kBrickCells;
        const int E3 = P.tile * P.tile * P.tile;
        const size_t lds = sizeof(unsigned long long) * (size_t)nch * E3;
        k_p2g_real<<<brick_grid(bricks), kP2GThreads, lds, s>>>(P, n, B.list, B.count, x, v, r, cb, ce, part, nch,
                                                                 reinterpret_cast<unsigned long long *>(fx));
    }
    unsigned g = grid_for(nch * G, 256);
    if (g > 4096) g = 4096;
    k_fix_finish<<<g, 256, 0, s>>>(G, nch, part, fx, alpha, mom, acc);
    return hipGetLastError();
}

// Grid part of the G2P pullback, deterministic like k_p2g_real: g_alpha_k =
// -sum_i w_ik gaf_i on nodes below the clamp, the contributions rounded to
// integers at the scale of the largest |gaf_i|.
__global__ void __launch_bounds__(256) k_g2p_vjp_grid(DevParams P, int64_t n, const int32_t *__restrict__ bl,
                                                      const int32_t *__restrict__ bcnt,
                                                      const double *__restrict__ x, const double *__restrict__ A,
                                                      const double *__restrict__ gaf,
                                                      const int32_t *__restrict__ cb, const int32_t *__restrict__ ce,
                                                      const double *__restrict__ part,
                                                      unsigned long long *__restrict__ fx)
{
    extern __shared__ unsigned long long itile[];
    __shared__ int32_t s_range[2];
    const int64_t b = brick_of_block(bl, bcnt);
    if (b < 0) return;
    brick_range(n, b, cb, ce, s_range);
    const int E = P.tile;
    const int E3 = E * E * E;
    for (int k = threadIdx.x; k < E3; k += 256) itile[k] = 0ull;
    __syncthreads();
    const int32_t beg = s_range[0], end = s_range[1];
    if (end <= beg) return;
    const double sc = part[kFixScale];
    int32_t o[3];
    tile_origin(P, b, o);
    for (int64_t q = beg + (int64_t)threadIdx.x; q < end; q += 256) {
        const double xa[3] = {x[q], x[n + q], x[2 * n + q]};
        Stencil s;
        stencil_of(P, xa, s);
        const double sg = -gaf[q];
        for (int cz = 0; cz < 3; ++cz)
            for (int cy = 0; cy < 3; ++cy)
                for (int cx = 0; cx < 3; ++cx) {
                    const int32_t ni = s.node[0][cx], nj = s.node[1][cy], nk = s.node[2][cz];
                    const int64_t gidx = node_index(P, ni, nj, nk);
                    if (!(A[gidx] < P.alpha_max)) continue;
                    const int64_t val = rint_i64((((s.w[0][cx] * s.w[1][cy]) * s.w[2][cz]) * sg) * sc);
                    const int32_t li = ni - o[0], lj = nj - o[1], lk = nk - o[2];
                    const bool in = li >= 0 && lj >= 0 && lk >= 0 && li < E && lj < E && lk < E;
                    tile_add(itile, fx, in, (lk * E + lj) * E + li, gidx, val);
                }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < E3; k += 256) {
        const unsigned long long val = itile[k];
        if (val == 0ull) continue;
        const int32_t ni = o[0] + k % E, nj = o[1] + (k / E) % E, nk = o[2] + k / (E * E);
        atomicAdd(&fx[node_index(P, ni, nj, nk)], val);
    }
}

hipError_t launch_g2p_vjp_grid(const DevParams &P, int64_t n, int64_t K, const double *x, const double *A,
                               const double *gaf, const int32_t *cb, const int32_t *ce, const BrickList &B,
                               double *gA, int64_t *fx, double *part, hipStream_t s)
{
    const int64_t G = P.G;
    const int64_t per = n > 0 ? (n + kFixParts - 1) / kFixParts : 1;
    const int nb = (int)(n > 0 ? (n + per - 1) / per : 1);
    k_fix_prep<<<nb, 256, 0, s>>>(P, n, per, nullptr, nullptr, gaf, fx, G, part);
    k_fix_scale<<<1, 256, 0, s>>>(part, nb, 1);
    if (n > 0) {
        const int64_t bricks = K / kBrickCells;
        const size_t lds = sizeof(unsigned long long) * (size_t)P.tile * P.tile * P.tile;
        k_g2p_vjp_grid<<<brick_grid(bricks), 256, lds, s>>>(P, n, B.list, B.count, x, A, gaf, cb, ce, part,
                                                            reinterpret_cast<unsigned long long *>(fx));
    }
    unsigned g = grid_for(G, 256);
    if (g > 4096) g = 4096;
    k_fix_finish<<<g, 256, 0, s>>>(G, 1, part, fx, gA, nullptr, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_g2p(const DevParams &P, int64_t n, const double *x, const T *u, const int64_t *afx,
                      const double *are, T *uat, T *af, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t nblk = (n + 255) / 256;
    if (afx)
        k_g2p<T, true><<<xcd_grid(nblk), 256, 0, s>>>(P, n, nblk, x, u, afx, nullptr, uat, af);
    else
        k_g2p<T, false><<<xcd_grid(nblk), 256, 0, s>>>(P, n, nblk, x, u, nullptr, are, uat, af);
    return hipGetLastError();
}

template hipError_t launch_g2p<float>(const DevParams &, int64_t, const double *, const float *, const int64_t *,
                                      const double *, float *, float *, hipStream_t);
template hipError_t launch_g2p<double>(const DevParams &, int64_t, const double *, const double *,
                                       const int64_t *, const double *, double *, double *, hipStream_t);

}  // namespace gic
