// a1: cell binning, stable LSD radix sort of the cell keys, cell ranges and
// the gather of granule arrays into sorted order (gfx950).
//
// The contact test of Sec. 3.1 only pairs granules closer than r_i + r_j;
// binning granules into cells of edge >= 2 r_max and sorting them by cell
// makes each granule's candidates the occupants of at most 27 cells, stored
// contiguously so that later stages read them coalesced.
#include "gic_launch.hpp"

namespace gic {

namespace {

constexpr int kRadix = 256;

// Key of every granule; flags non-finite and out-of-box positions.
__global__ void __launch_bounds__(256) k_cell_keys(DevParams P, int64_t n, const double *__restrict__ x,
                                                   uint32_t *__restrict__ key, int64_t *err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xa[3] = {x[i], x[n + i], x[2 * n + i]};
    int32_t c[3];
    bool bad = false, out = false;
    for (int a = 0; a < 3; ++a) {
        bad |= !isfinite(xa[a]);
        out |= !(xa[a] >= 0.0 && xa[a] < P.L[a]);
        c[a] = cell_coord(xa[a], P.inv_cell, P.nc[a]);
    }
    if (bad) raise_error(err, kErrNonFinite, i);
    else if (out) raise_error(err, kErrDomain, i);
    key[i] = key_of_cell(P, c[0], c[1], c[2]);
}

// Per-tile histogram of one 8-bit digit: hist[d * tiles + tile].
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                             int shift, uint32_t *__restrict__ hist, int64_t tiles)
{
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        int64_t p = base + (int64_t)it * kSortThreads + tid;
        if (p < n) atomicAdd(&h[(keys[p] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * tiles + blockIdx.x] = h[tid];
}

// Exclusive prefix sum of len entries in place, one workgroup of 1024
// threads: each thread sums a contiguous chunk, the chunk sums are scanned in
// LDS, then each chunk is rewritten with its running prefix.
__global__ void __launch_bounds__(1024) k_scan_exclusive(uint32_t *a, int64_t len)
{
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (len + 1023) / 1024;
    const int64_t lo = tid * chunk;
    const int64_t hi = lo + chunk < len ? lo + chunk : len;
    uint32_t s = 0;
    for (int64_t k = lo; k < hi; ++k) s += a[k];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t t = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += t;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    for (int64_t k = lo; k < hi; ++k) {
        uint32_t t = a[k];
        a[k] = run;
        run += t;
    }
}

// Stable scatter of one digit pass.  The tile is processed in rounds of 256
// consecutive keys; inside a wave, lanes with equal digits are found with
// eight ballots (one per digit bit), which gives each key its rank among
// earlier lanes of the same digit; per-wave digit counts in LDS order the
// four waves, and a running count per digit orders the rounds.  vin == NULL
// means the values are the input positions.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                const int32_t *__restrict__ vin,
                                                                uint32_t *__restrict__ kout,
                                                                int32_t *__restrict__ vout, int64_t n, int shift,
                                                                const uint32_t *__restrict__ offs, int64_t tiles)
{
    __shared__ uint32_t base[kRadix];
    __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    base[tid] = offs[(int64_t)tid * tiles + blockIdx.x];
    for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t p = tile0 + (int64_t)it * kSortThreads + tid;
        const bool valid = p < n;
        const uint32_t k = valid ? kin[p] : 0u;
        const int32_t val = valid ? (vin ? vin[p] : (int32_t)p) : 0;
        const uint32_t d = (k >> shift) & (kRadix - 1);
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt_mask);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = k;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        base[tid] += add;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t *a, int64_t len, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// begin/end of each occupied cell from the sorted keys.
__global__ void __launch_bounds__(256) k_cell_ranges(const uint32_t *__restrict__ sk, int64_t n,
                                                     int32_t *__restrict__ cb, int32_t *__restrict__ ce)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    uint32_t k = sk[q];
    if (q == 0 || sk[q - 1] != k) cb[k] = (int32_t)q;
    if (q == n - 1 || sk[q + 1] != k) ce[k] = (int32_t)(q + 1);
}

__global__ void __launch_bounds__(256) k_reorder(int64_t n, const int32_t *__restrict__ order,
                                                 const double *__restrict__ x, const double *__restrict__ v,
                                                 const double *__restrict__ r, const int32_t *__restrict__ id,
                                                 double *__restrict__ xo, double *__restrict__ vo,
                                                 double *__restrict__ ro, int32_t *__restrict__ ido)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int64_t i = order[q];
    for (int a = 0; a < 3; ++a) {
        xo[a * n + q] = x[a * n + i];
        vo[a * n + q] = v[a * n + i];
    }
    ro[q] = r[i];
    if (ido) ido[q] = id[i];
}

}  // namespace

hipError_t launch_sort_cells(const DevParams &P, int64_t n, const double *x, uint32_t *key, int32_t *order,
                             int32_t *cell_begin, int32_t *cell_end, int64_t K, SortScratch &S, int64_t *err,
                             hipStream_t s)
{
    {
        unsigned g = grid_for(K, 256);
        if (g > 65536) g = 65536;
        k_fill_i32<<<g, 256, 0, s>>>(cell_begin, K, 0);
        k_fill_i32<<<g, 256, 0, s>>>(cell_end, K, 0);
    }
    if (n == 0) return hipGetLastError();
    k_cell_keys<<<grid_for(n, 256), 256, 0, s>>>(P, n, x, key, err);
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    const uint32_t *kin = key;
    const int32_t *vin = nullptr;
    for (int pass = 0; pass < S.passes; ++pass) {
        const bool last = pass == S.passes - 1;
        uint32_t *kout = last ? S.skeys : ((pass & 1) ? S.kB : S.kA);
        int32_t *vout = last ? order : ((pass & 1) ? S.vB : S.vA);
        const int shift = 8 * pass;
        k_radix_hist<<<(unsigned)tiles, kSortThreads, 0, s>>>(kin, n, shift, S.hist, tiles);
        k_scan_exclusive<<<1, 1024, 0, s>>>(S.hist, tiles * kRadix);
        k_radix_scatter<<<(unsigned)tiles, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, shift, S.hist, tiles);
        kin = kout;
        vin = vout;
    }
    k_cell_ranges<<<grid_for(n, 256), 256, 0, s>>>(S.skeys, n, cell_begin, cell_end);
    return hipGetLastError();
}

hipError_t launch_reorder(int64_t n, const int32_t *order, const double *x, const double *v, const double *r,
                          const int32_t *id, double *xo, double *vo, double *ro, int32_t *ido, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_reorder<<<grid_for(n, 256), 256, 0, s>>>(n, order, x, v, r, ido ? id : nullptr, xo, vo, ro, ido);
    return hipGetLastError();
}

}  // namespace gic
