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
constexpr int64_t kRtsGrid = 1024;  // workgroups of the tile loops of the digit passes

// Key of every granule; flags non-finite and out-of-box positions.  With
// the previous sorted keys pk (same n), granules whose key differs from
// pk at their position are appended to chg (up to kChgCap; ctl[0] counts
// them all).  With xref (the positions of the neighbour list's build, same
// order), each workgroup writes the largest squared displacement of its
// granules since the build to dpart[block] (no atomics: one address hit by
// every wave would serialise them).
__global__ void __launch_bounds__(256) k_cell_keys(DevParams P, int64_t n, const double *__restrict__ x,
                                                   uint32_t *__restrict__ key, int64_t *err,
                                                   const uint32_t *__restrict__ pk, uint64_t *__restrict__ chg,
                                                   int32_t *__restrict__ ctl, const float *__restrict__ xref,
                                                   float *__restrict__ dpart)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (xref) {
        float d2 = 0.0f;
        if (i < n) {
            double s2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double d = x[a * n + i] - (double)xref[a * n + i];
                s2 += d * d;
            }
            d2 = (float)s2;
            if (!(d2 >= 0.0f)) d2 = __builtin_huge_valf();  // NaN: rebuild (the position is flagged below)
        }
        __shared__ float s_d2[4];
        for (int off = 32; off > 0; off >>= 1) d2 = fmaxf(d2, __shfl_xor(d2, off));
        if ((threadIdx.x & 63) == 0) s_d2[threadIdx.x >> 6] = d2;
        __syncthreads();
        if (threadIdx.x == 0) dpart[blockIdx.x] = fmaxf(fmaxf(s_d2[0], s_d2[1]), fmaxf(s_d2[2], s_d2[3]));
    }
    bool changed = false;
    uint32_t k = 0;
    if (i < n) {
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
        k = key_of_cell(P, c[0], c[1], c[2]);
        key[i] = k;
        changed = pk && pk[i] != k;
    }
    if (!pk) return;
    // changed keys appended with one counter atomic per workgroup that has
    // any (a moving bed changes many keys, and atomics on one address
    // serialise: one per wave cost 11 us on 65,536 granules)
    __shared__ int32_t s_cnt[4];
    __shared__ int32_t s_base;
    const uint64_t mask = __ballot(changed);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_cnt[wave] = (int32_t)__popcll(mask);
    __syncthreads();
    const int32_t tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    if (tot == 0) return;
    if (threadIdx.x == 0) s_base = atomicAdd(&ctl[0], tot);
    __syncthreads();
    if (changed) {
        int32_t slot = s_base + (int32_t)__popcll(mask & ((1ull << lane) - 1ull));
        for (int w = 0; w < wave; ++w) slot += s_cnt[w];
        if (slot < kChgCap) chg[slot] = ((uint64_t)k << 32) | (uint64_t)i;
    }
}

// Exclusive prefix sum in place, in three coalesced phases: each workgroup
// reduces one contiguous chunk, one workgroup scans the chunk totals, then
// each workgroup rescans its chunk 1024 entries at a time from its offset.
constexpr int kScanThreads = 1024;

__device__ inline uint32_t block_reduce_sum(uint32_t v, uint32_t *lds)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    uint32_t t = 0;
    if (threadIdx.x < 64) {
        t = threadIdx.x < (blockDim.x >> 6) ? lds[threadIdx.x] : 0u;
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    }
    __syncthreads();
    return t;  // valid in wave 0
}

// Inclusive scan over the workgroup (thread order); *total = sum of all.
__device__ inline uint32_t block_scan_inclusive(uint32_t v, uint32_t *lds, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int nw = blockDim.x >> 6;
        uint32_t w = threadIdx.x < nw ? lds[threadIdx.x] : 0u;
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t t = __shfl_up(w, off);
            if (lane >= off) w += t;
        }
        if (threadIdx.x < nw) lds[threadIdx.x] = w;  // inclusive prefix of wave totals
    }
    __syncthreads();
    const uint32_t before = wave > 0 ? lds[wave - 1] : 0u;
    *total = lds[(blockDim.x >> 6) - 1];
    __syncthreads();
    return v + before;
}

// skip (optional): the sort's control words; skip[2] set means the cell
// ranges of the last sort still hold (no key changed) and are kept.
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t *__restrict__ a, int64_t len,
                                                              int64_t chunk, uint32_t *__restrict__ sums,
                                                              const int32_t *__restrict__ skip)
{
    if (skip && skip[2]) return;
    __shared__ uint32_t lds[kScanThreads / 64];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < len ? lo + chunk : len;
    uint32_t s = 0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += kScanThreads) s += a[k];
    s = block_reduce_sum(s, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_spine(uint32_t *sums, int nb, const int32_t *__restrict__ skip)
{
    if (skip && skip[2]) return;
    __shared__ uint32_t lds[kScanThreads / 64];
    const uint32_t v = threadIdx.x < nb ? sums[threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t inc = block_scan_inclusive(v, lds, &total);
    if (threadIdx.x < nb) sums[threadIdx.x] = inc - v;
}

// ---- digit passes (reduce, scan, scatter) --------------------------------
//
// Each 8-bit digit pass is three kernels with no waits between workgroups:
// every tile of 2,048 keys (256 for sorts of at most 2^18 keys, so that a
// small sort still spreads over many workgroups) counts its digits
// (k_rts_count, into tcnt[digit][tile]); one workgroup per digit turns its
// row into the exclusive prefix over the tiles and records the row's total
// (k_rts_scan); every tile then scatters its keys stably (k_rts_scatter)
// from the prefix
// of its tile plus the keys of all smaller digits (a scan of the 256 row
// totals).  The tile loops stride over the grid, so a launch needs no more
// workgroups than it has tiles.

// Rank of each lane's digit among the lanes of its wave with the same digit
// (8 ballots), and the number of such lanes.
__device__ inline uint64_t digit_mask(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Mask of the lanes below this one in its wave.
__device__ inline uint64_t lanes_below()
{
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Digit counts of every tile of ITEMS x 256 keys: tcnt[d * tiles + t].
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads) k_rts_count(const uint32_t *__restrict__ kin, int64_t n, int pass,
                                                            int64_t tiles, uint32_t *__restrict__ tcnt,
                                                            const int32_t *__restrict__ skip)
{
    if (skip && skip[1]) return;  // the incremental path sorted this time
    __shared__ uint32_t s_cnt[kRadix];
    const int tid = threadIdx.x;
    const int shift = 8 * pass;
    const uint64_t lt = lanes_below();
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        s_cnt[tid] = 0;
        __syncthreads();
        const int64_t tile0 = t * (kSortThreads * ITEMS);
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int64_t p = tile0 + (int64_t)it * kSortThreads + tid;
            const bool valid = p < n;
            const uint32_t d = valid ? (kin[p] >> shift) & (kRadix - 1) : 0u;
            const uint64_t m = digit_mask(d, valid);
            if (valid && (m & lt) == 0) atomicAdd(&s_cnt[d], (uint32_t)__popcll(m));
        }
        __syncthreads();
        tcnt[(int64_t)tid * tiles + t] = s_cnt[tid];
        __syncthreads();
    }
}

// Workgroup d: tcnt[d][t] <- keys with digit d in tiles before t;
// rowtot[d] <- keys with digit d.  Thread i takes a contiguous chunk of the
// row, so the row is read in one sweep and scanned once.
__global__ void __launch_bounds__(kSortThreads) k_rts_scan(uint32_t *__restrict__ tcnt, int64_t tiles,
                                                           uint32_t *__restrict__ rowtot,
                                                           const int32_t *__restrict__ skip)
{
    if (skip && skip[1]) return;
    __shared__ uint32_t lds[kSortThreads / 64];
    const int d = blockIdx.x;
    uint32_t *row = tcnt + (int64_t)d * tiles;
    const int64_t chunk = (tiles + kSortThreads - 1) / kSortThreads;
    const int64_t lo = (int64_t)threadIdx.x * chunk;
    const int64_t hi = lo + chunk < tiles ? lo + chunk : tiles;
    uint32_t sum = 0;
    for (int64_t t = lo; t < hi; ++t) sum += row[t];
    uint32_t total;
    uint32_t run = block_scan_inclusive(sum, lds, &total) - sum;
    for (int64_t t = lo; t < hi; ++t) {
        const uint32_t c = row[t];
        row[t] = run;
        run += c;
    }
    if (threadIdx.x == 0) rowtot[d] = total;
}

// Stable scatter of every tile's keys (and values: vin, or the positions)
// from the offsets of k_rts_scan, in rounds of 256 keys in position order.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads) k_rts_scatter(const uint32_t *__restrict__ kin,
                                                              const int32_t *__restrict__ vin,
                                                              uint32_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                              int64_t n, int pass, int64_t tiles,
                                                              const uint32_t *__restrict__ tcnt,
                                                              const uint32_t *__restrict__ rowtot,
                                                              const int32_t *__restrict__ skip)
{
    if (skip && skip[1]) return;
    __shared__ uint32_t s_base[kRadix];  // where this tile's next key of each digit goes
    __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];
    __shared__ uint32_t lds[kSortThreads / 64];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int shift = 8 * pass;
    const uint64_t lt = lanes_below();
    for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
    // keys of all smaller digits
    const uint32_t g = rowtot[tid];
    uint32_t total;
    const uint32_t dbase = block_scan_inclusive(g, lds, &total) - g;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t tile0 = t * (kSortThreads * ITEMS);
        uint32_t k[ITEMS];
        int32_t val[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int64_t p = tile0 + (int64_t)it * kSortThreads + tid;
            const bool valid = p < n;
            k[it] = valid ? kin[p] : 0xffffffffu;
            val[it] = valid ? (vin ? vin[p] : (int32_t)p) : 0;
        }
        s_base[tid] = dbase + tcnt[(int64_t)tid * tiles + t];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int64_t p = tile0 + (int64_t)it * kSortThreads + tid;
            const bool valid = p < n;
            const uint32_t d = (k[it] >> shift) & (kRadix - 1);
            const uint64_t m = digit_mask(d, valid);
            const uint32_t rank = (uint32_t)__popcll(m & lt);
            if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
            __syncthreads();
            if (valid) {
                uint32_t pos = s_base[d] + rank;
                for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
                if ((int64_t)pos < n) {
                    kout[pos] = k[it];
                    vout[pos] = val[it];
                }
            }
            __syncthreads();
            uint32_t add = 0;
            for (int w = 0; w < kSortThreads / 64; ++w) {
                add += wcnt[w][tid];
                wcnt[w][tid] = 0;
            }
            s_base[tid] += add;
            __syncthreads();
        }
    }
}

// Number of granules per cell key, from the sorted keys: the first lane of
// each run of equal keys inside a wave adds the run's length.
__global__ void __launch_bounds__(256) k_cell_count(const uint32_t *__restrict__ sk, int64_t n,
                                                    uint32_t *__restrict__ cnt, const int32_t *__restrict__ skip)
{
    if (skip && skip[2]) return;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = q < n;
    const uint32_t k = valid ? sk[q] : 0u;
    const bool start = valid && (lane == 0 || sk[q - 1] != k);
    const uint64_t starts = __ballot(start) | (~__ballot(valid));  // invalid lanes end the last run
    if (start) {
        const uint64_t above = lane == 63 ? 0ull : (starts >> (lane + 1)) << (lane + 1);
        const int next = above ? __ffsll((unsigned long long)above) - 1 : 64;
        atomicAdd(&cnt[k], (uint32_t)(next - lane));
    }
}

// Last phase of the scan of the per-cell counts: begin = exclusive prefix,
// end = inclusive prefix; the counts are reset to zero for the next sort.
__global__ void __launch_bounds__(kScanThreads) k_scan_down_ranges(uint32_t *__restrict__ cnt,
                                                                   uint32_t *__restrict__ begin,
                                                                   uint32_t *__restrict__ end, int64_t len,
                                                                   int64_t chunk, const uint32_t *__restrict__ sums,
                                                                   int32_t *__restrict__ ctl, int keep)
{
    if (keep && ctl[2]) return;  // ranges unchanged (and no changed granule to uncount)
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[0] = 0;  // no changed granules counted for the next sort
    __shared__ uint32_t lds[kScanThreads / 64];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < len ? lo + chunk : len;
    uint32_t carry = sums[blockIdx.x];
    for (int64_t base = lo; base < hi; base += kScanThreads) {
        const int64_t k = base + threadIdx.x;
        const uint32_t v = k < hi ? cnt[k] : 0u;
        uint32_t total;
        const uint32_t inc = block_scan_inclusive(v, lds, &total);
        if (k < hi) {
            begin[k] = carry + inc - v;
            end[k] = carry + inc;
            cnt[k] = 0u;
        }
        carry += total;
    }
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
    if ((uint64_t)i >= (uint64_t)n) return;  // not a permutation of [0, n): position q left untouched
    for (int a = 0; a < 3; ++a) {
        xo[a * n + q] = x[a * n + i];
        vo[a * n + q] = v[a * n + i];
    }
    ro[q] = r[i];
    if (ido) ido[q] = id[i];
}

// ---- incremental path: few keys changed since the last sort -------------
//
// The previous sorted keys pk are non-decreasing by position, so the
// granules whose key still equals pk at their position (U) are in sorted
// order already, whatever state they come from; the others (C, at most
// kChgCap) are sorted here.  The stable sort by (key, position) is then the
// merge of U and C: an element's place is the number of U elements before
// it plus the number of C elements before it.  For u in U at position i
// that is (i - #C positions below i) + #C pairs below (key, i); for c in C
// it is its rank in C plus #U pairs below (k_c, i_c) = L - #C positions
// below L, with L the number of positions i with (pk[i], i) < (k_c, i_c).

__device__ inline int lower_bound_u64(const uint64_t *a, int m, uint64_t v)
{
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline int lower_bound_u32(const uint32_t *a, int m, uint32_t v)
{
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// One workgroup: decides the path, sorts C by (key, position) and by
// position (bitonic, in LDS), and places the C elements.  With nl it also
// decides whether the neighbour list must be rebuilt this step (nl[0]):
// when force is set, when any key changed (the sorted order may change), or
// when the largest squared displacement since the build (the maximum of the
// nd per-workgroup maxima dpart of the key kernel) reaches thr2.
__global__ void __launch_bounds__(1024) k_chg_sort(int64_t n, const uint32_t *__restrict__ pk,
                                                   const uint64_t *__restrict__ chg, int32_t *__restrict__ ctl,
                                                   uint64_t *__restrict__ chg_s, uint32_t *__restrict__ chg_p,
                                                   uint32_t *__restrict__ skeys, int32_t *__restrict__ order,
                                                   uint32_t *__restrict__ nl, int force, float thr2,
                                                   const float *__restrict__ dpart, int64_t nd)
{
    __shared__ uint64_t sk[kChgCap];
    __shared__ uint32_t sp[kChgCap];
    __shared__ float s_dm[1024 / 64];
    const int tid = threadIdx.x;
    const int m = ctl[0];
    const bool incremental = m <= kChgCap;
    float dm = 0.0f;
    if (dpart)
        for (int64_t i = tid; i < nd; i += 1024) dm = fmaxf(dm, dpart[i]);
    for (int off = 32; off > 0; off >>= 1) dm = fmaxf(dm, __shfl_xor(dm, off));
    if ((tid & 63) == 0) s_dm[tid >> 6] = dm;
    __syncthreads();  // every thread has read ctl[0] before thread 0 writes ctl[1]
    if (tid == 0) {
        ctl[1] = incremental ? 1 : 0;
        ctl[2] = m == 0 ? 1 : 0;  // no key changed: the last sort's order, ranges and bricks hold
    }
    if (tid == 0 && nl) {
        float d2 = 0.0f;
        for (int w = 0; w < 1024 / 64; ++w) d2 = fmaxf(d2, s_dm[w]);
        nl[0] = (force || m != 0 || !(d2 < thr2)) ? 1u : 0u;
    }
    if (!incremental || m == 0) return;
    int N = 2;
    while (N < m) N <<= 1;
    for (int i = tid; i < N; i += 1024) {
        const uint64_t e = i < m ? chg[i] : ~0ull;
        sk[i] = e;
        sp[i] = i < m ? (uint32_t)(e & 0xffffffffu) : 0xffffffffu;
    }
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < N; i += 1024) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t a = sk[i], b = sk[l];
                    if ((a > b) == up) {
                        sk[i] = b;
                        sk[l] = a;
                    }
                    const uint32_t c = sp[i], d = sp[l];
                    if ((c > d) == up) {
                        sp[i] = d;
                        sp[l] = c;
                    }
                }
            }
            __syncthreads();
        }
    for (int r = tid; r < m; r += 1024) {
        chg_s[r] = sk[r];
        chg_p[r] = sp[r];
        const uint32_t kc = (uint32_t)(sk[r] >> 32), ic = (uint32_t)(sk[r] & 0xffffffffu);
        int64_t lo = 0, hi = n;  // L: positions i with (pk[i], i) < (kc, ic)
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            const uint32_t pm = pk[mid];
            if (pm < kc || (pm == kc && mid < (int64_t)ic)) lo = mid + 1; else hi = mid;
        }
        const int64_t place = r + lo - lower_bound_u32(sp, m, (uint32_t)lo);
        order[place] = (int32_t)ic;
        skeys[place] = kc;
    }
}

// Places the U elements (one thread per position).
__global__ void __launch_bounds__(256) k_merge(int64_t n, const uint32_t *__restrict__ key,
                                               const uint32_t *__restrict__ pk, const int32_t *__restrict__ ctl,
                                               const uint64_t *__restrict__ chg_s, const uint32_t *__restrict__ chg_p,
                                               uint32_t *__restrict__ skeys, int32_t *__restrict__ order)
{
    if (!ctl[1]) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = key[i];
    if (k != pk[i]) return;  // an element of C, placed by k_chg_sort
    const int m = ctl[0];
    int64_t place = i;
    if (m > 0)
        place = i - lower_bound_u32(chg_p, m, (uint32_t)i) +
                lower_bound_u64(chg_s, m, ((uint64_t)k << 32) | (uint64_t)i);
    order[place] = (int32_t)i;
    skeys[place] = k;
}

// ---- occupied bricks, in brick order (the schedule of the brick kernels) ----

__device__ inline bool brick_occupied(int64_t b, const int32_t *__restrict__ cb, const int32_t *__restrict__ ce)
{
    return ce[b * kBrickCells + kBrickCells - 1] > cb[b * kBrickCells];
}

__global__ void __launch_bounds__(256) k_brick_count(int64_t nbricks, int64_t per_block, const int32_t *__restrict__ cb,
                                                     const int32_t *__restrict__ ce, uint32_t *__restrict__ sums,
                                                     const int32_t *__restrict__ skip)
{
    if (skip && skip[2]) return;
    __shared__ uint32_t lds[4];
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = lo + per_block < nbricks ? lo + per_block : nbricks;
    uint32_t c = 0;
    for (int64_t b = lo + threadIdx.x; b < hi; b += 256) c += brick_occupied(b, cb, ce) ? 1u : 0u;
    c = block_reduce_sum(c, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = c;
}

// Exclusive scan of the block counts in place; the total is the list length.
__global__ void __launch_bounds__(kScanThreads) k_brick_spine(uint32_t *sums, int nb, int32_t *count,
                                                              const int32_t *__restrict__ skip)
{
    if (skip && skip[2]) return;
    __shared__ uint32_t lds[kScanThreads / 64];
    const uint32_t v = threadIdx.x < nb ? sums[threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t inc = block_scan_inclusive(v, lds, &total);
    if (threadIdx.x < nb) sums[threadIdx.x] = inc - v;
    if (threadIdx.x == 0) *count = (int32_t)total;
}

__global__ void __launch_bounds__(256) k_brick_scatter(int64_t nbricks, int64_t per_block,
                                                       const int32_t *__restrict__ cb, const int32_t *__restrict__ ce,
                                                       const uint32_t *__restrict__ sums, int32_t *__restrict__ list,
                                                       int32_t *__restrict__ slot_of, const int32_t *__restrict__ skip)
{
    if (skip && skip[2]) return;
    __shared__ uint32_t lds[4];
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = lo + per_block < nbricks ? lo + per_block : nbricks;
    uint32_t base = sums[blockIdx.x];
    for (int64_t b0 = lo; b0 < hi; b0 += 256) {  // same trip count for the whole workgroup
        const int64_t b = b0 + threadIdx.x;
        const uint32_t f = b < hi && brick_occupied(b, cb, ce) ? 1u : 0u;
        uint32_t total;
        const uint32_t inc = block_scan_inclusive(f, lds, &total);
        if (f) list[base + inc - 1] = (int32_t)b;
        if (b < hi) slot_of[b] = f ? (int32_t)(base + inc - 1) : -1;
        base += total;
    }
}

}  // namespace

namespace {

int64_t scan_chunk(int64_t len)
{
    int64_t chunk = (len + kScanThreads - 1) / kScanThreads;
    return ((chunk + kScanThreads - 1) / kScanThreads) * kScanThreads;
}

}  // namespace

hipError_t launch_sort_cells(const DevParams &P, int64_t n, const double *x, uint32_t *key, int32_t *order,
                             int32_t *cell_begin, int32_t *cell_end, int64_t K, SortScratch &S, int64_t *err,
                             hipStream_t s, const NbrList *nl, int force, int keep_ranges)
{
    uint32_t *cnt = S.cnt;  // all zero between sorts
    // previous sorted keys: usable when the last sort had the same n
    const bool inc = n > 0 && S.last_n == n;
    const uint32_t *pk = inc ? S.skeys[S.cur] : nullptr;
    uint32_t *skeys = S.skeys[S.cur ^ 1];
    const int32_t *skip = inc ? S.ctl : nullptr;
    // the displacement since the list's build is measured when the list may
    // be kept (its build had this sorted order: the caller checked that)
    const bool measure = nl && inc && !force && nl->thr2 > 0.0f;
    if (n > 0) {
        k_cell_keys<<<grid_for(n, 256), 256, 0, s>>>(P, n, x, key, err, pk, S.chg, S.ctl,
                                                     measure ? nl->xref : nullptr, measure ? nl->dpart : nullptr);
        if (inc) {
            k_chg_sort<<<1, 1024, 0, s>>>(n, pk, S.chg, S.ctl, S.chg_s, S.chg_p, skeys, order,
                                          nl ? nl->ctl : nullptr, measure ? 0 : 1, nl ? nl->thr2 : 0.0f,
                                          measure ? nl->dpart : nullptr, (int64_t)grid_for(n, 256));
            k_merge<<<grid_for(n, 256), 256, 0, s>>>(n, key, pk, S.ctl, S.chg_s, S.chg_p, skeys, order);
        }
        // digit passes (skipped on the device when the incremental path sorted)
        const int items = sort_items(n);
        const int64_t tiles = (n + kSortThreads * items - 1) / (kSortThreads * items);
        const unsigned tg = (unsigned)(tiles < kRtsGrid ? tiles : kRtsGrid);
        const uint32_t *kin = key;
        const int32_t *vin = nullptr;
        for (int pass = 0; pass < S.passes; ++pass) {
            const bool last = pass == S.passes - 1;
            uint32_t *kout = last ? skeys : ((pass & 1) ? S.kB : S.kA);
            int32_t *vout = last ? order : ((pass & 1) ? S.vB : S.vA);
            if (items == 1)
                k_rts_count<1><<<tg, kSortThreads, 0, s>>>(kin, n, pass, tiles, S.tcnt, skip);
            else
                k_rts_count<kSortItems><<<tg, kSortThreads, 0, s>>>(kin, n, pass, tiles, S.tcnt, skip);
            k_rts_scan<<<kRadix, kSortThreads, 0, s>>>(S.tcnt, tiles, S.rowtot, skip);
            if (items == 1)
                k_rts_scatter<1><<<tg, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, pass, tiles, S.tcnt,
                                                             S.rowtot, skip);
            else
                k_rts_scatter<kSortItems><<<tg, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, pass, tiles, S.tcnt,
                                                                      S.rowtot, skip);
            kin = kout;
            vin = vout;
        }
    }
    // cell ranges: kept when the caller's tables hold the last sort's ranges
    // and no key changed (decided on the device by k_chg_sort)
    const int keep = keep_ranges && inc ? 1 : 0;
    const int32_t *kskip = keep ? S.ctl : nullptr;
    if (n > 0) k_cell_count<<<grid_for(n, 256), 256, 0, s>>>(skeys, n, cnt, kskip);
    const int64_t chunk = scan_chunk(K);
    const int nb = (int)((K + chunk - 1) / chunk);
    k_scan_reduce<<<nb, kScanThreads, 0, s>>>(cnt, K, chunk, S.sums, kskip);
    k_scan_spine<<<1, kScanThreads, 0, s>>>(S.sums, nb, kskip);
    k_scan_down_ranges<<<nb, kScanThreads, 0, s>>>(cnt, reinterpret_cast<uint32_t *>(cell_begin),
                                                   reinterpret_cast<uint32_t *>(cell_end), K, chunk, S.sums, S.ctl,
                                                   keep);
    S.cur ^= 1;  // this sort's keys are the previous keys of the next
    S.last_n = n;
    return hipGetLastError();
}

hipError_t launch_brick_list(const int32_t *cb, const int32_t *ce, BrickList &B, hipStream_t s, const int32_t *skip)
{
    const int64_t nb = B.nbricks;
    if (nb <= 0) return hipSuccess;
    int64_t per = 1024;
    while ((nb + per - 1) / per > kScanThreads) per *= 2;
    const int blocks = (int)((nb + per - 1) / per);
    k_brick_count<<<blocks, 256, 0, s>>>(nb, per, cb, ce, B.sums, skip);
    k_brick_spine<<<1, kScanThreads, 0, s>>>(B.sums, blocks, B.count, skip);
    k_brick_scatter<<<blocks, 256, 0, s>>>(nb, per, cb, ce, B.sums, B.list, B.slot_of, skip);
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
