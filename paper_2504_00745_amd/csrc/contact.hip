// a2 + a3: neighbour candidates and contact forces (Sec. 3.1, Eq. 1a-c) on
// gfx950.
//
// The dry contact runs in two kernels: a neighbour-list build (k_nbr_build,
// one workgroup per brick, candidates from an LDS copy of the brick's cell
// shell) that lists every granule closer than r_i + r_j + skin, and the
// contact forces from that list (k_contact_list, one thread per granule),
// which runs the exact double test of Sec. 3.1 on every listed partner each
// step.  The stepping path builds the list only when the sorted order
// changed or a granule moved by skin / 2 since the last build; a granule's
// force sum runs over its touching partners in one canonical order
// (canon_before: by distance in sorted order) either way, so the forces do
// not depend on when the list was built, nor on which kernel summed them.  The capillary
// instantiation of k_contact_lds (candidates and forces in one brick kernel)
// serves wet beds.
//
// Each granule visits only the neighbour cells its search box
// [x - (r_i + r_max), x + (r_i + r_max)] overlaps (at most 27, typically 8
// when the cell is twice the largest diameter); candidates of a cell are
// contiguous in sorted order.  The contact test, the overlap and the normal
// are double in both forms (the overlap is a small difference of nearly
// equal distances); the pair law and the per-granule sum run in T.
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

// Visit the candidate ranges of granule q: for each row (cy, cz) of the
// search box the cells [lo_x, hi_x] split into at most two runs of
// consecutive keys (a run ends at a brick face), and consecutive keys have
// contiguous granule ranges, so each run is one range [begin, end).
template <typename F>
__device__ inline void for_each_run(const DevParams &P, int64_t n, const int32_t lo[3], const int32_t hi[3],
                                    const int32_t *__restrict__ cb, const int32_t *__restrict__ ce, F &&f)
{
    for (int32_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int32_t cy = lo[1]; cy <= hi[1]; ++cy) {
            int32_t cx = lo[0];
            while (cx <= hi[0]) {
                const int32_t brick_end = (cx & ~(kBrick - 1)) + (kBrick - 1);
                const int32_t cend = hi[0] < brick_end ? hi[0] : brick_end;
                const uint32_t k0 = key_of_cell(P, cx, cy, cz);
                int32_t jb = cb[k0], je = ce[k0 + (uint32_t)(cend - cx)];
                clip_range(n, jb, je);
                f(jb, je);
                cx = cend + 1;
            }
        }
}

// Canonical order of a granule's partners, in which every kernel sums its
// pair forces: by distance in sorted order from the granule, |j - q|, the
// lower position first at equal distance.  It depends on the sorted order
// only, so lists built at different steps of one order give the same sums;
// and in a regular packing the partners at one place of neighbouring
// granules' lists lie in the same direction, so their state loads coalesce
// and the in-workgroup partners come first.
__device__ inline bool canon_before(int64_t a, int64_t b, int64_t q)
{
    const int64_t da = a > q ? a - q : q - a, db = b > q ? b - q : q - b;
    return da < db || (da == db && a < b);
}

// Insertion sort into canonical order of the m entries of granule q at
// a[0], a[stride], ... (an LDS column or a list column); j_of maps an entry
// to its sorted position.
template <typename E, typename J>
__device__ inline void canon_sort(E *a, int64_t stride, int m, int64_t q, J &&j_of)
{
    for (int i = 1; i < m; ++i) {
        const E e = a[i * stride];
        const int64_t je = j_of(e);
        int k = i - 1;
        while (k >= 0) {
            const E f = a[k * stride];
            if (!canon_before(je, j_of(f), q)) break;
            a[(k + 1) * stride] = f;
            --k;
        }
        a[(k + 1) * stride] = e;
    }
}

// Every granule in the cell runs of q's search box (cells lo..hi), q
// itself excepted, visited once in canonical order.  For the rare granules
// whose partners overflow a list: each step rescans the runs, taking in
// each run the nearest position beyond the last distance.
template <typename F>
__device__ inline void for_each_canonical(const DevParams &P, int64_t n, int64_t q, const int32_t lo[3],
                                          const int32_t hi[3], const int32_t *__restrict__ cb,
                                          const int32_t *__restrict__ ce, F &&f)
{
    int64_t d = 0;      // distance of the last granule visited (q itself at 0)
    bool upper = true;  // q + d already considered
    for (;;) {
        if (!upper) {  // q - d was visited: q + d next, if it is a candidate
            upper = true;
            const int64_t j = q + d;
            bool cand = false;
            for_each_run(P, n, lo, hi, cb, ce, [&](int32_t jb, int32_t je) { cand |= j >= jb && j < je; });
            if (cand) {
                f((int32_t)j);
                continue;
            }
        }
        // the least distance beyond d with a candidate, the lower side first
        int64_t best = INT64_MAX;
        bool low = false;
        for_each_run(P, n, lo, hi, cb, ce, [&](int32_t jb, int32_t je) {
            if (je <= jb) return;
            const int64_t jl = (int64_t)je - 1 < q - d - 1 ? (int64_t)je - 1 : q - d - 1;
            if (jl >= jb && (q - jl < best || (q - jl == best && !low))) {
                best = q - jl;
                low = true;
            }
            const int64_t ju = (int64_t)jb > q + d + 1 ? (int64_t)jb : q + d + 1;
            if (ju < je && ju - q < best) {
                best = ju - q;
                low = false;
            }
        });
        if (best == INT64_MAX) return;
        d = best;
        upper = !low;
        f((int32_t)(low ? q - d : q + d));
    }
}

constexpr int kUnroll = 4;
constexpr int kMaxPartners = 12;  // partners listed per granule before forces are evaluated

// Double state of a partner granule, loaded in one go so that its loads
// overlap.
struct Partner {
    double x[3], v[3], r;
};

__device__ inline Partner fetch_partner(int64_t n, const double *__restrict__ x, const double *__restrict__ v,
                                        const double *__restrict__ r, int32_t j)
{
    Partner p;
    p.x[0] = x[j];
    p.x[1] = x[n + j];
    p.x[2] = x[2 * n + j];
    p.r = r[j];
    p.v[0] = v[j];
    p.v[1] = v[n + j];
    p.v[2] = v[2 * n + j];
    return p;
}

// Force that partner p exerts on granule i: the overlap, its normal and the
// relative velocity come from double positions and velocities; the pair law
// of Eq. (1a)-(1c) runs in T.
// WET: the partner's mass mj_d is given (the wet mass of Eq. 19); otherwise
// it is rho_s V of the partner's radius.
template <typename T, bool WET = false>
__device__ inline void pair_from(const DevParams &P, const double xi[3], const double vi[3], double ri, double mi,
                                 const Partner &p, double mj_d, T acc[3])
{
    const double d0 = xi[0] - p.x[0], d1 = xi[1] - p.x[1], d2c = xi[2] - p.x[2];
    const double rj = p.r;
    double d2;
    {
#pragma clang fp contract(off)
        d2 = (d0 * d0 + d1 * d1) + d2c * d2c;
    }
    const double R = ri + rj;
    T nh[3];
    T delta;
    if constexpr (sizeof(T) == sizeof(float)) {
        // delta = (R^2 - d^2) / (R + d): the cancellation happens in the
        // double difference of squares; the quotient needs only float d.
        const float df = __builtin_amdgcn_sqrtf((float)d2);
        const float inv_d = __builtin_amdgcn_rcpf(df);
        nh[0] = (float)d0 * inv_d;
        nh[1] = (float)d1 * inv_d;
        nh[2] = (float)d2c * inv_d;
        double dsq;
        {
#pragma clang fp contract(off)
            dsq = R * R - d2;
        }
        delta = (float)dsq * __builtin_amdgcn_rcpf((float)R + df);
    } else {
        const double d = sqrt(d2);
        const double inv_d = 1.0 / d;
        nh[0] = d0 * inv_d;
        nh[1] = d1 * inv_d;
        nh[2] = d2c * inv_d;
        delta = R - d;
    }
    const T w[3] = {(T)(vi[0] - p.v[0]), (T)(vi[1] - p.v[1]), (T)(vi[2] - p.v[2])};
    const T mj = WET ? (T)mj_d : (T)mass_of(P, rj);
    const T mit = (T)mi;
    const T meff = law_div(mit * mj, mit + mj);
    T Fp[3];
    pair_force<T>(P, nh, delta, w, meff, Fp);
    acc[0] += Fp[0];
    acc[1] += Fp[1];
    acc[2] += Fp[2];
}

// Wall forces of Eq. (1a)-(1c) with the box faces as infinite-mass partners.
template <typename T>
__device__ inline void add_walls(const DevParams &P, const double xi[3], const double vi[3], double ri, double mi,
                                 T acc[3], int32_t &cnt)
{
    if (!P.walls) return;
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

// Exact contact test of Sec. 3.1 against partner j (state p) and, if the
// two touch, the pair force added to acc (returns 1 for a contact).  With
// moisture ratios (CAP) a pair that does not touch gets the
// capillary force of its liquid bridge instead (Sec. 5.4).
template <typename T, bool CAP>
__device__ inline int exact_pair(const DevParams &P, const double xi[3], const double vi[3], double ri, double mi,
                                 int64_t q, int32_t j, const Partner &p, T sri, const T *__restrict__ sr,
                                 const double *__restrict__ held, T acc[3])
{
    if (j == q) return 0;
    const double dx[3] = {xi[0] - p.x[0], xi[1] - p.x[1], xi[2] - p.x[2]};
    double d2;
    if (touching(dx[0], dx[1], dx[2], ri + p.r, d2)) {
        if (d2 == 0.0) return 0;
        if constexpr (CAP) {
            // a wet partner's mass includes the water it holds (Eq. 19)
            const double mj = held ? wet_mass(P, p.r, held[j]) : mass_of(P, p.r);
            pair_from<T, true>(P, xi, vi, ri, mi, p, mj, acc);
        } else {
            pair_from<T>(P, xi, vi, ri, mi, p, 0.0, acc);
        }
        return 1;
    }
    if (CAP) capillary_pair<T>(P, dx, d2, ri, p.r, sri, sr[j], acc);
    return 0;
}

// Contact force on granule q reading its candidates from global memory, in
// two passes: the candidate pass runs only the double contact test and lists
// touching partners in `plist` (kMaxPartners x 256 ints in LDS, column tid);
// the force pass then evaluates the pair law for the listed partners in
// canonical order.  Lanes of a wave touch partners at different candidate
// positions, so evaluating forces inside the candidate loop would run the
// expensive branch for almost every candidate.  A granule with more
// partners than the list holds walks its candidates in canonical order.
template <typename T, bool CAP>
__device__ inline void contact_global(const DevParams &P, int64_t n, const double *__restrict__ x,
                                      const double *__restrict__ v, const double *__restrict__ r,
                                      const int32_t *__restrict__ cb, const int32_t *__restrict__ ce, int64_t q,
                                      int32_t *plist, int tid, const T *__restrict__ sr,
                                      const double *__restrict__ held, T *__restrict__ F,
                                      int32_t *__restrict__ ncont, int64_t *err)
{
    const double xi[3] = {x[q], x[n + q], x[2 * n + q]};
    const double vi[3] = {v[q], v[n + q], v[2 * n + q]};
    const double ri = r[q];
    if (ri > P.r_max) raise_error(err, kErrRange, q);
    const double mi = (CAP && held) ? wet_mass(P, ri, held[q]) : mass_of(P, ri);
    const double reach = CAP ? P.dr_max : 0.0;  // liquid bridges reach beyond contact
    const T sri = CAP ? sr[q] : (T)0;
    const double Rs = (ri + P.r_max + reach) * P.search_scale;
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) search_range(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
    T acc[3] = {(T)0, (T)0, (T)0};
    int32_t cnt = 0, nc = 0;
    for_each_run(P, n, lo, hi, cb, ce, [&](int32_t jb, int32_t je) {
        for (int32_t j0 = jb; j0 < je; j0 += kUnroll) {
            double cx[kUnroll], cy[kUnroll], cz[kUnroll], cr[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int32_t j = j0 + u < je ? j0 + u : je - 1;  // in range; duplicates skipped below
                cx[u] = x[j];
                cy[u] = x[n + j];
                cz[u] = x[2 * n + j];
                cr[u] = r[j];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int32_t j = j0 + u;
                if (j >= je || j == q) continue;
                double d2;
                if (!touching(xi[0] - cx[u], xi[1] - cy[u], xi[2] - cz[u], ri + cr[u] + reach, d2) || d2 == 0.0)
                    continue;
                if (cnt < kMaxPartners) plist[cnt * 256 + tid] = j;
                ++cnt;
            }
        }
    });
    if (cnt <= kMaxPartners) {
        canon_sort(plist + tid, 256, cnt, q, [](int32_t j) { return (int64_t)j; });
        for (int k = 0; k < cnt; ++k) {
            const int32_t j = plist[k * 256 + tid];
            nc += exact_pair<T, CAP>(P, xi, vi, ri, mi, q, j, fetch_partner(n, x, v, r, j), sri, sr, held, acc);
        }
    } else {  // rare: more partners than the list holds
        for_each_canonical(P, n, q, lo, hi, cb, ce, [&](int32_t j) {
            nc += exact_pair<T, CAP>(P, xi, vi, ri, mi, q, j, fetch_partner(n, x, v, r, j), sri, sr, held, acc);
        });
    }
    add_walls<T>(P, xi, vi, ri, mi, acc, nc);
    F[q] = acc[0];
    F[n + q] = acc[1];
    F[2 * n + q] = acc[2];
    if (ncont) ncont[q] = nc;
}

// ---------------------------------------------------------------------------
// LDS-staged contact: one workgroup per brick of 4x4x4 cells.  The 6x6x6
// cells around the brick (the brick and a one-cell shell) are copied once
// into LDS, cell after cell in (z, y, x) order, kPad empty slots (never a
// candidate) after each cell; consecutive cells of a row stay one
// contiguous range of slots.
//
// A slot holds, in single precision, the granule's position p relative to
// the brick's centre and Q = |p|^2 - 2 r^2 (16 bytes, one LDS read per
// candidate).  For granule i at a (relative) with b_i = |a|^2 - 2 r_i^2,
//     b_i + Q_j - 2 a.p_j = |x_i - x_j|^2 - 2 r_i^2 - 2 r_j^2
//                        <= |x_i - x_j|^2 - (r_i + r_j)^2
// because 2 r_i r_j <= r_i^2 + r_j^2 (equality for equal radii), so the
// candidate pass keeps j when Q_j - 2 a.p_j < M - b_i: three FMAs and a
// compare per candidate, and every touching pair passes as long as the
// single-precision evaluation errs by less than M.  The force pass then
// runs the exact double test of Sec. 3.1 on the listed partners (from
// global memory, as the force needs their double state anyway) and
// evaluates Eq. (1) for those that touch.
//
// Margin: relative coordinates lie within 3 cells of the centre per axis
// (the own granule's within 2) and radii are at most half a cell, so Q is
// below 27 cell^2, b_i below 12 cell^2 and every partial sum of the FMA
// chain below 63 cell^2; the roundings of Q, b_i, M - b_i and the chain
// (12 of at most 2^-24 of those bounds) sum to less than 2^-15.5 cell^2,
// and rounding the positions and radii to float moves the exact value by
// less than 2^-16.7 cell^2.  M = 2^-12 cell^2, eight times the total.  (For
// positions outside the box, which the key kernel reports as a domain
// error, the bound does not hold and the step's result is unspecified.)
//
// A brick whose shell does not fit in LDS takes the global path.
constexpr int kHaloCells = 216;
constexpr int kLdsPartners = 10;
constexpr int kCand = 4;  // candidates read from LDS before they are tested
constexpr int kPad = 1;   // empty slots after each cell
constexpr int kCopyRounds = 8;  // shell copy rounds of 256 slots: covers every cap <= 2047

// Fixed compare-exchange networks sorting 4, 6, 8 and 10 entries (5, 12,
// 19 and 29 comparators, the least known for those sizes).
constexpr int kNet4[5][2] = {{0, 2}, {1, 3}, {0, 1}, {2, 3}, {1, 2}};
constexpr int kNet6[12][2] = {{0, 5}, {1, 3}, {2, 4}, {1, 2}, {3, 4}, {0, 3},
                              {2, 5}, {0, 1}, {2, 3}, {4, 5}, {1, 2}, {3, 4}};
constexpr int kNet8[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {0, 1}, {2, 3},
                              {4, 5}, {6, 7}, {2, 4}, {3, 5}, {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
constexpr int kNet10[29][2] = {{0, 8}, {1, 9}, {2, 7}, {3, 5}, {4, 6}, {0, 2}, {1, 4}, {5, 8}, {7, 9}, {0, 3},
                               {2, 4}, {5, 7}, {6, 9}, {0, 1}, {3, 6}, {8, 9}, {1, 5}, {2, 3}, {4, 8}, {6, 7},
                               {1, 2}, {3, 5}, {4, 6}, {7, 8}, {2, 3}, {4, 5}, {6, 7}, {3, 4}, {5, 6}};

template <int C>
__device__ inline void run_net(const int (&net)[C][2], uint32_t key[], uint32_t sl[])
{
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = net[c][0], b = net[c][1];
        const bool sw = key[b] < key[a];
        const uint32_t ka = sw ? key[b] : key[a], kb = sw ? key[a] : key[b];
        const uint32_t sa = sw ? sl[b] : sl[a], sb = sw ? sl[a] : sl[b];
        key[a] = ka;
        key[b] = kb;
        sl[a] = sa;
        sl[b] = sb;
    }
}

// The listed slots of granule q (plist column, m <= kLdsPartners entries)
// into canonical order: a 32-bit key per entry, 2 |j - q| plus 1 above q
// (a distance holds at most the two positions q - d and q + d, so the key
// orders by distance, the lower position first), sorted in registers by the
// smallest network that covers the longest list in the wave (none when no
// list has two entries), written back.
template <typename J>
__device__ inline void lds_list_canonical(uint16_t *col, int m, int64_t q, J &&j_of)
{
    static_assert(kLdsPartners == 10, "the networks sort up to ten entries");
    if (__ballot(m >= 2) == 0ull) return;
    uint32_t key[kLdsPartners];
    uint32_t sl[kLdsPartners];
#pragma unroll
    for (int i = 0; i < kLdsPartners; ++i) {
        key[i] = 0xFFFFFFFFu;  // past the last entry: sorts last
        sl[i] = 0;
        if (i < m) {
            sl[i] = col[i * 256];
            const int64_t j = j_of((int)sl[i]);
            key[i] = j > q ? (uint32_t)(2 * (j - q) + 1) : (uint32_t)(2 * (q - j));
        }
    }
    if (__ballot(m > 8) != 0ull)
        run_net(kNet10, key, sl);
    else if (__ballot(m > 6) != 0ull)
        run_net(kNet8, key, sl);
    else if (__ballot(m > 4) != 0ull)
        run_net(kNet6, key, sl);
    else
        run_net(kNet4, key, sl);
#pragma unroll
    for (int i = 0; i < kLdsPartners; ++i)
        if (i < m) col[i * 256] = (uint16_t)sl[i];
}

// Candidate test of the LDS pass (see above): p = (p, Q) of a slot,
// m = -2 a, thr = M - b_i.
__device__ inline bool near_slot(float4 p, float mx, float my, float mz, float thr)
{
    return fmaf(mx, p.x, fmaf(my, p.y, fmaf(mz, p.z, p.w))) < thr;
}

// The bridge-force instantiation is held to four waves per SIMD: it needs
// one register more than 128 and spills three.  The dry instantiation
// serves beds whose neighbour list could never be kept (no skin: cells of
// exactly 2 r_max), where building a list every step costs more.
template <typename T, bool CAP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CAP ? 4 : 1)))
k_contact_lds(DevParams P, int64_t n, const int32_t *__restrict__ bl,
                                                     const int32_t *__restrict__ bcnt, int cap,
                                                     const double *__restrict__ x, const double *__restrict__ v,
                                                     const double *__restrict__ r, const int32_t *__restrict__ cb,
                                                     const int32_t *__restrict__ ce, const T *__restrict__ sr,
                                                     const double *__restrict__ held, T *__restrict__ F,
                                                     int32_t *__restrict__ ncont, int64_t *err,
                                                     int32_t *__restrict__ hmax, int32_t *__restrict__ hclr)
{
    extern __shared__ float4 smem4[];
    float4 *spos = smem4;                                        // [cap + kCand] (p, Q), see above
    uint16_t *plist = reinterpret_cast<uint16_t *>(spos + cap + kCand);  // [kLdsPartners][256] partner slots
    int32_t *clo = reinterpret_cast<int32_t *>(plist + kLdsPartners * 256);  // [216] first slot of each cell
    int32_t *cnum = clo + kHaloCells;                                      // [216] granules of each shell cell
    int32_t *cgb = cnum + kHaloCells;                                      // [216] global begin of each shell cell
    int32_t *s_wave = cgb + kHaloCells;                                    // [4]
    uint8_t *scell = reinterpret_cast<uint8_t *>(s_wave + 4);              // [cap] shell cell of each slot
    const int tid = threadIdx.x;
    if (hclr && blockIdx.x == 0 && tid == 0) *hclr = 0;  // the next recording call's record
    const int64_t b = brick_of_block(bl, bcnt);
    if (b < 0) return;
    const int32_t bc[3] = {(int32_t)(b % P.nb[0]), (int32_t)((b / P.nb[0]) % P.nb[1]),
                           (int32_t)(b / ((int64_t)P.nb[0] * P.nb[1]))};
    const int32_t c0[3] = {bc[0] * kBrick - 1, bc[1] * kBrick - 1, bc[2] * kBrick - 1};  // shell origin cell
    int32_t gb = cb[b * kBrickCells], ge = ce[b * kBrickCells + kBrickCells - 1];
    clip_range(n, gb, ge);
    if (ge <= gb) return;
    const double o[3] = {(c0[0] + 3) * P.cell, (c0[1] + 3) * P.cell, (c0[2] + 3) * P.cell};  // brick centre
    // ---- shell cells: counts, then slots (count + kPad each) by a scan
    int32_t num = 0, gbeg = 0;
    if (tid < kHaloCells) {
        const int hx = tid % 6, hy = (tid / 6) % 6, hz = tid / 36;
        const int32_t cx = c0[0] + hx, cy = c0[1] + hy, cz = c0[2] + hz;
        if (cx >= 0 && cy >= 0 && cz >= 0 && cx < P.nc[0] && cy < P.nc[1] && cz < P.nc[2]) {
            const uint32_t k = key_of_cell(P, cx, cy, cz);
            int32_t e = ce[k];
            gbeg = cb[k];
            clip_range(n, gbeg, e);
            num = e - gbeg;
        }
    }
    const int32_t slots = tid < kHaloCells ? num + kPad : 0;
    int32_t first = 0;
    {
        const int lane = tid & 63, wave = tid >> 6;
        int32_t incl = slots;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        int32_t before = 0;
        for (int w = 0; w < wave; ++w) before += s_wave[w];
        first = before + incl - slots;
        if (tid < kHaloCells) {
            clo[tid] = first;
            cnum[tid] = num;
            cgb[tid] = gbeg;
        }
    }
    const int32_t H = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    // the largest shell (an atomic only when this one is larger than the record)
    if (hmax && tid == 0 && H > __hip_atomic_load(hmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(hmax, H);
    if (H > cap) {  // shell too large for LDS: global candidate path for this brick
        __syncthreads();  // every thread has read s_wave
        int32_t *glist = reinterpret_cast<int32_t *>(smem4);  // the slot arrays are unused on this path
        for (int64_t q = gb + tid; q < ge; q += 256)
            contact_global<T, CAP>(P, n, x, v, r, cb, ce, q, glist, tid, sr, held, F, ncont, err);
        return;
    }
    // ---- slot -> shell cell map (pads take their cell's number too)
    if (tid < kHaloCells)
        for (int32_t k = first; k < first + slots; ++k) scell[k] = (uint8_t)tid;
    __syncthreads();
    // with liquid bridges the candidate pass looks d_r further: each radius
    // grows by d_r / 2 in Q and b_i, so r_i + r_j grows by d_r
    const float hreach = CAP ? (float)(0.5 * P.dr_max) : 0.0f;
    // ---- copy the shell's granules, relative to the centre, in single precision.
    // H <= cap < kCopyRounds * 256: all loads of a thread are issued before
    // any of them is used, so they are in flight together.
    {
        double gx[kCopyRounds], gy[kCopyRounds], gz[kCopyRounds], gr[kCopyRounds];
        bool real[kCopyRounds];
#pragma unroll
        for (int it = 0; it < kCopyRounds; ++it) {
            const int k = tid + it * 256;
            real[it] = false;
            gx[it] = gy[it] = gz[it] = gr[it] = 0.0;
            if (k < H) {
                const int c = scell[k];
                const int off = k - clo[c];
                if (off < cnum[c]) {
                    const int64_t g = cgb[c] + off;
                    gx[it] = x[g];
                    gy[it] = x[n + g];
                    gz[it] = x[2 * n + g];
                    gr[it] = r[g];
                    real[it] = true;
                }
            }
        }
#pragma unroll
        for (int it = 0; it < kCopyRounds; ++it) {
            const int k = tid + it * 256;
            if (k >= H) continue;
            float4 p;
            if (real[it]) {
                const float px = (float)(gx[it] - o[0]), py = (float)(gy[it] - o[1]), pz = (float)(gz[it] - o[2]);
                const float rg = (float)gr[it] + hreach;
                p = make_float4(px, py, pz, ((px * px + py * py) + pz * pz) - 2.0f * (rg * rg));
            } else {
                const float nan = __builtin_nanf("");
                p = make_float4(nan, nan, nan, nan);
            }
            spos[k] = p;
        }
    }
    __syncthreads();
    const float M = (float)(P.cell * P.cell * (1.0 / 4096.0));
    // ---- granules of the brick, one thread each: the listed partners are
    // evaluated in canonical order, the order of the dry contact's
    // neighbour list, so a bed without bridges gives the dry contact's bits
    constexpr int L = 1;
    constexpr int sub = 0;
    for (int64_t qb = gb; qb < ge; qb += 256) {  // same trip count in every lane
        const int64_t q = qb + tid;
        const bool live = q < ge;
        T acc[3] = {(T)0, (T)0, (T)0};
        int32_t nc = 0;
        bool bad = false;
        double xi[3] = {0.0, 0.0, 0.0}, vi[3] = {0.0, 0.0, 0.0}, ri = 0.0, mi = 0.0;
        if (live) {
            xi[0] = x[q];
            xi[1] = x[n + q];
            xi[2] = x[2 * n + q];
            ri = r[q];
            if (ri > P.r_max) raise_error(err, kErrRange, q);
            const float ax = (float)(xi[0] - o[0]), ay = (float)(xi[1] - o[1]), az = (float)(xi[2] - o[2]);
            const float rf = (float)ri + hreach;
            const float thr = M - (((ax * ax + ay * ay) + az * az) - 2.0f * (rf * rf));
            const float mx = -2.0f * ax, my = -2.0f * ay, mz = -2.0f * az;
            const double Rs = (ri + P.r_max + (CAP ? P.dr_max : 0.0)) * P.search_scale;
            int32_t lo[3], hi[3], ca[3];
            for (int a = 0; a < 3; ++a) {
                ca[a] = cell_coord(xi[a], P.inv_cell, P.nc[a]) - c0[a];  // in [1, 4]: q lies in the brick
                search_range(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
                lo[a] -= c0[a];
                hi[a] -= c0[a];
            }
            // the cell ranges do not match the positions (not the ranges of this state's sort)
            bad = ca[0] < 1 || ca[0] > 4 || ca[1] < 1 || ca[1] > 4 || ca[2] < 1 || ca[2] > 4;
            if (bad) {
                raise_error(err, kErrRange, q);
            } else {
                // slot of q itself, skipped by the candidate pass (the exact test skips q too)
                const int own = (ca[2] * 6 + ca[1]) * 6 + ca[0];
                const int32_t qoff = (int32_t)(q - cgb[own]);
                const int32_t kself = qoff >= 0 && qoff < cnum[own] ? clo[own] + qoff : -1;
                // this lane's rows (hz, hy) of the search box, f(first cell of the row)
                auto for_rows = [&](auto &&f) {
                    const int ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
                    if (ny <= 0 || nz <= 0) return;  // empty box (a NaN or negative radius): no rows
                    const int nrow = nz * ny;
                    int hz = lo[2], hy = lo[1] + sub;
                    while (hy > hi[1]) { hy -= ny; ++hz; }
                    for (int row = sub; row < nrow; row += L) {
                        f((hz * 6 + hy) * 6);
                        hy += L;
                        while (hy > hi[1]) { hy -= ny; ++hz; }
                    }
                };
                int32_t cnt = 0;
                for_rows([&](int c) {
                    // cells lo..hi of this row: one contiguous run of slots
                    const int k0 = clo[c + lo[0]];
                    const int k1 = clo[c + hi[0]] + cnum[c + hi[0]];
                    for (int k = k0; k < k1; k += kCand) {
                        // slots up to k1 + kCand - 2 < cap + kCand are read; those past k1 are ignored
                        float4 p[kCand];
#pragma unroll
                        for (int u = 0; u < kCand; ++u) p[u] = spos[k + u];
#pragma unroll
                        for (int u = 0; u < kCand; ++u) {
                            if (k + u < k1 && k + u != kself && near_slot(p[u], mx, my, mz, thr)) {
                                if (cnt < kLdsPartners) plist[cnt * 256 + tid] = (uint16_t)(k + u);
                                ++cnt;
                            }
                        }
                    }
                });
                auto global_of = [&](int k) { const int c = scell[k]; return (int64_t)cgb[c] + (k - clo[c]); };
                if (cnt <= kLdsPartners) lds_list_canonical(plist + tid, cnt, q, global_of);
                vi[0] = v[q];
                vi[1] = v[n + q];
                vi[2] = v[2 * n + q];
                mi = (CAP && held) ? wet_mass(P, ri, held[q]) : mass_of(P, ri);
                const T sri = CAP ? sr[q] : (T)0;
                if (cnt <= kLdsPartners) {
                    for (int i = 0; i < cnt; i += 2) {
                        // two partners per round, their loads in flight together
                        const bool two = i + 1 < cnt;
                        const int32_t j0 = (int32_t)global_of(plist[i * 256 + tid]);
                        const int32_t j1 = two ? (int32_t)global_of(plist[(i + 1) * 256 + tid]) : j0;
                        const Partner p0 = fetch_partner(n, x, v, r, j0);
                        const Partner p1 = fetch_partner(n, x, v, r, j1);
                        nc += exact_pair<T, CAP>(P, xi, vi, ri, mi, q, j0, p0, sri, sr, held, acc);
                        if (two) nc += exact_pair<T, CAP>(P, xi, vi, ri, mi, q, j1, p1, sri, sr, held, acc);
                    }
                } else {
                    // more candidates than listed (rare): every granule of the
                    // search box in canonical order, from global memory
                    int32_t glo[3], ghi[3];
                    for (int a = 0; a < 3; ++a) {
                        glo[a] = lo[a] + c0[a];
                        ghi[a] = hi[a] + c0[a];
                    }
                    for_each_canonical(P, n, q, glo, ghi, cb, ce, [&](int32_t j) {
                        nc += exact_pair<T, CAP>(P, xi, vi, ri, mi, q, j, fetch_partner(n, x, v, r, j), sri, sr,
                                                 held, acc);
                    });
                }
            }
        }
        if (live) {
            if (!bad) add_walls<T>(P, xi, vi, ri, mi, acc, nc);
            F[q] = acc[0];
            F[n + q] = acc[1];
            F[2 * n + q] = acc[2];
            if (ncont) ncont[q] = nc;
        }
    }
}

// ---------------------------------------------------------------------------
// Neighbour list.  The list build stages the brick's shell in LDS like the
// contact kernel above, with every radius grown by skin / 2, and keeps every
// shell granule that passes the three-FMA test and then a single-precision
// distance test d^2 < (r_i + r_j + skin)^2 + M (same margin M: the float
// evaluation errs by less than M / 8), so the list holds every pair closer
// than r_i + r_j + skin, in canonical order (canon_before): the touching
// pairs of two lists built from the same sorted order (whatever the
// positions) come in the same order, and the forces summed over them are
// the same bits.
constexpr int kNbrThreads = 256;

// Partners of granule q by a search of its cells in global memory (shells
// that do not fit in LDS), exact double test with the skin; the same order.
__device__ inline int nbr_global(const DevParams &P, int64_t n, const double *__restrict__ x,
                                 const double *__restrict__ r, const int32_t *__restrict__ cb,
                                 const int32_t *__restrict__ ce, int64_t q, const double xi[3], double ri,
                                 double skin, int32_t *__restrict__ nbr)
{
    const double Rs = (ri + P.r_max + skin) * P.search_scale;
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) search_range(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
    int cnt = 0;
    for_each_run(P, n, lo, hi, cb, ce, [&](int32_t jb, int32_t je) {
        for (int32_t j = jb; j < je; ++j) {
            if (j == q) continue;
            double d2;
            if (!touching(xi[0] - x[j], xi[1] - x[n + j], xi[2] - x[2 * n + j], ri + r[j] + skin, d2)) continue;
            if (cnt < kNbrCap) nbr[(int64_t)cnt * n + q] = j;
            ++cnt;
        }
    });
    canon_sort(nbr + q, n, cnt < kNbrCap ? cnt : kNbrCap, q, [](int32_t j) { return (int64_t)j; });
    return cnt;
}

// The list of the granules of brick b (one workgroup; LDS from smem4).
__device__ inline void nbr_build_brick(const DevParams &P, int64_t n, int64_t b, int cap,
                                       const double *__restrict__ x, const double *__restrict__ r,
                                       const int32_t *__restrict__ cb, const int32_t *__restrict__ ce,
                                       int32_t *__restrict__ nbr, int32_t *__restrict__ ncnt,
                                       float *__restrict__ xref, double skin, int64_t *err, float4 *smem4)
{
    float4 *spos = smem4;                                                 // [cap + kCand] (p, Q)
    float *srad = reinterpret_cast<float *>(spos + cap + kCand);          // [cap] radius + skin / 2
    uint16_t *plist = reinterpret_cast<uint16_t *>(srad + cap);           // [kNbrCap][256] listed slots
    int32_t *clo = reinterpret_cast<int32_t *>(plist + kNbrCap * kNbrThreads);  // [216] first slot of each cell
    int32_t *cnum = clo + kHaloCells;                                     // [216] granules of each shell cell
    int32_t *cgb = cnum + kHaloCells;                                     // [216] global begin of each shell cell
    int32_t *s_wave = cgb + kHaloCells;                                   // [4]
    uint8_t *scell = reinterpret_cast<uint8_t *>(s_wave + 4);             // [cap] shell cell of each slot
    const int tid = threadIdx.x;
    const int32_t bc[3] = {(int32_t)(b % P.nb[0]), (int32_t)((b / P.nb[0]) % P.nb[1]),
                           (int32_t)(b / ((int64_t)P.nb[0] * P.nb[1]))};
    const int32_t c0[3] = {bc[0] * kBrick - 1, bc[1] * kBrick - 1, bc[2] * kBrick - 1};
    int32_t gb = cb[b * kBrickCells], ge = ce[b * kBrickCells + kBrickCells - 1];
    clip_range(n, gb, ge);
    if (ge <= gb) return;
    const double o[3] = {(c0[0] + 3) * P.cell, (c0[1] + 3) * P.cell, (c0[2] + 3) * P.cell};
    int32_t num = 0, gbeg = 0;
    if (tid < kHaloCells) {
        const int hx = tid % 6, hy = (tid / 6) % 6, hz = tid / 36;
        const int32_t cx = c0[0] + hx, cy = c0[1] + hy, cz = c0[2] + hz;
        if (cx >= 0 && cy >= 0 && cz >= 0 && cx < P.nc[0] && cy < P.nc[1] && cz < P.nc[2]) {
            const uint32_t k = key_of_cell(P, cx, cy, cz);
            int32_t e = ce[k];
            gbeg = cb[k];
            clip_range(n, gbeg, e);
            num = e - gbeg;
        }
    }
    const int32_t slots = tid < kHaloCells ? num + kPad : 0;
    int32_t first = 0;
    {
        const int lane = tid & 63, wave = tid >> 6;
        int32_t incl = slots;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        int32_t before = 0;
        for (int w = 0; w < wave; ++w) before += s_wave[w];
        first = before + incl - slots;
        if (tid < kHaloCells) {
            clo[tid] = first;
            cnum[tid] = num;
            cgb[tid] = gbeg;
        }
    }
    const int32_t H = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    if (H > cap) {  // shell too large for LDS: search the cells in global memory
        for (int64_t q = gb + tid; q < ge; q += kNbrThreads) {
            const double xi[3] = {x[q], x[n + q], x[2 * n + q]};
            const double ri = r[q];
            if (ri > P.r_max) raise_error(err, kErrRange, q);
            ncnt[q] = nbr_global(P, n, x, r, cb, ce, q, xi, ri, skin, nbr);
            for (int a = 0; a < 3; ++a) xref[a * n + q] = (float)xi[a];
        }
        return;
    }
    if (tid < kHaloCells)
        for (int32_t k = first; k < first + slots; ++k) scell[k] = (uint8_t)tid;
    __syncthreads();
    const float hskin = (float)(0.5 * skin);
    {
        double gx[kCopyRounds], gy[kCopyRounds], gz[kCopyRounds], gr[kCopyRounds];
        bool real[kCopyRounds];
#pragma unroll
        for (int it = 0; it < kCopyRounds; ++it) {
            const int k = tid + it * kNbrThreads;
            real[it] = false;
            gx[it] = gy[it] = gz[it] = gr[it] = 0.0;
            if (k < H) {
                const int c = scell[k];
                const int off = k - clo[c];
                if (off < cnum[c]) {
                    const int64_t g = cgb[c] + off;
                    gx[it] = x[g];
                    gy[it] = x[n + g];
                    gz[it] = x[2 * n + g];
                    gr[it] = r[g];
                    real[it] = true;
                }
            }
        }
#pragma unroll
        for (int it = 0; it < kCopyRounds; ++it) {
            const int k = tid + it * kNbrThreads;
            if (k >= H) continue;
            float4 p;
            float rg = 0.0f;
            if (real[it]) {
                const float px = (float)(gx[it] - o[0]), py = (float)(gy[it] - o[1]), pz = (float)(gz[it] - o[2]);
                rg = (float)gr[it] + hskin;
                p = make_float4(px, py, pz, ((px * px + py * py) + pz * pz) - 2.0f * (rg * rg));
            } else {
                const float nan = __builtin_nanf("");
                p = make_float4(nan, nan, nan, nan);
            }
            spos[k] = p;
            srad[k] = rg;
        }
    }
    __syncthreads();
    const float M = (float)(P.cell * P.cell * (1.0 / 4096.0));
    for (int64_t q = gb + tid; q < ge; q += kNbrThreads) {
        const double xi[3] = {x[q], x[n + q], x[2 * n + q]};
        const double ri = r[q];
        if (ri > P.r_max) raise_error(err, kErrRange, q);
        for (int a = 0; a < 3; ++a) xref[a * n + q] = (float)xi[a];
        const float ax = (float)(xi[0] - o[0]), ay = (float)(xi[1] - o[1]), az = (float)(xi[2] - o[2]);
        const float rf = (float)ri + hskin;
        const float thr = M - (((ax * ax + ay * ay) + az * az) - 2.0f * (rf * rf));
        const float mx = -2.0f * ax, my = -2.0f * ay, mz = -2.0f * az;
        const double Rs = (ri + P.r_max + skin) * P.search_scale;
        int32_t lo[3], hi[3], ca[3];
        for (int a = 0; a < 3; ++a) {
            ca[a] = cell_coord(xi[a], P.inv_cell, P.nc[a]) - c0[a];
            search_range(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
            lo[a] -= c0[a];
            hi[a] -= c0[a];
        }
        if (ca[0] < 1 || ca[0] > 4 || ca[1] < 1 || ca[1] > 4 || ca[2] < 1 || ca[2] > 4) {
            // the cell ranges do not match the positions
            raise_error(err, kErrRange, q);
            ncnt[q] = 0;
            continue;
        }
        const int own = (ca[2] * 6 + ca[1]) * 6 + ca[0];
        const int32_t qoff = (int32_t)(q - cgb[own]);
        const int kself = qoff >= 0 && qoff < cnum[own] ? clo[own] + qoff : -1;
        int32_t cnt = 0;
        for (int hz = lo[2]; hz <= hi[2]; ++hz)
            for (int hy = lo[1]; hy <= hi[1]; ++hy) {
                const int c = (hz * 6 + hy) * 6;
                const int k0 = clo[c + lo[0]];
                const int k1 = clo[c + hi[0]] + cnum[c + hi[0]];
                for (int k = k0; k < k1; k += kCand) {
                    float4 p[kCand];
#pragma unroll
                    for (int u = 0; u < kCand; ++u) p[u] = spos[k + u];
#pragma unroll
                    for (int u = 0; u < kCand; ++u) {
                        if (k + u >= k1 || k + u == kself || !near_slot(p[u], mx, my, mz, thr)) continue;
                        const float ex = ax - p[u].x, ey = ay - p[u].y, ez = az - p[u].z;
                        const float rs = rf + srad[k + u];
                        if (!(((ex * ex + ey * ey) + ez * ez) < rs * rs + M)) continue;
                        if (cnt < kNbrCap) plist[cnt * kNbrThreads + tid] = (uint16_t)(k + u);
                        ++cnt;
                    }
                }
            }
        ncnt[q] = cnt;
        const int listed = cnt < kNbrCap ? cnt : kNbrCap;
        auto j_of = [&](int slot) { const int c = scell[slot]; return (int64_t)cgb[c] + (slot - clo[c]); };
        canon_sort(plist + tid, kNbrThreads, listed, q, j_of);
        for (int k = 0; k < listed; ++k) nbr[(int64_t)k * n + q] = (int32_t)j_of(plist[k * kNbrThreads + tid]);
    }
}

// Builds the list when asked (force, or ctl[0] set by the sort); a small
// grid loops over the occupied bricks, so the launch costs little when the
// list is kept.
__global__ void __launch_bounds__(kNbrThreads) k_nbr_build(DevParams P, int64_t n, const int32_t *__restrict__ bl,
                                                           const int32_t *__restrict__ bcnt, int cap,
                                                           const double *__restrict__ x, const double *__restrict__ r,
                                                           const int32_t *__restrict__ cb,
                                                           const int32_t *__restrict__ ce, int32_t *__restrict__ nbr,
                                                           int32_t *__restrict__ ncnt, float *__restrict__ xref,
                                                           uint32_t *__restrict__ ctl, int force, double skin,
                                                           int64_t *err)
{
    if (!force && !ctl[0]) return;  // the list of the last build still holds every pair that can touch
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctl[2], 1u);  // builds, for the caller's statistics
    extern __shared__ float4 smem4[];
    for (int64_t it = 0;; ++it) {
        const int64_t b = brick_at(bl, bcnt, it);
        if (b < 0) break;
        nbr_build_brick(P, n, b, cap, x, r, cb, ce, nbr, ncnt, xref, skin, err, smem4);
        __syncthreads();  // the next brick reuses the LDS
    }
}

// Contact forces from the neighbour list: one thread per granule in sorted
// order (each XCD one contiguous eighth, so partners mostly share its L2).
// The workgroup first copies the double state of its own granules into
// LDS with coalesced loads; a listed partner among them (the granules of the
// same few cells) is read from there, any other from global memory, two
// partners' state fetched together so their loads overlap.  The list's
// canonical order puts each granule's nearest sorted positions first, which
// lie in the workgroup, so the global partners of a wave gather in the
// last few list places and in like directions: fewer load instructions
// issue, and they touch fewer cache lines.  (A wider window of sorted
// positions in LDS served more partners but lowered the waves per SIMD,
// which cost more.)  Each listed partner runs the exact test of Sec. 3.1
// and, if touching, Eq. (1); walls last.  A granule whose partners did not
// fit in its list walks its cells' granules in the same order.
constexpr int kListBatch = 2;
constexpr int kListThreads = 256;  // granules (threads) per workgroup

template <typename T>
__global__ void __launch_bounds__(kListThreads) k_contact_list(DevParams P, int64_t n, int64_t nblk,
                                                      const double *__restrict__ x, const double *__restrict__ v,
                                                      const double *__restrict__ r, const int32_t *__restrict__ cb,
                                                      const int32_t *__restrict__ ce,
                                                      const int32_t *__restrict__ nbr,
                                                      const int32_t *__restrict__ ncnt, T *__restrict__ F,
                                                      int32_t *__restrict__ ncont, int32_t *__restrict__ pairs,
                                                      int pair_cap, int64_t *err)
{
    __shared__ double sw[7][kListThreads];  // x0, x1, x2, v0, v1, v2, r of the workgroup's granules
    const int64_t lb = xcd_block(nblk);
    if (lb < 0) return;
    const int64_t wbeg = lb * kListThreads;
    const int32_t wlen = (int32_t)(n - wbeg < kListThreads ? n - wbeg : kListThreads);
    for (int32_t i = threadIdx.x; i < wlen; i += kListThreads) {
        const int64_t g = wbeg + i;
        sw[0][i] = x[g];
        sw[1][i] = x[n + g];
        sw[2][i] = x[2 * n + g];
        sw[3][i] = v[g];
        sw[4][i] = v[n + g];
        sw[5][i] = v[2 * n + g];
        sw[6][i] = r[g];
    }
    __syncthreads();
    // a partner's state from LDS, or from global memory
    auto partner = [&](int32_t j) {
        const uint32_t w = (uint32_t)((int64_t)j - wbeg);
        if (w < (uint32_t)wlen) {
            Partner p;
            p.x[0] = sw[0][w];
            p.x[1] = sw[1][w];
            p.x[2] = sw[2][w];
            p.v[0] = sw[3][w];
            p.v[1] = sw[4][w];
            p.v[2] = sw[5][w];
            p.r = sw[6][w];
            return p;
        }
        return fetch_partner(n, x, v, r, j);
    };
    const int64_t q = wbeg + threadIdx.x;
    if (q >= n) return;
    const int32_t qw = (int32_t)(q - wbeg);
    const double xi[3] = {sw[0][qw], sw[1][qw], sw[2][qw]};
    const double vi[3] = {sw[3][qw], sw[4][qw], sw[5][qw]};
    const double ri = sw[6][qw];
    const int32_t cnt = ncnt[q];
    if (ri > P.r_max) raise_error(err, kErrRange, q);
    const double mi = mass_of(P, ri);
    T acc[3] = {(T)0, (T)0, (T)0};
    int32_t nc = 0, np = 0;
    auto take = [&](int32_t j, const Partner &p) {
        if (exact_pair<T, false>(P, xi, vi, ri, mi, q, j, p, (T)0, nullptr, nullptr, acc)) {
            ++nc;
            if (pairs && np < pair_cap) pairs[(int64_t)np * n + q] = j;
            ++np;
        }
    };
    if (cnt <= kNbrCap) {
        for (int k = 0; k < cnt; k += kListBatch) {
            int32_t j[kListBatch];
            Partner p[kListBatch];
#pragma unroll
            for (int u = 0; u < kListBatch; ++u) {
                const int32_t jj = k + u < cnt ? nbr[(int64_t)(k + u) * n + q] : -1;
                j[u] = (uint32_t)jj < (uint32_t)n ? jj : -1;  // a list entry outside [0, n) is skipped
            }
#pragma unroll
            for (int u = 0; u < kListBatch; ++u) p[u] = partner(j[u] >= 0 ? j[u] : (int32_t)q);
#pragma unroll
            for (int u = 0; u < kListBatch; ++u)
                if (j[u] >= 0) take(j[u], p[u]);
        }
    } else {
        const double Rs = (ri + P.r_max) * P.search_scale;
        int32_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) search_range(P, xi[a], Rs, P.nc[a], lo[a], hi[a]);
        for_each_canonical(P, n, q, lo, hi, cb, ce, [&](int32_t jj) { take(jj, partner(jj)); });
    }
    add_walls<T>(P, xi, vi, ri, mi, acc, nc);
    F[q] = acc[0];
    F[n + q] = acc[1];
    F[2 * n + q] = acc[2];
    if (ncont) ncont[q] = nc;
    if (pairs)
        for (int k = np; k < pair_cap; ++k) pairs[(int64_t)k * n + q] = -1;
}

}  // namespace

// LDS bytes of the staged contact kernel for a shell capacity of cap granules.
static size_t contact_lds_bytes(int cap)
{
    size_t b = (size_t)(cap + kCand) * sizeof(float4) + (size_t)cap + sizeof(uint16_t) * kLdsPartners * 256 +
               sizeof(int32_t) * (kHaloCells * 3 + 4);
    const size_t fallback = sizeof(int32_t) * kMaxPartners * 256;  // list of the global path, aliasing the slots
    return b > fallback ? b : fallback;
}

// Shell slots held in LDS: at most 1,948 (40,908 bytes, four workgroups per
// CU); with a record of the largest shell met, an eighth and 64 slots more
// than it, in steps of 64 (a sparser bed: smaller workgroups, more of them
// per CU; the shells of the c5 bed took the kernel from 2.96 to 1.61 ms).
constexpr int kShellCapMax = 1948;

static int shell_cap(const SizeRecord *ss)
{
    // an earlier call's record (the largest shell, in the first word), or 0
    const int32_t seen = ss && ss->host ? *(volatile const int32_t *)ss->host : 0;
    if (seen <= 0) return kShellCapMax;
    const int64_t want = ((int64_t)seen + seen / 8 + 64 + 63) / 64 * 64;
    return want < kShellCapMax ? (int)want : kShellCapMax;
}

template <typename T>
hipError_t launch_contact(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                          const int32_t *cb, const int32_t *ce, const BrickList &B, const T *sr, const double *held,
                          T *F, int32_t *ncont, int64_t *err, hipStream_t s, SizeRecord *ss)
{
    if (n == 0) return hipSuccess;
    const int64_t nbricks = (int64_t)P.nb[0] * P.nb[1] * P.nb[2];
    const int cap = shell_cap(ss);
    const bool copy = record_copy(ss);  // only these calls record (the stores contend)
    int32_t *hm = copy ? ss->dev + ss->par * kRecSlots : nullptr;
    int32_t *hc = copy ? ss->dev + (ss->par ^ 1) * kRecSlots : nullptr;
    if (sr)
        k_contact_lds<T, true><<<brick_grid(nbricks), 256, contact_lds_bytes(cap), s>>>(
            P, n, B.list, B.count, cap, x, v, r, cb, ce, sr, held, F, ncont, err, hm, hc);
    else
        k_contact_lds<T, false><<<brick_grid(nbricks), 256, contact_lds_bytes(cap), s>>>(
            P, n, B.list, B.count, cap, x, v, r, cb, ce, nullptr, nullptr, F, ncont, err, hm, hc);
    hipError_t e = hipGetLastError();
    if (copy) {
        ss->par ^= 1;
        if (e == hipSuccess) e = hipMemcpyAsync(ss->host, hm, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    }
    return e;
}

template hipError_t launch_contact<float>(const DevParams &, int64_t, const double *, const double *,
                                          const double *, const int32_t *, const int32_t *, const BrickList &,
                                          const float *, const double *, float *, int32_t *, int64_t *,
                                          hipStream_t, SizeRecord *);
template hipError_t launch_contact<double>(const DevParams &, int64_t, const double *, const double *,
                                           const double *, const int32_t *, const int32_t *, const BrickList &,
                                           const double *, const double *, double *, int32_t *, int64_t *,
                                           hipStream_t, SizeRecord *);

// LDS bytes of the neighbour-list build for a shell capacity of cap granules.
static size_t nbr_lds_bytes(int cap)
{
    return (size_t)(cap + kCand) * sizeof(float4) + (size_t)cap * sizeof(float) +
           sizeof(uint16_t) * kNbrCap * kNbrThreads + sizeof(int32_t) * (kHaloCells * 3 + 4) + (size_t)cap;
}

hipError_t launch_nbr_build(const DevParams &P, int64_t n, const double *x, const double *r, const int32_t *cb,
                            const int32_t *ce, const BrickList &B, NbrList &L, int force, int64_t *err,
                            hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t nbricks = (int64_t)P.nb[0] * P.nb[1] * P.nb[2];
    const int cap = 1948;  // shell slots in LDS: 51,772 bytes, three workgroups per CU
    k_nbr_build<<<brick_loop_grid(nbricks), kNbrThreads, nbr_lds_bytes(cap), s>>>(
        P, n, B.list, B.count, cap, x, r, cb, ce, L.nbr, L.cnt, L.xref, L.ctl, force, L.skin, err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_contact_list(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                               const int32_t *cb, const int32_t *ce, const NbrList &L, T *F, int32_t *ncont,
                               int32_t *pairs, int pair_cap, int64_t *err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t nblk = (n + kListThreads - 1) / kListThreads;
    k_contact_list<T><<<xcd_grid(nblk), kListThreads, 0, s>>>(P, n, nblk, x, v, r, cb, ce, L.nbr, L.cnt, F, ncont, pairs,
                                                      pair_cap, err);
    return hipGetLastError();
}

template hipError_t launch_contact_list<float>(const DevParams &, int64_t, const double *, const double *,
                                               const double *, const int32_t *, const int32_t *, const NbrList &,
                                               float *, int32_t *, int32_t *, int, int64_t *, hipStream_t);
template hipError_t launch_contact_list<double>(const DevParams &, int64_t, const double *, const double *,
                                                const double *, const int32_t *, const int32_t *, const NbrList &,
                                                double *, int32_t *, int32_t *, int, int64_t *, hipStream_t);

}  // namespace gic
