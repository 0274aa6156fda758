// Host-side launchers of the gfx950 kernels (one translation unit per stage
// family); the C ABI in gic_api.hip validates arguments and calls these.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gic_device.hpp"

namespace gic {

// Granules whose key changed since the last sort that the incremental path
// takes (more go through the radix passes).
constexpr int kChgCap = 4096;

// Sort scratch owned by a context.
struct SortScratch {
    uint32_t *kA, *kB;
    uint32_t *skeys[2];  // sorted keys; skeys[cur] holds those of the last sort
    int cur;
    int64_t last_n;      // granules of the last sort, -1 before the first
    int32_t *vA, *vB;
    uint32_t *sums;      // 1024 chunk totals of the digit-offset scan
    uint32_t *cnt;       // [K] granules per cell; zero between sorts
    uint64_t *chg;       // [kChgCap] changed granules as (key << 32 | position), in arrival order
    uint64_t *chg_s;     // [kChgCap] the same sorted
    uint32_t *chg_p;     // [kChgCap] their positions sorted
    int32_t *ctl;        // [4] changed count (zero between sorts), path of this sort (1 = incremental),
                         // no key changed (1: order, ranges and bricks of the last sort hold), spare
    int64_t tiles_max;
    int passes;          // 8-bit digit passes over the key bits
    uint32_t *tcnt;      // [256][tiles_max] digit counts, then output offsets, of each tile in a digit pass
    uint32_t *rowtot;    // [256] keys with each digit in a digit pass
};

// Occupied bricks of a set of cell ranges, in brick order (see
// brick_of_block), built by launch_brick_list before the brick kernels.
struct BrickList {
    int32_t *list;     // [nbricks]
    int32_t *count;    // [1]
    uint32_t *sums;    // [<= 1024] block totals
    int32_t *slot_of;  // [nbricks] position of each brick in list, -1 if empty
    int64_t nbricks;
};

// skip (optional): the sort's control words; the list is kept when the sort
// found no changed key (the caller checked that cb, ce are the tables the
// list was built from).
hipError_t launch_brick_list(const int32_t *cb, const int32_t *ce, BrickList &B, hipStream_t s,
                             const int32_t *skip = nullptr);

// Persistent neighbour list of the contact stage (owned by a context): for
// every granule (sorted position q) the sorted positions of the granules
// closer than r_i + r_j + skin when the list was built, in the order of
// their cells (z, then y, then x) and of their positions inside a cell.  The
// contact kernel runs the exact test of Sec. 3.1 on the listed granules
// every step, so the list only has to hold every pair that can touch: it
// stays valid while the sorted order is unchanged and no granule has moved
// by skin / 2 since the build.
constexpr int kNbrCap = 16;  // partners listed per granule; more: the contact kernel searches the cells
struct NbrList {
    int32_t *nbr;   // [kNbrCap][n]: partner k of granule q at k * n + q
    int32_t *cnt;   // [n] partners found (> kNbrCap: not listed, searched)
    float *xref;    // [3][n] positions at the build
    uint32_t *ctl;  // [4] rebuild flag of this step, spare, builds, spare
    float *dpart;   // [n / 256] largest squared displacement since the build per key-kernel workgroup
    double skin;    // reach of the list beyond r_i + r_j [m]
    float thr2;     // squared displacement since the build that calls for a rebuild (< 0: every step)
};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
// Up to this many keys the digit passes take tiles of one key per thread,
// so a small sort still spreads over many workgroups.
constexpr int64_t kSmallSort = (int64_t)1 << 18;
inline int sort_items(int64_t n) { return n <= kSmallSort ? 1 : kSortItems; }
// Tiles of the digit passes for up to n_max keys (the larger of the two tilings).
inline int64_t sort_tiles_max(int64_t n_max)
{
    const int64_t big = (n_max + kSortTile - 1) / kSortTile;
    const int64_t m = n_max < kSmallSort ? n_max : kSmallSort;
    const int64_t small = (m + kSortThreads - 1) / kSortThreads;
    return big > small ? big : small;
}

// nl: the neighbour list of the stepping path, or NULL.  With nl, the key
// kernel also measures every granule's displacement since the list's build
// (x in the order of that build) and the sort decides nl->ctl[0]: rebuild
// when force is set, when the sorted order changes, or when a granule moved
// by more than the list's skin / 2.
// keep_ranges: cell_begin, cell_end hold the ranges of the last sort on S
// (same n); they are then rewritten only if a key changed.
hipError_t launch_sort_cells(const DevParams &P, int64_t n, const double *x, uint32_t *key, int32_t *order,
                             int32_t *cell_begin, int32_t *cell_end, int64_t K, SortScratch &S, int64_t *err,
                             hipStream_t s, const NbrList *nl = nullptr, int force = 1, int keep_ranges = 0);
hipError_t launch_reorder(int64_t n, const int32_t *order, const double *x, const double *v, const double *r,
                          const int32_t *id, double *xo, double *vo, double *ro, int32_t *ido, hipStream_t s);

// The largest size a brick kernel met: dev[2][kRecSlots] (device,
// alternating between recording calls: one records into dev[par] and clears
// dev[par ^ 1]), host[kRecSlots] (pinned: a copy of the record, read by
// later calls without waiting; zeros until the first copy lands).  Only
// every 16th call records and copies (a copy costs a few microseconds of
// the stream).  The direct contact kernel keeps the largest brick shell
// (granule slots, pads included) in the first word (an atomic maximum,
// taken only when the word is smaller); the P2G tile kernel keeps flags of
// the granules of its bricks by steps of 64 (a brick of v granules sets
// flag ceil(v / 64) with a plain store).  The next launches are shaped from
// the record; a brick beyond the shape takes a slower path with the same
// bits, and the calls after adapt.
constexpr int kRecSlots = 64;  // flags of sizes up to 64 (kRecSlots - 1)
struct SizeRecord {
    int32_t *dev;
    int32_t *host;
    int par;
    unsigned calls;
};
// Whether this call copies its record to the host.
inline bool record_copy(SizeRecord *r)
{
    return r && r->host && (r->calls++ & 15u) == 0u;
}
// An upper bound (a multiple of 64) of the largest size in the last copy
// that reached the host (0: none yet).
inline int32_t record_seen(const SizeRecord *r)
{
    if (!r || !r->host) return 0;
    int32_t m = 0;
    for (int i = 0; i < kRecSlots; ++i)
        if (((volatile const int32_t *)r->host)[i]) m = 64 * i;
    return m;
}
// The flag of size v (the last flag for sizes beyond the table).
__host__ __device__ inline int record_flag(int32_t v)
{
    const int32_t f = (v + 63) / 64;
    return f < kRecSlots - 1 ? (f > 0 ? f : 0) : kRecSlots - 1;
}
template <typename T>
hipError_t launch_contact(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                          const int32_t *cb, const int32_t *ce, const BrickList &B, const T *sr, const double *held,
                          T *F, int32_t *ncont, int64_t *err, hipStream_t s, SizeRecord *ss = nullptr);
// Neighbour-list build (only when force is set or the sort asked for it)
// and the contact forces from the list (Sec. 3.1, Eq. 1a-1c, walls).
// pairs (optional, pair_cap x n, column-major): the partners that touch, in
// the order their forces are summed, -1 after the last.
hipError_t launch_nbr_build(const DevParams &P, int64_t n, const double *x, const double *r, const int32_t *cb,
                            const int32_t *ce, const BrickList &B, NbrList &L, int force, int64_t *err,
                            hipStream_t s);
template <typename T>
hipError_t launch_contact_list(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                               const int32_t *cb, const int32_t *ce, const NbrList &L, T *F, int32_t *ncont,
                               int32_t *pairs, int pair_cap, int64_t *err, hipStream_t s);

template <typename T>
hipError_t launch_g2p(const DevParams &P, int64_t n, const double *x, const T *u, const int64_t *afx,
                      const double *are, T *uat, T *af, hipStream_t s);
template <typename T>
hipError_t launch_moisture_ratio(int64_t n, const double *held, const T *af, T *sr, hipStream_t s);
template <typename T>
hipError_t launch_drag(const DevParams &P, int64_t n, const double *r, const double *v, const T *uat, const T *af,
                       T *Fd, hipStream_t s);
template <typename T>
hipError_t launch_integrate(const DevParams &P, int64_t n, const double *r, const T *Fc, const T *Fd, double *x,
                            double *v, hipStream_t s);

// Scratch of the assembled P2G of the stepping path: one node tile (4
// channels) per occupied brick, and the list of granules whose stencil left
// their brick's tile (at most n) with its counter.
struct P2GStore {
    unsigned long long *tiles;  // [occupied bricks][4][tile nodes]
    int32_t *esc;               // [n]
    uint32_t *esc_n;            // [1] granules listed
    const int32_t *cover;       // per axis and node: (brick, node in its tile) twice, -1 for none
    // per node row (j, k) and segment of 4 nodes along x (row-major, (n0 + 3) / 4
    // segments a row): 1 where the grids may hold a nonzero value, i.e. a
    // tile reached the segment at the last assembly or a listed granule was
    // deposited there since; NULL: every node is written
    uint8_t *live;
    int full;  // 1: write every node (the grids hold no earlier assembly's values)
    // the tile kernel's record of the most granules in a brick (max into
    // nrec, clear nclr for the next call); NULL: none
    int32_t *nrec, *nclr;
};
// The table P2GStore::cover for the parameters P (host; 4 (n0 + n1 + n2)
// int32): for node i of axis a, at 4 (n0 + ... + n_{a-1} + i), the bricks
// along the axis whose tile holds the node, with the node's offset in it.
void p2g_cover_table(const DevParams &P, int32_t *out);
// Integrate + P2G of the stepping path (dry, alpha and momentum) in two
// launches: launch_integrate_p2g_store moves the granules and stores each
// occupied brick's tile (listing the granules whose stencil left it);
// launch_p2g_assemble then writes the grids from the tiles (written, not
// added to: alpha and mom need no clearing) and deposits the listed
// granules.  esc_next: the escape counter of the next call, cleared here.
// With st.live and !st.full the grids hold the previous assembly's result
// (and its deposits): segments that no tile reaches now and that were not
// live are zero already and are not written again.
template <typename T>
hipError_t launch_integrate_p2g_store(const DevParams &P, int64_t n, int64_t K, double *x, double *v,
                                      const double *r, const T *Fc, const T *Fd, const int32_t *cb,
                                      const int32_t *ce, const BrickList &B, int64_t *err, hipStream_t s,
                                      const P2GStore &st, SizeRecord *rec = nullptr);
hipError_t launch_p2g_assemble(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                               const BrickList &B, int64_t *alpha, int64_t *mom, int64_t *err, hipStream_t s,
                               const P2GStore &st, uint32_t *esc_next);

hipError_t launch_fill_i64(int64_t *a, int64_t len, hipStream_t s);
hipError_t launch_fill_f64(double *a, int64_t len, hipStream_t s);
hipError_t launch_p2g_fixed(const DevParams &P, int64_t n, int64_t K, const double *x, const double *v,
                            const double *r, const int32_t *cb, const int32_t *ce, const BrickList &B,
                            int64_t *alpha, int64_t *mom, int64_t *err, hipStream_t s);
template <typename T>
hipError_t launch_integrate_p2g(const DevParams &P, int64_t n, int64_t K, double *x, double *v, const double *r,
                                const T *Fc, const T *Fd, const int32_t *cb, const int32_t *ce, const BrickList &B,
                                int64_t *alpha, int64_t *mom, int64_t *err, hipStream_t s,
                                const double *held = nullptr);  // held: water per granule volume (wet mass), or NULL
// Exchange deposit of one sub-step (Sec. 5.2) into the 3 x G int64 grid fs.
template <typename T>
hipError_t launch_exchange_p2g(const DevParams &P, int64_t n, int64_t K, const double *x, const double *r,
                               const T *Fc, const T *Ffl, const int32_t *cb, const int32_t *ce, const BrickList &B,
                               double exsc, int64_t *fs, int64_t *err, hipStream_t s,
                               const double *held = nullptr);  // held: wet mass and volume, or NULL
template <typename T>
hipError_t launch_gather_g2p_fluid(const DevParams &P, int64_t n, int64_t K, const int32_t *order, const double *x,
                                   const double *v, const double *r, const int32_t *id, double *xo, double *vo,
                                   double *ro, int32_t *ido, const T *u, const int64_t *afx, const T *gp,
                                   const T *fa, const int32_t *cb, const int32_t *ce, const BrickList &B, T *Ff,
                                   hipStream_t s, const double *held = nullptr, double *heldo = nullptr);
template <typename T>
hipError_t launch_gather_g2p_drag(const DevParams &P, int64_t n, int64_t K, const int32_t *order, const double *x,
                                  const double *v, const double *r, const int32_t *id, double *xo, double *vo,
                                  double *ro, int32_t *ido, const T *u, const int64_t *afx, const int32_t *cb,
                                  const int32_t *ce, const BrickList &B, T *Fd, T *uat, T *af, hipStream_t s);
// Unquantised P2G (alpha G, momentum 3G doubles; = or += with acc),
// summed deterministically as integers at a scale set by the largest
// contribution; fx: 4 G int64 and part: 4 x 1024 + 8 doubles of scratch.
hipError_t launch_p2g_real(const DevParams &P, int64_t n, int64_t K, const double *x, const double *v,
                           const double *r, const int32_t *cb, const int32_t *ce, const BrickList &B,
                           double *alpha, double *mom, int acc, int64_t *fx, double *part, hipStream_t s);
hipError_t launch_g2p_vjp_grid(const DevParams &P, int64_t n, int64_t K, const double *x, const double *A,
                               const double *gaf, const int32_t *cb, const int32_t *ce, const BrickList &B,
                               double *gA, int64_t *fx, double *part, hipStream_t s);

hipError_t launch_contact_vjp(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                              const int32_t *cb, const int32_t *ce, const double *gF, double *gx, double *gv,
                              double *gmu, hipStream_t s);
hipError_t launch_drag_vjp(const DevParams &P, int64_t n, const double *r, const double *v, const double *uat,
                           const double *af, const double *gF, double *gv, double *guat, double *gaf, double *gcd,
                           hipStream_t s);
hipError_t launch_integrate_vjp(const DevParams &P, int64_t n, const double *r, const double *gx, double *gv,
                                double *gF, hipStream_t s);
hipError_t launch_g2p_vjp(const DevParams &P, int64_t n, int64_t K, const double *x, const double *u,
                          const double *A, const double *guat, const double *gaf, const int32_t *cb,
                          const int32_t *ce, const BrickList &B, double *gx, double *gA, int64_t *fx, double *part,
                          hipStream_t s);
hipError_t launch_p2g_vjp(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                          const double *gA, const double *gP, double *gx, double *gv, hipStream_t s);
hipError_t launch_sum(const double *a, const double *b, int64_t n, double *part, int nparts, double *out, int acc,
                      hipStream_t s);
hipError_t launch_permute(int64_t n, int comps, const int32_t *order, const double *in, double *out, int scatter,
                          hipStream_t s);
hipError_t launch_scale(int64_t n, const double *a, const double *sp, double factor, double *out, hipStream_t s);

inline unsigned grid_for(int64_t n, int threads)
{
    int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace gic
