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
    uint32_t *hist;      // RADIX x tiles
    uint32_t *sums;      // 1024 chunk totals of the digit-offset scan
    uint32_t *cnt;       // [K] granules per cell; zero between sorts
    uint64_t *chg;       // [kChgCap] changed granules as (key << 32 | position), in arrival order
    uint64_t *chg_s;     // [kChgCap] the same sorted
    uint32_t *chg_p;     // [kChgCap] their positions sorted
    int32_t *ctl;        // [2] changed count (zero between sorts), path of this sort (1 = incremental)
    int64_t tiles_max;
    int passes;          // 8-bit digit passes over the key bits
};

// Occupied bricks of a set of cell ranges, in brick order (see
// brick_of_block), built by launch_brick_list before the brick kernels.
struct BrickList {
    int32_t *list;    // [nbricks]
    int32_t *count;   // [1]
    uint32_t *sums;   // [<= 1024] block totals
    int64_t nbricks;
};

hipError_t launch_brick_list(const int32_t *cb, const int32_t *ce, BrickList &B, hipStream_t s);

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;

hipError_t launch_sort_cells(const DevParams &P, int64_t n, const double *x, uint32_t *key, int32_t *order,
                             int32_t *cell_begin, int32_t *cell_end, int64_t K, SortScratch &S, int64_t *err,
                             hipStream_t s);
hipError_t launch_reorder(int64_t n, const int32_t *order, const double *x, const double *v, const double *r,
                          const int32_t *id, double *xo, double *vo, double *ro, int32_t *ido, hipStream_t s);

template <typename T>
hipError_t launch_contact(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                          const int32_t *cb, const int32_t *ce, const BrickList &B, const T *sr, const double *held,
                          T *F, int32_t *ncont, int64_t *err, hipStream_t s);
hipError_t launch_contact_pairs(const DevParams &P, int64_t n, const double *x, const double *r,
                                const int32_t *cb, const int32_t *ce, int32_t *pairs, int64_t cap,
                                int64_t *count, hipStream_t s);

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
hipError_t launch_p2g_real(const DevParams &P, int64_t n, int64_t K, const double *x, const double *v,
                           const double *r, const int32_t *cb, const int32_t *ce, const BrickList &B,
                           double *alpha, double *mom, hipStream_t s);

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
                          const int32_t *ce, const BrickList &B, double *gx, double *gA, hipStream_t s);
hipError_t launch_p2g_vjp(const DevParams &P, int64_t n, const double *x, const double *v, const double *r,
                          const double *gA, const double *gP, double *gx, double *gv, hipStream_t s);
hipError_t launch_sum(const double *a, const double *b, int64_t n, double *part, int nparts, double *out, int acc,
                      hipStream_t s);
hipError_t launch_permute(int64_t n, int comps, const int32_t *order, const double *in, double *out, int scatter,
                          hipStream_t s);

inline unsigned grid_for(int64_t n, int threads)
{
    int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace gic
