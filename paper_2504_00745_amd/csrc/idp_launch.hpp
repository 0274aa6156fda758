// Host-side launchers of the density-projection kernels (Sec. 5.1, Eq. 12b
// and 13; App. B discretisation) and the solver workspace layout; the C ABI
// in gic_api.hip validates arguments and calls these.
#pragma once

#include "gic_launch.hpp"

namespace gic {

constexpr uint8_t kIdpFluid = 0, kIdpAir = 1, kIdpSolid = 2;  // cell labels
constexpr int kIdpMaxBlocks = 1024;  // partial sums per reduced quantity

struct IdpDims {
    int64_t nx, ny, nz, sxy, G;
    // floor(n / nx) = (n * mx) >> shx and floor(n / ny) = (n * my) >> shy for
    // 0 <= n < 2^31 (set by idp_dims_finish)
    uint32_t mx, my;
    int32_t shx, shy;
};

// Conjugate-gradient scalars kept on the device between kernels.
struct CgState {
    double rz[2];   // r.z of the current iteration, by iteration parity
    double ss;      // s.s
    double thr;     // tol^2 s.s
    double rr;      // r.r after the last completed iteration
    int64_t done;   // iteration count at convergence, -1 while running
    int64_t iters;  // completed iterations
};

// One level of the solver's hierarchy: its cells, operator scale
// (A_l = scale L_l), signed coefficients (alpha_f' on fluid cells, -alpha_f'
// on air cells, 0 on solid cells), 1 / diag(A_l), right-hand side,
// correction and the prolonged iterate.  Level 0 is the fine grid.
struct MgLevel {
    IdpDims D;
    double scale;
    double *ac;
    double *dinv, *b, *e, *t;
};

constexpr int kMgMaxLevels = 24;
constexpr int64_t kMgCoarsest = 256;  // cells of the coarsest level, solved in one block

// Solver workspace carved from one caller buffer.  nlev = 1: Jacobi
// preconditioner; nlev > 1: multigrid over lev[0 .. nlev).
struct IdpWork {
    double *r, *d, *w, *dinv;
    double *part;     // [3 * kIdpMaxBlocks]
    CgState *state;
    int nlev;
    MgLevel lev[kMgMaxLevels];
};

IdpDims idp_dims(const DevParams &P);
// Fills sxy, G and the division constants from nx, ny, nz.
void idp_dims_finish(IdpDims &D);
hipError_t launch_idp_setup(const IdpDims &D, double alpha_max, const int64_t *afx, const double *astar,
                            const uint8_t *lab, double *at, double *s, int64_t *err, hipStream_t st);
hipError_t launch_idp_apply(const IdpDims &D, const double *at, const uint8_t *lab, const double *v, double *out,
                            hipStream_t st);
hipError_t launch_idp_faces(const IdpDims &D, double dx, const double *q, const uint8_t *lab, double *fx,
                            double *fy, double *fz, hipStream_t st);
hipError_t launch_cg_start(const IdpDims &D, const double *at, const uint8_t *lab, const double *s, const double *q,
                           const IdpWork &W, double tol, int64_t *err, hipStream_t st);
hipError_t launch_cg_iterations(const IdpDims &D, const double *at, const uint8_t *lab, double *q,
                                const IdpWork &W, int k0, int count, hipStream_t st);

}  // namespace gic
