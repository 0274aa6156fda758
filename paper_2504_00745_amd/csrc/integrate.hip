// a6 + a7: interphase drag (Sec. 3.3 Eq. 5b; App. A relaxation drag in
// Stokes form, scaled by the local fluid fraction) and the semi-implicit
// Euler move (Sec. 4: the velocity is advanced first and the position with
// the new velocity) on gfx950.  Streaming kernels, one thread per granule.
#include "gic_launch.hpp"

namespace gic {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_drag(DevParams P, int64_t n, const double *__restrict__ r,
                                              const double *__restrict__ v, const T *__restrict__ uat,
                                              const T *__restrict__ af, T *__restrict__ Fd)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const T beta = (T)(P.cdrag * r[q]) * af[q];
    for (int a = 0; a < 3; ++a) Fd[a * n + q] = beta * (uat[a * n + q] - (T)v[a * n + q]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_integrate(DevParams P, int64_t n, const double *__restrict__ r,
                                                   const T *__restrict__ Fc, const T *__restrict__ Fd,
                                                   double *__restrict__ x, double *__restrict__ v)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double inv_m = 1.0 / mass_of(P, r[q]);
    for (int a = 0; a < 3; ++a) {
        double f = (double)Fc[a * n + q];
        if (Fd) f += (double)Fd[a * n + q];
        const double vn = v[a * n + q] + P.dt * (f * inv_m + P.g[a]);
        v[a * n + q] = vn;
        x[a * n + q] = x[a * n + q] + P.dt * vn;
    }
}

}  // namespace

template <typename T>
hipError_t launch_drag(const DevParams &P, int64_t n, const double *r, const double *v, const T *uat, const T *af,
                       T *Fd, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_drag<T><<<grid_for(n, 256), 256, 0, s>>>(P, n, r, v, uat, af, Fd);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_integrate(const DevParams &P, int64_t n, const double *r, const T *Fc, const T *Fd, double *x,
                            double *v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_integrate<T><<<grid_for(n, 256), 256, 0, s>>>(P, n, r, Fc, Fd, x, v);
    return hipGetLastError();
}

template hipError_t launch_drag<float>(const DevParams &, int64_t, const double *, const double *, const float *,
                                       const float *, float *, hipStream_t);
template hipError_t launch_drag<double>(const DevParams &, int64_t, const double *, const double *,
                                        const double *, const double *, double *, hipStream_t);
template hipError_t launch_integrate<float>(const DevParams &, int64_t, const double *, const float *,
                                            const float *, double *, double *, hipStream_t);
template hipError_t launch_integrate<double>(const DevParams &, int64_t, const double *, const double *,
                                             const double *, double *, double *, hipStream_t);

}  // namespace gic
