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
    const double vq[3] = {v[q], v[n + q], v[2 * n + q]};
    const T ua[3] = {uat[q], uat[n + q], uat[2 * n + q]};
    T f[3];
    drag_one<T>(P, r[q], vq, ua, af[q], f);
    for (int a = 0; a < 3; ++a) Fd[a * n + q] = f[a];
}

template <typename T>
__global__ void __launch_bounds__(256) k_integrate(DevParams P, int64_t n, const double *__restrict__ r,
                                                   const T *__restrict__ Fc, const T *__restrict__ Fd,
                                                   double *__restrict__ x, double *__restrict__ v)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double xq[3] = {x[q], x[n + q], x[2 * n + q]};
    double vq[3] = {v[q], v[n + q], v[2 * n + q]};
    const T fc[3] = {Fc[q], Fc[n + q], Fc[2 * n + q]};
    if (Fd) {
        const T fd[3] = {Fd[q], Fd[n + q], Fd[2 * n + q]};
        integrate_one<T>(P, r[q], fc, fd, xq, vq);
    } else {
        integrate_one<T>(P, r[q], fc, (const T *)nullptr, xq, vq);
    }
    for (int a = 0; a < 3; ++a) {
        x[a * n + q] = xq[a];
        v[a * n + q] = vq[a];
    }
}

// Moisture ratio of each granule (Sec. 5.4, the definition following Eq. 26):
// the water it holds plus the free water around it per unit sand volume,
// sr = held + alpha_f / (1 - alpha_f), in double (+inf at alpha_f = 1).
template <typename T>
__global__ void __launch_bounds__(256) k_moisture_ratio(int64_t n, const double *__restrict__ held,
                                                        const T *__restrict__ af, T *__restrict__ sr)
{
#pragma clang fp contract(off)
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double a = (double)af[q];
    sr[q] = (T)(held[q] + a / (1.0 - a));
}

}  // namespace

template <typename T>
hipError_t launch_moisture_ratio(int64_t n, const double *held, const T *af, T *sr, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_moisture_ratio<T><<<grid_for(n, 256), 256, 0, s>>>(n, held, af, sr);
    return hipGetLastError();
}

template hipError_t launch_moisture_ratio<float>(int64_t, const double *, const float *, float *, hipStream_t);
template hipError_t launch_moisture_ratio<double>(int64_t, const double *, const double *, double *, hipStream_t);

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
