// Forward launchers: dispatch on the lattice to the kernels compiled in
// step_d2q9.hip and step_d3q19.hip, and the fixed-order FP64 reduction of the
// observables' per-tile partials.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lbmmc {

template <int LAT>
hipError_t launch_step_lat(int ns, const Launch& L);
template <int LAT>
hipError_t launch_init_lat(int ns, const LatParams* lp, int lat, const LatParams& h,
                           const double* x0, const float* accel, float* f0, float* ft,
                           unsigned* flag, hipStream_t s);
template <int LAT>
hipError_t launch_moments_lat(int ns, const Launch& L, int direct, float* rho, float* x,
                              float* u, float* ueq, float* us, double* partial, int nq);

extern template hipError_t launch_step_lat<0>(int, const Launch&);
extern template hipError_t launch_step_lat<1>(int, const Launch&);
extern template hipError_t launch_init_lat<0>(int, const LatParams*, int, const LatParams&,
                                              const double*, const float*, float*, float*,
                                              unsigned*, hipStream_t);
extern template hipError_t launch_init_lat<1>(int, const LatParams*, int, const LatParams&,
                                              const double*, const float*, float*, float*,
                                              unsigned*, hipStream_t);
extern template hipError_t launch_moments_lat<0>(int, const Launch&, int, float*, float*, float*,
                                                 float*, float*, double*, int);
extern template hipError_t launch_moments_lat<1>(int, const Launch&, int, float*, float*, float*,
                                                 float*, float*, double*, int);

hipError_t launch_step(int lattice, int ns, const Launch& L) {
    if (lattice == 0) return launch_step_lat<0>(ns, L);
    if (lattice == 1) return launch_step_lat<1>(ns, L);
    return hipErrorInvalidValue;
}

hipError_t launch_init(int lattice, int ns, const LatParams* lp, int lat, const LatParams& h,
                       const double* x0, const float* accel, float* f0, float* ft,
                       unsigned* flag, hipStream_t s) {
    if (lattice == 0) return launch_init_lat<0>(ns, lp, lat, h, x0, accel, f0, ft, flag, s);
    if (lattice == 1) return launch_init_lat<1>(ns, lp, lat, h, x0, accel, f0, ft, flag, s);
    return hipErrorInvalidValue;
}

hipError_t launch_moments(int lattice, int ns, const Launch& L, int direct, float* rho, float* x,
                          float* u, float* ueq, float* us, double* partial, int nq) {
    if (lattice == 0) return launch_moments_lat<0>(ns, L, direct, rho, x, u, ueq, us, partial, nq);
    if (lattice == 1) return launch_moments_lat<1>(ns, L, direct, rho, x, u, ueq, us, partial, nq);
    return hipErrorInvalidValue;
}

// Fixed-order FP64 sum of the per-tile partials of each lattice: one
// work-group per lattice, thread t takes tiles begin+t, begin+t+256, ..., then
// a fixed shuffle and LDS tree (reproducible run to run).
__global__ void __launch_bounds__(256) k_reduce(const LatParams* __restrict__ lps, int nlat,
                                                const double* __restrict__ partial, int nq,
                                                double* __restrict__ totals) {
    __shared__ double red[4];
    const int l = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int t0 = lps[l].tile_begin, t1 = lps[l].tile_end;
    for (int q = 0; q < nq; ++q) {
        double v = 0.0;
        for (int t = t0 + tid; t < t1; t += 256) v += partial[(int64_t)t * nq + q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (tid == 0) totals[(int64_t)l * nq + q] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

hipError_t launch_reduce(const LatParams* lp, int nlat, const double* partial, int nq,
                         double* totals, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(nlat), dim3(256), 0, s, lp, nlat, partial, nq, totals);
    return hipGetLastError();
}

}  // namespace lbmmc
