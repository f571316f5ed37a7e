// Mole-fraction profiles of a stored state and their vector-Jacobian product.
//
// The paper reports mole fractions averaged over regions of the domain
// (Sec. 4.1); a profile along x, averaged over y and z, is the observable
// the adjoint's misfit is built from.  For a stored state s (population
// layout, P0 = f~_0 and g_a = f~_a - (w_a/w_0) P0 per species and node) the
// species density is rho_i = P0/w_0 + sum_{a>=1} g_a (collision conserves it,
// so it is also the density of the streamed populations), the mole fraction is
// x_i = (rho_i/M_i)/n with n = sum_j rho_j/M_j (Sec. 3), and
//     xbar_i(x) = (1/R) sum over the R rows (y, z) of x_i(x, y, z).
// Everything here is evaluated in FP64 from the FP32 state.
//
// Reduction: work-group (bx, c) owns 64 columns and the c-th chunk of rows; it
// writes one FP64 partial sum per (chunk, species, column) into a scratch
// array, and a second kernel adds the chunks of each (species, column) in
// chunk order.  The result does not depend on timing (no atomics).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "common.hpp"
#include "lattice.hpp"

namespace lbmmc {

// Scratch of the allocation-free profile (lbm_mc_profile_static): the FP64
// partial sums live in this fixed device array instead of context memory.
// Host code never uses the array's name as an address: profile_scratch()
// looks up each device's copy with hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kProfileScratchDoubles];

// Species densities (FP64) of node (x, row) of a lattice's stored state.
template <int LAT, int NS>
__device__ __forceinline__ void node_densities(const float* __restrict__ s, const LatParams& P,
                                               int x, int64_t row, double (&rho)[NS]) {
    constexpr int Q = Lat<LAT>::Q;
    const float* b = s + P.base + row * P.pitch + x;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const float* p = b + (int64_t)(i * Q) * P.plane;
        double r = (double)p[0] * (double)Lat<LAT>::inv_w0;
#pragma unroll
        for (int a = 1; a < Q; ++a) r += (double)p[(int64_t)a * P.plane];
        rho[i] = r;
    }
}

template <int NS>
__device__ __forceinline__ void mole_fractions(const double (&rho)[NS], const LatParams& P,
                                               double (&xm)[NS], double& n) {
    n = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        xm[i] = rho[i] / (double)P.M[i];
        n += xm[i];
    }
    const double in = 1.0 / n;
#pragma unroll
    for (int i = 0; i < NS; ++i) xm[i] *= in;
}

// part[(c * NS + i) * nx + x] = sum over the rows of chunk c of x_i(x, row)
template <int LAT, int NS>
__global__ void __launch_bounds__(64) k_profile_part(const float* __restrict__ s,
                                                     const LatParams* __restrict__ lps,
                                                     int rows_per, double* __restrict__ part) {
    const LatParams& P = lps[0];
    const int x = blockIdx.x * 64 + (int)threadIdx.x;
    const int c = blockIdx.y;
    if (x >= P.nx) return;
    const int64_t rows = (int64_t)P.ny * P.nz;
    const int64_t r0 = (int64_t)c * rows_per;
    const int64_t r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
    double acc[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) acc[i] = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        double rho[NS], xm[NS], n;
        node_densities<LAT, NS>(s, P, x, r, rho);
        mole_fractions<NS>(rho, P, xm, n);
#pragma unroll
        for (int i = 0; i < NS; ++i) acc[i] += xm[i];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) part[((int64_t)c * NS + i) * P.nx + x] = acc[i];
}

// xbar[i * nx + x] = (sum over chunks in order) / rows
__global__ void __launch_bounds__(256) k_profile_sum(const LatParams* __restrict__ lps, int ns,
                                                     int nchunks, const double* __restrict__ part,
                                                     double* __restrict__ xbar) {
    const LatParams& P = lps[0];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)ns * P.nx;
    if (k >= total) return;
    double v = 0.0;
    for (int c = 0; c < nchunks; ++c) v += part[(int64_t)c * total + k];
    xbar[k] = v / ((double)P.ny * (double)P.nz);
}

// Vector-Jacobian product: with d_i(x) = dL/dxbar_i(x),
//   dL/drho_j = (1/R) (d_j - sum_i d_i x_i) / (M_j n),
// and rho_j = P0/w_0 + sum_{a>=1} g_a gives lam(P0) = dL/drho_j / w_0,
// lam(g_a) = dL/drho_j.  Written (not added) at every node; the row padding
// of lam is not touched.
template <int LAT, int NS>
__global__ void __launch_bounds__(256) k_profile_vjp(const float* __restrict__ s,
                                                     const LatParams* __restrict__ lps,
                                                     const double* __restrict__ dxbar,
                                                     float* __restrict__ lam) {
    constexpr int Q = Lat<LAT>::Q;
    const LatParams& P = lps[0];
    const int64_t rows = (int64_t)P.ny * P.nz;
    const int64_t nodes = rows * P.nx;
    const double inv_rows = 1.0 / (double)rows;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < nodes;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(id % P.nx);
        const int64_t r = id / P.nx;
        double rho[NS], xm[NS], n;
        node_densities<LAT, NS>(s, P, x, r, rho);
        mole_fractions<NS>(rho, P, xm, n);
        double cx = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) cx += dxbar[(int64_t)i * P.nx + x] * xm[i];
        float* b = lam + P.base + r * P.pitch + x;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const double dr =
                inv_rows * (dxbar[(int64_t)j * P.nx + x] - cx) / ((double)P.M[j] * n);
            float* p = b + (int64_t)(j * Q) * P.plane;
            p[0] = (float)(dr * (double)Lat<LAT>::inv_w0);
#pragma unroll
            for (int a = 1; a < Q; ++a) p[(int64_t)a * P.plane] = (float)dr;
        }
    }
}

template <class Fn>
static hipError_t by_lat_ns(int lattice, int ns, Fn&& fn) {
    using std::integral_constant;
    if (lattice == 0) {
        if (ns == 2) return fn(integral_constant<int, 0>{}, integral_constant<int, 2>{});
        if (ns == 3) return fn(integral_constant<int, 0>{}, integral_constant<int, 3>{});
        if (ns == 4) return fn(integral_constant<int, 0>{}, integral_constant<int, 4>{});
    } else if (lattice == 1) {
        if (ns == 2) return fn(integral_constant<int, 1>{}, integral_constant<int, 2>{});
        if (ns == 3) return fn(integral_constant<int, 1>{}, integral_constant<int, 3>{});
        if (ns == 4) return fn(integral_constant<int, 1>{}, integral_constant<int, 4>{});
    }
    return hipErrorInvalidValue;
}

hipError_t launch_profile(int lattice, int ns, const LatParams* lp, const LatParams& h,
                          const float* state, int rows_per, int nchunks, double* part,
                          double* xbar, hipStream_t st) {
    const int xb = (h.nx + 63) / 64;
    hipError_t e = by_lat_ns(lattice, ns, [&](auto la, auto n) {
        constexpr int LAT = decltype(la)::value, NS = decltype(n)::value;
        hipLaunchKernelGGL((k_profile_part<LAT, NS>), dim3(xb, nchunks), dim3(64), 0, st, state,
                           lp, rows_per, part);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)ns * h.nx;
    hipLaunchKernelGGL(k_profile_sum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, lp,
                       ns, nchunks, part, xbar);
    return hipGetLastError();
}

hipError_t launch_profile_vjp(int lattice, int ns, const LatParams* lp, const LatParams& h,
                              const float* state, const double* dxbar, float* lam,
                              int max_blocks, hipStream_t st) {
    const int64_t nodes = (int64_t)h.nx * h.ny * h.nz;
    const int64_t want = (nodes + 255) / 256;
    const unsigned blocks = (unsigned)(want < max_blocks ? want : max_blocks);
    return by_lat_ns(lattice, ns, [&](auto la, auto n) {
        constexpr int LAT = decltype(la)::value, NS = decltype(n)::value;
        hipLaunchKernelGGL((k_profile_vjp<LAT, NS>), dim3(blocks), dim3(256), 0, st, state, lp,
                           dxbar, lam);
        return hipGetLastError();
    });
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept for the process.
hipError_t profile_scratch(double** out) {
    static std::mutex mu;
    static std::map<int, double*> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        double* p = nullptr;
        e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(dev, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

}  // namespace lbmmc
