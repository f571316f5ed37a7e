// A streaming device copy used as the read-write reference of the benchmark:
// it moves every byte once in each direction, with non-temporal 16-byte loads
// and stores, over a grid-stride loop with four independent transfers in
// flight per thread.  (Measured on MI355X: best with one 256-thread
// work-group per compute unit; more work-groups interleave more streams and
// lose bandwidth, plain loads or stores lose a few per cent.)  Its rate is the practical ceiling of a
// kernel that reads one array and writes another of the same size, and its
// FETCH_SIZE / WRITE_SIZE counters calibrate those of the fused step.
#include <hip/hip_runtime.h>

#include "../../include/lbm_mc_copy.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_copy(const f4* __restrict__ src,
                                                     f4* __restrict__ dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const f4 a = __builtin_nontemporal_load(src + i);
        const f4 b = __builtin_nontemporal_load(src + i + stride);
        const f4 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const f4 d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n4; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" int32_t lbm_mc_stream_copy(const float* src, float* dst, int64_t n_floats,
                                      int32_t blocks, void* hip_stream) {
    if (!src || !dst || n_floats < 0 || n_floats % 4 || blocks < 1) return 1;
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return 1;
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst, bytes = (uintptr_t)n_floats * 4;
    if (a < b + bytes && b < a + bytes) return 1;
    if (n_floats == 0) return 0;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)hip_stream, reinterpret_cast<const f4*>(src),
                       reinterpret_cast<f4*>(dst), n_floats / 4);
    return hipGetLastError() == hipSuccess ? 0 : 3;
}
