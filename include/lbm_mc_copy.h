/*
 * Measurement aid of the lbm_mc library (not part of the method): a streaming
 * device-to-device copy whose rate is the practical ceiling of a kernel that
 * reads one array and writes another, the memory pattern of the fused step
 * (one FP32 read and one FP32 write per population).  The benchmark reports
 * the fused step against it as well as against the HBM peak, and profiles
 * calibrate their byte counters with it.
 */
#ifndef LBM_MC_COPY_H
#define LBM_MC_COPY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * dst[0 .. n_floats) = src[0 .. n_floats), asynchronously on hip_stream
 * (NULL = null stream), with `blocks` work-groups of 256 threads in a
 * grid-stride loop (non-temporal 16-byte loads and stores).
 *   src, dst   device memory, 16-byte aligned, not overlapping; caller-owned.
 *   n_floats   a multiple of 4, >= 0.
 * Returns 0 on success, 1 (LBM_MC_ERR_INVALID) for a bad argument, 3
 * (LBM_MC_ERR_HIP) if the launch failed.
 */
int32_t lbm_mc_stream_copy(const float* src, float* dst, int64_t n_floats, int32_t blocks,
                           void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_MC_COPY_H */
