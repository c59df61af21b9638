// Launchers of the point-correction kernels (Sec. III-C.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "s3a.h"

namespace s3a {

// flag: device int32 scratch, set to 1 when the offsets are invalid (and
// copied to status, the caller's device int32, when that is not null).
hipError_t launch_check_offsets(int64_t n, int32_t n_sub, const int64_t* off, int32_t* flag, int32_t* status,
                                hipStream_t st);

// Reads the flag written by launch_check_offsets earlier on the stream.
hipError_t launch_transform(int dtype, int64_t n, int32_t n_sub, const int64_t* off, const s3a_sim3* T,
                            const void* x, const void* y, const void* z, float* ox, float* oy, float* oz,
                            const int32_t* flag, hipStream_t st);

hipError_t launch_correct(int64_t n_corr, const int64_t* src, const int64_t* dst, int64_t n_world, const float* wx,
                          const float* wy, const float* wz, int64_t n_sparse, float* sx, float* sy, float* sz,
                          unsigned long long* skipped, hipStream_t st);

}  // namespace s3a
