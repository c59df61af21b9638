// Host-side launch helpers shared by the API translation unit and the kernels.
#pragma once

#include "s3a_internal.h"

namespace s3a {

struct LaunchCfg {
  int wg = 256;
  int items = 4;
  int occupancy = 4;  // persistent workgroups per CU
  int window = 0;     // pairs per window in the persistent launch (0: all)
};

// BF16 planes (xyz or depth) load 8 elements per 16 bytes, FP32 ones 4.
inline int vec_of(int dtype) { return (dtype == S3A_BF16 || dtype == DT_DEPTH_BF16) ? 8 : 4; }
inline int64_t tile_elems(int dtype, const LaunchCfg& lc) { return (int64_t)lc.wg * lc.items * vec_of(dtype); }
// Upper bound of the tile count of any batch (see k_sched).
inline int64_t max_tiles(int64_t n_points, int n_pairs, int64_t tile) { return n_points / tile + 2 * (int64_t)n_pairs + 1; }

hipError_t launch_sched(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st);
hipError_t launch_pass(int dtype, int mode, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                       int32_t tile_lo, int32_t tile_hi, int grid, hipStream_t st);
hipError_t launch_finalize(int kind, const Shape& sh, const CallDesc* cd, const Work& w, int pass, int32_t pair_lo,
                           int32_t n, hipStream_t st);
hipError_t launch_prep(const Shape& sh, const CallDesc* cd, const Work& w, int adjoint, hipStream_t st);
// Depth input: per-pair cameras into pass form; invalid geometry marks the pair bad.
hipError_t launch_depth_prep(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st);
hipError_t launch_finalize_cost(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st);
hipError_t launch_adjoint(int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w, int grid,
                          hipStream_t st);
hipError_t launch_finalize_adjoint(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st);
hipError_t launch_persistent(int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                             int grid, hipStream_t st);
hipError_t launch_fill_zero(uint32_t* p, int64_t n, hipStream_t st);
hipError_t launch_init_outputs(const Shape& sh, const CallDesc* cd, hipStream_t st);

}  // namespace s3a
