// Launcher of the implicit derivative of the solved pose.
#pragma once

#include "align_launch.h"

namespace s3a {

// hpart: device scratch of 52 doubles per slot, max_tiles + n_pairs slots. gS: the caller's upstream
// gradient (16 per pair, s3a_sim3 layout, or 7 per pair with
// S3A_IMPLICIT_TANGENT). Gradients go to the planes in the call descriptor.
// grid: workgroups of the per-point gradient pass; the Hessian pass runs as
// many workgroups as fit on the n_cu compute units at once (at most
// max_tiles), each over an equal share of the call's rows.
hipError_t launch_implicit(int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                           double* hpart, const double* gS, uint32_t iflags, double* v_out, int32_t* status_out,
                           int grid, int64_t max_tiles, int n_cu, hipStream_t st);

}  // namespace s3a
