// Sim(3) pose-graph solve (Sec. III-E): host symbolic analysis and the FP64
// device factorisation.
#pragma once

#include <hip/hip_runtime.h>

#include "s3a.h"

namespace s3a {

struct PgoWorkspace;

int pgo_solve(PgoWorkspace** ws, int* last_hip, int32_t n_nodes, int32_t n_edges, const int32_t* ij,
              const s3a_sim3* T_meas, const double* omega, s3a_sim3* T, const s3a_pgo_params* params,
              s3a_pgo_report* report, hipStream_t stream);
void pgo_free(PgoWorkspace* ws);
hipError_t launch_edges_from_alignment(int n, const s3a_sim3* S, const s3a_align_info* info, double info_scale,
                                       s3a_sim3* T_out, double* omega, int32_t* status, hipStream_t st);

}  // namespace s3a
