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

}  // namespace s3a
