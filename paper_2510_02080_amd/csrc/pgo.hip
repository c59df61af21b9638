#include "pgo.h"

namespace s3a {
struct PgoWorkspace {};
int pgo_solve(PgoWorkspace**, int*, int32_t, int32_t, const int32_t*, const s3a_sim3*, const double*, s3a_sim3*,
              const s3a_pgo_params*, s3a_pgo_report*, hipStream_t) {
  return S3A_EINVAL;
}
void pgo_free(PgoWorkspace* ws) { delete ws; }
}  // namespace s3a
