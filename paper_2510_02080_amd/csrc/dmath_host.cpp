// Host build of the FP64 per-pair / per-edge math that the kernels run on the
// device, exported with C linkage so it can be checked on a machine without a
// GPU. Internal test hooks; not part of the public interface.
#include "dmath.h"

using namespace s3a;

static Sim3d load(const double* T) {  // R[9], t[3], s
  Sim3d r;
  for (int i = 0; i < 9; ++i) r.R[i] = T[i];
  for (int i = 0; i < 3; ++i) r.t[i] = T[9 + i];
  r.s = T[12];
  return r;
}

static void store(const Sim3d& a, double* T) {
  for (int i = 0; i < 9; ++i) T[i] = a.R[i];
  for (int i = 0; i < 3; ++i) T[9 + i] = a.t[i];
  T[12] = a.s;
}

extern "C" {

void s3a_host_sim3_exp(const double* xi, double* T) { store(sim3_exp(xi), T); }

void s3a_host_sim3_log(const double* T, double* xi) { sim3_log(load(T), xi); }

void s3a_host_sim3_compose(const double* A, const double* B, double* T) {
  store(sim3_compose(load(A), load(B)), T);
}

void s3a_host_sim3_inverse(const double* A, double* T) { store(sim3_inverse(load(A)), T); }

void s3a_host_sim3_ad(const double* xi, double* A) { sim3_ad(xi, A); }

void s3a_host_sim3_Ad(const double* T, double* A) { sim3_Ad(load(T), A); }

void s3a_host_sim3_jacobian(const double* xi, double sgn, double* J) { sim3_jacobian(xi, sgn, J); }

int s3a_host_inv7(const double* A, double* X) { return inv7(A, X) ? 0 : 1; }

int s3a_host_cholesky7(const double* H, const double* b, double* x) {
  double Hc[49];
  for (int i = 0; i < 49; ++i) Hc[i] = H[i];
  return cholesky_solve<7>(Hc, b, x) ? 0 : 1;
}

int s3a_host_cholesky7_packed(const double* H, const double* b, double* x) {
  double L[28];
  int u = 0;
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j <= i; ++j) L[u++] = H[7 * i + j];
  return cholesky_solve_packed<7>(L, b, x) ? 0 : 1;
}

// moments: W, sp[3], sq[3], spp, sqp[9]
int s3a_host_umeyama(const double* m, double* T) {
  Sim3d S;
  const int st = umeyama_from_moments(m[0], m + 1, m + 4, m[7], m + 8, &S, nullptr);
  store(S, T);
  return st;
}

void s3a_host_rotation_from_cross_cov(const double* M, double* R) { rotation_from_cross_cov(M, R); }

void s3a_host_singular_values3(const double* M, double* sv) { singular_values3(M, sv); }
}
