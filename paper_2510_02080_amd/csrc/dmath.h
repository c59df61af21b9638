// FP64 small-matrix and Sim(3) math for the per-pair and per-edge solves.
//
// Everything here runs on one lane (one thread per pair or per edge) in FP64 on
// the GPU, and is also compiled for the host so that it can be unit-tested
// without a device. Conventions (Sec. III-C.2 and Sec. III-E):
//   * a similarity {s, R, t} maps x -> s R x + t; R is row-major 3x3;
//   * tangent coordinates xi = (rho, omega, sigma): translation, rotation,
//     log-scale; perturbations act on the left, S <- Exp(xi) S.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define S3A_HD __host__ __device__ inline
#define S3A_NO_UNROLL _Pragma("unroll 1")
#define S3A_UNROLL _Pragma("unroll")
#else
#define S3A_HD inline
#define S3A_NO_UNROLL
#define S3A_UNROLL
#endif

namespace s3a {

struct Sim3d {
  double R[9];
  double t[3];
  double s;
};

S3A_HD Sim3d sim3_identity() {
  Sim3d r;
  for (int i = 0; i < 9; ++i) r.R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  r.t[0] = r.t[1] = r.t[2] = 0.0;
  r.s = 1.0;
  return r;
}

S3A_HD void mat3_mul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

S3A_HD void mat3_vec(const double* A, const double* x, double* y) {
  for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

S3A_HD void mat3T_vec(const double* A, const double* x, double* y) {
  for (int i = 0; i < 3; ++i) y[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
}

// a o b : x -> a(b(x))
S3A_HD Sim3d sim3_compose(const Sim3d& a, const Sim3d& b) {
  Sim3d r;
  mat3_mul(a.R, b.R, r.R);
  double Rt[3];
  mat3_vec(a.R, b.t, Rt);
  for (int i = 0; i < 3; ++i) r.t[i] = a.s * Rt[i] + a.t[i];
  r.s = a.s * b.s;
  return r;
}

S3A_HD Sim3d sim3_inverse(const Sim3d& a) {
  Sim3d r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.R[3 * i + j] = a.R[3 * j + i];
  r.s = 1.0 / a.s;
  double Rt[3];
  mat3_vec(r.R, a.t, Rt);
  for (int i = 0; i < 3; ++i) r.t[i] = -r.s * Rt[i];
  return r;
}

// Cyclic Jacobi eigen-decomposition of a symmetric N x N matrix (row-major, in
// place). On return A's diagonal holds the eigenvalues and the columns of V the
// eigenvectors. Unsorted.
template <int N>
S3A_HD void jacobi_eig(double* A, double* V) {
  for (int i = 0; i < N * N; ++i) V[i] = (i % (N + 1) == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < N; ++i) {
      diag += A[i * N + i] * A[i * N + i];
      for (int j = i + 1; j < N; ++j) off += A[i * N + j] * A[i * N + j];
    }
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < N - 1; ++p) {
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p * N + q];
        if (apq == 0.0) continue;
        const double app = A[p * N + p], aqq = A[q * N + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < N; ++k) {  // A <- A J (columns p, q)
          const double akp = A[k * N + p], akq = A[k * N + q];
          A[k * N + p] = c * akp - s * akq;
          A[k * N + q] = s * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {  // A <- J^T A (rows p, q)
          const double apk = A[p * N + k], aqk = A[q * N + k];
          A[p * N + k] = c * apk - s * aqk;
          A[q * N + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < N; ++k) {
          const double vkp = V[k * N + p], vkq = V[k * N + q];
          V[k * N + p] = c * vkp - s * vkq;
          V[k * N + q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

// Rotation maximising tr(R^T M) over SO(3) (M = sum w dq dp^T), through the
// unit quaternion of the largest eigenvalue of the symmetric 4x4 form of
// tr(R(q)^T M) (Horn's method). For rank(M) >= 2 this is the same rotation as
// the reflection-corrected SVD solution of Umeyama's estimate.
S3A_HD void rotation_from_cross_cov(const double* M, double* R) {
  double N[16] = {
      M[0] + M[4] + M[8], M[7] - M[5], M[2] - M[6], M[3] - M[1],
      M[7] - M[5], M[0] - M[4] - M[8], M[1] + M[3], M[2] + M[6],
      M[2] - M[6], M[1] + M[3], -M[0] + M[4] - M[8], M[5] + M[7],
      M[3] - M[1], M[2] + M[6], M[5] + M[7], -M[0] - M[4] + M[8]};
  double V[16];
  jacobi_eig<4>(N, V);
  int best = 0;
  for (int i = 1; i < 4; ++i)
    if (N[i * 5] > N[best * 5]) best = i;
  double q0 = V[best], q1 = V[4 + best], q2 = V[8 + best], q3 = V[12 + best];
  const double n = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  q0 /= n; q1 /= n; q2 /= n; q3 /= n;
  R[0] = q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3;
  R[1] = 2.0 * (q1 * q2 - q0 * q3);
  R[2] = 2.0 * (q1 * q3 + q0 * q2);
  R[3] = 2.0 * (q1 * q2 + q0 * q3);
  R[4] = q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3;
  R[5] = 2.0 * (q2 * q3 - q0 * q1);
  R[6] = 2.0 * (q1 * q3 - q0 * q2);
  R[7] = 2.0 * (q2 * q3 + q0 * q1);
  R[8] = q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3;
}

// Singular values of a 3x3 matrix, descending, from the eigenvalues of M^T M.
S3A_HD void singular_values3(const double* M, double* sv) {
  double A[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      A[3 * i + j] = M[i] * M[j] + M[3 + i] * M[3 + j] + M[6 + i] * M[6 + j];
  double V[9];
  jacobi_eig<3>(A, V);
  double e[3] = {A[0], A[4], A[8]};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (e[j] > e[i]) { const double x = e[i]; e[i] = e[j]; e[j] = x; }
  for (int i = 0; i < 3; ++i) sv[i] = sqrt(e[i] > 0.0 ? e[i] : 0.0);
}

enum { UMEYAMA_OK = 0, UMEYAMA_EMPTY = 1, UMEYAMA_DEGENERATE = 2 };

// Weighted Umeyama from raw weighted moments (Sec. III-C.2, eq. (sim3)):
//   W = sum w, sp = sum w p, sq = sum w q, spp = sum w |p|^2,
//   sqp[3a+b] = sum w q_a p_b.
// Degeneracy: W <= 0 (empty); centred spread <= 1e-12 of the second moment;
// second singular value of the cross-covariance <= 1e-5 of the first.
S3A_HD int umeyama_from_moments(double W, const double* sp, const double* sq, double spp,
                                const double* sqp, Sim3d* out, double* mu_q) {
  *out = sim3_identity();
  if (!(W > 0.0)) return UMEYAMA_EMPTY;
  double mp[3], mq[3];
  for (int i = 0; i < 3; ++i) { mp[i] = sp[i] / W; mq[i] = sq[i] / W; }
  if (mu_q) for (int i = 0; i < 3; ++i) mu_q[i] = mq[i];
  const double mp2 = mp[0] * mp[0] + mp[1] * mp[1] + mp[2] * mp[2];
  const double var_p = spp / W - mp2;
  if (!(var_p > 1e-12 * (var_p + mp2))) return UMEYAMA_DEGENERATE;
  double M[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[3 * a + b] = sqp[3 * a + b] / W - mq[a] * mp[b];
  double sv[3];
  singular_values3(M, sv);
  if (!(sv[1] > 1e-5 * sv[0])) return UMEYAMA_DEGENERATE;
  double R[9];
  rotation_from_cross_cov(M, R);
  double tr = 0.0;
  for (int i = 0; i < 9; ++i) tr += R[i] * M[i];
  const double s = tr / var_p;
  if (!(s > 0.0)) return UMEYAMA_DEGENERATE;
  double Rmp[3];
  mat3_vec(R, mp, Rmp);
  for (int i = 0; i < 9; ++i) out->R[i] = R[i];
  for (int i = 0; i < 3; ++i) out->t[i] = mq[i] - s * Rmp[i];
  out->s = s;
  return UMEYAMA_OK;
}

// In-place Cholesky solve of the SPD system H x = b (n <= 7). H is overwritten.
// Returns false when a pivot is not positive.
template <int N>
S3A_HD bool cholesky_solve(double* H, const double* b, double* x) {
  for (int j = 0; j < N; ++j) {
    double d = H[j * N + j];
    for (int k = 0; k < j; ++k) d -= H[j * N + k] * H[j * N + k];
    if (!(d > 0.0)) return false;
    d = sqrt(d);
    H[j * N + j] = d;
    for (int i = j + 1; i < N; ++i) {
      double v = H[i * N + j];
      for (int k = 0; k < j; ++k) v -= H[i * N + k] * H[j * N + k];
      H[i * N + j] = v / d;
    }
  }
  double y[N];
  for (int i = 0; i < N; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= H[i * N + k] * y[k];
    y[i] = v / H[i * N + i];
  }
  for (int i = N - 1; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < N; ++k) v -= H[k * N + i] * x[k];
    x[i] = v / H[i * N + i];
  }
  return true;
}

// Cholesky solve of the SPD system H x = b with H given as its packed lower
// triangle (row i holds H[i][0..i], at offset i (i + 1) / 2), overwritten by
// the factor. Returns false when a pivot is not positive.
template <int N>
S3A_HD bool cholesky_solve_packed(double* L, const double* b, double* x) {
  for (int j = 0; j < N; ++j) {
    const int rj = j * (j + 1) / 2;
    double d = L[rj + j];
    for (int k = 0; k < j; ++k) d -= L[rj + k] * L[rj + k];
    if (!(d > 0.0)) return false;
    d = sqrt(d);
    const double inv = 1.0 / d;
    L[rj + j] = inv;  // the diagonal is kept as its reciprocal
    for (int i = j + 1; i < N; ++i) {
      const int ri = i * (i + 1) / 2;
      double v = L[ri + j];
      for (int k = 0; k < j; ++k) v -= L[ri + k] * L[rj + k];
      L[ri + j] = v * inv;
    }
  }
  double y[N];
  for (int i = 0; i < N; ++i) {
    const int ri = i * (i + 1) / 2;
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[ri + k] * y[k];
    y[i] = v * L[ri + i];
  }
  for (int i = N - 1; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < N; ++k) v -= L[k * (k + 1) / 2 + i] * x[k];
    x[i] = v * L[i * (i + 1) / 2 + i];
  }
  return true;
}

// F_n(sigma) = int_0^1 exp(sigma u) u^n du.
S3A_HD double int_exp_pow(int n, double sg) {
  if (fabs(sg) < 2.0) {  // power series sum_k sg^k / (k! (n + k + 1))
    double term = 1.0, sum = 0.0;
    for (int k = 0; k < 40; ++k) {
      sum += term / (double)(n + k + 1);
      term *= sg / (double)(k + 1);
    }
    return sum;
  }
  const double e = exp(sg);  // F_0 = (e - 1)/sg, F_n = (e - n F_{n-1})/sg
  double F = (e - 1.0) / sg;
  for (int k = 1; k <= n; ++k) F = (e - (double)k * F) / sg;
  return F;
}

// 1 / n! for the series below (folded to constants where the loops unroll).
constexpr double inv_factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return 1.0 / f;
}

// Rotation R = exp([omega]_x) (Rodrigues) and the translation map
// V = int_0^1 e^{sigma u} exp(u [omega]_x) du = a0 I + c1 [omega]_x + c2 [omega]_x^2,
// a0 = F_0(sigma), c1 = int e^{sigma u} sin(u th)/th du,
// c2 = int e^{sigma u} (1 - cos(u th))/th^2 du, th = |omega|.
S3A_HD void sim3_RV(const double* w, double sg, double* R, double* V) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double A, B;  // Rodrigues coefficients sin(th)/th, (1 - cos th)/th^2
  double c1, c2, a0;
  if (th < 0.1 && fabs(sg) < 4.0) {
    // Expansion in th^2 with F_n(sigma) = int_0^1 e^{sigma u} u^n du:
    //   c1 = sum_m (-1)^m th^{2m} F_{2m+1} / (2m+1)!,  c2 = sum_m (-1)^m th^{2m} F_{2m+2} / (2m+2)!,
    //   a0 = F_0, and A, B the Taylor series of sin th / th and (1 - cos th) / th^2,
    // truncated after m = 4 (th^10 / 11! < 3e-18). The F_n come from the downward
    // recurrence n F_{n-1} = e^sigma - sigma F_n started at n = 40 from
    // F_40 ~ e^sigma / (41 + sigma): each step scales the start error by |sigma| / n,
    // so below n = 10 it is under 1e-23 for |sigma| < 4. Horner in th^2 runs
    // with the recurrence (m falls as n falls).
    const double es = exp(sg);
    double F = es / (41.0 + sg);
    c1 = 0.0; c2 = 0.0;
    S3A_UNROLL
    for (int n = 40; n >= 1; --n) {
      F = (es - sg * F) * (1.0 / n);  // F_{n-1}
      const int j = n - 1;
      if (j >= 1 && j <= 10) {
        const double coef = (((j - 1) / 2) & 1 ? -1.0 : 1.0) * inv_factorial(j);
        if (j & 1) c1 = c1 * th2 + coef * F;
        else c2 = c2 * th2 + coef * F;
      }
    }
    a0 = F;
    A = 0.0; B = 0.0;
    S3A_UNROLL
    for (int m = 4; m >= 0; --m) {
      const double sgn = (m & 1) ? -1.0 : 1.0;
      A = A * th2 + sgn * inv_factorial(2 * m + 1);
      B = B * th2 + sgn * inv_factorial(2 * m + 2);
    }
  } else if (th < 0.1) {
    a0 = int_exp_pow(0, sg);
    // series in th^2: sin(u th)/th = sum (-1)^k th^{2k} u^{2k+1}/(2k+1)!,
    // (1-cos(u th))/th^2 = sum (-1)^k th^{2k} u^{2k+2}/(2k+2)!
    A = 0.0; B = 0.0; c1 = 0.0; c2 = 0.0;
    double p = 1.0, f1 = 1.0, f2 = 2.0;  // th^{2k}, (2k+1)!, (2k+2)!
    for (int k = 0; k < 7; ++k) {
      const double sgn = (k & 1) ? -1.0 : 1.0;
      A += sgn * p / f1;
      B += sgn * p / f2;
      c1 += sgn * p / f1 * int_exp_pow(2 * k + 1, sg);
      c2 += sgn * p / f2 * int_exp_pow(2 * k + 2, sg);
      p *= th2;
      f1 *= (double)((2 * k + 2) * (2 * k + 3));
      f2 *= (double)((2 * k + 3) * (2 * k + 4));
    }
  } else {
    a0 = sg == 0.0 ? 1.0 : expm1(sg) / sg;
    const double sn = sin(th), cs = cos(th);
    A = sn / th;
    B = (1.0 - cs) / th2;
    const double den = sg * sg + th2;
    const double es = exp(sg);
    const double Is = (es * (sg * sn - th * cs) + th) / den;
    const double Ic = (es * (sg * cs + th * sn) - sg) / den;
    c1 = Is / th;
    c2 = (a0 - Ic) / th2;
  }
  const double Wm[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  double W2[9];
  mat3_mul(Wm, Wm, W2);
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    R[i] = I + A * Wm[i] + B * W2[i];
    V[i] = a0 * I + c1 * Wm[i] + c2 * W2[i];
  }
}

// Exp of xi = (rho, omega, sigma) = {e^sigma, exp([omega]_x), V rho}.
S3A_HD Sim3d sim3_exp(const double* xi) {
  Sim3d r;
  double V[9];
  sim3_RV(xi + 3, xi[6], r.R, V);
  mat3_vec(V, xi, r.t);
  r.s = exp(xi[6]);
  return r;
}

// Rotation vector of R (angle in [0, pi]).
S3A_HD void so3_log(const double* R, double* w) {
  const double tr = R[0] + R[4] + R[8];
  const double v0 = R[7] - R[5], v1 = R[2] - R[6], v2 = R[3] - R[1];
  const double sn2 = sqrt(v0 * v0 + v1 * v1 + v2 * v2);  // 2 sin th
  const double th = atan2(sn2, tr - 1.0);
  if (th < 1e-5) {
    const double f = 0.5 * (1.0 + th * th / 6.0);  // th / (2 sin th)
    w[0] = f * v0; w[1] = f * v1; w[2] = f * v2;
    return;
  }
  if (th < 3.0) {
    const double f = th / sn2;
    w[0] = f * v0; w[1] = f * v1; w[2] = f * v2;
    return;
  }
  // near pi: axis from the symmetric part, sign from the skew part
  const double cth = cos(th);
  double a[3];
  for (int i = 0; i < 3; ++i) {
    const double d = (R[4 * i] - cth) / (1.0 - cth);
    a[i] = sqrt(d > 0.0 ? d : 0.0);
  }
  int k = 0;
  if (a[1] > a[k]) k = 1;
  if (a[2] > a[k]) k = 2;
  // off-diagonal symmetric terms give the relative signs
  const double S01 = R[1] + R[3], S02 = R[2] + R[6], S12 = R[5] + R[7];
  if (k == 0) { a[1] = (S01 >= 0 ? 1 : -1) * a[1]; a[2] = (S02 >= 0 ? 1 : -1) * a[2]; }
  if (k == 1) { a[0] = (S01 >= 0 ? 1 : -1) * a[0]; a[2] = (S12 >= 0 ? 1 : -1) * a[2]; }
  if (k == 2) { a[0] = (S02 >= 0 ? 1 : -1) * a[0]; a[1] = (S12 >= 0 ? 1 : -1) * a[1]; }
  const double dot = a[0] * v0 + a[1] * v1 + a[2] * v2;
  const double sgn = dot < 0.0 ? -1.0 : 1.0;
  const double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  for (int i = 0; i < 3; ++i) w[i] = sgn * th * a[i] / n;
}

// 3x3 solve by Cramer's rule (V is well conditioned for |omega| < pi).
S3A_HD void solve3(const double* A, const double* b, double* x) {
  const double c00 = A[4] * A[8] - A[5] * A[7];
  const double c01 = A[5] * A[6] - A[3] * A[8];
  const double c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const double inv[9] = {c00, A[2] * A[7] - A[1] * A[8], A[1] * A[5] - A[2] * A[4],
                         c01, A[0] * A[8] - A[2] * A[6], A[2] * A[3] - A[0] * A[5],
                         c02, A[1] * A[6] - A[0] * A[7], A[0] * A[4] - A[1] * A[3]};
  for (int i = 0; i < 3; ++i) x[i] = (inv[3 * i] * b[0] + inv[3 * i + 1] * b[1] + inv[3 * i + 2] * b[2]) / det;
}

// Log of a similarity: sigma = ln s, omega = Log(R), rho = V(omega, sigma)^{-1} t.
S3A_HD void sim3_log(const Sim3d& T, double* xi) {
  double w[3];
  so3_log(T.R, w);
  const double sg = log(T.s);
  double R[9], V[9];
  sim3_RV(w, sg, R, V);
  solve3(V, T.t, xi);
  xi[3] = w[0]; xi[4] = w[1]; xi[5] = w[2];
  xi[6] = sg;
}

// ad(xi) (7x7, row-major): [[sg I + [w]x, [rho]x, -rho], [0, [w]x, 0], [0, 0, 0]].
S3A_HD void sim3_ad(const double* xi, double* A) {
  for (int i = 0; i < 49; ++i) A[i] = 0.0;
  const double r0 = xi[0], r1 = xi[1], r2 = xi[2], w0 = xi[3], w1 = xi[4], w2 = xi[5], sg = xi[6];
  const double Wm[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
  const double Rm[9] = {0.0, -r2, r1, r2, 0.0, -r0, -r1, r0, 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A[7 * i + j] = Wm[3 * i + j] + (i == j ? sg : 0.0);
      A[7 * i + 3 + j] = Rm[3 * i + j];
      A[7 * (3 + i) + 3 + j] = Wm[3 * i + j];
    }
  A[7 * 0 + 6] = -r0; A[7 * 1 + 6] = -r1; A[7 * 2 + 6] = -r2;
}

// Ad(T) (7x7): [[s R, [t]x R, -t], [0, R, 0], [0, 0, 1]].
S3A_HD void sim3_Ad(const Sim3d& T, double* A) {
  for (int i = 0; i < 49; ++i) A[i] = 0.0;
  const double* t = T.t;
  const double Tm[9] = {0.0, -t[2], t[1], t[2], 0.0, -t[0], -t[1], t[0], 0.0};
  double TR[9];
  mat3_mul(Tm, T.R, TR);
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) {
      A[7 * i + j] = T.s * T.R[3 * i + j];
      A[7 * i + 3 + j] = TR[3 * i + j];
      A[7 * (3 + i) + 3 + j] = T.R[3 * i + j];
    }
    A[7 * i + 6] = -t[i];
  }
  A[48] = 1.0;
}

// sum_{n>=0} (sgn ad(xi))^n / (n+1)!  -> J_l (sgn = +1) or J_r (sgn = -1).
S3A_HD void sim3_jacobian(const double* xi, double sgn, double* J) {
  double A[49], P[49], Q[49];
  sim3_ad(xi, A);
  for (int i = 0; i < 49; ++i) { A[i] *= sgn; P[i] = (i % 8 == 0) ? 1.0 : 0.0; J[i] = P[i]; }
  for (int n = 1; n < 80; ++n) {
    double mx = 0.0;
    for (int i = 0; i < 7; ++i)
      for (int j = 0; j < 7; ++j) {
        double v = 0.0;
        for (int k = 0; k < 7; ++k) v += P[7 * i + k] * A[7 * k + j];
        Q[7 * i + j] = v / (double)(n + 1);
      }
    for (int i = 0; i < 49; ++i) {
      P[i] = Q[i];
      J[i] += Q[i];
      const double a = fabs(Q[i]);
      mx = a > mx ? a : mx;
    }
    if (mx < 1e-18) break;
  }
}

// Gauss-Jordan inverse with partial pivoting (n = 7). Returns false if singular.
S3A_HD bool inv7(const double* A, double* X) {
  double M[7 * 14];
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 14; ++j) M[14 * i + j] = j < 7 ? A[7 * i + j] : (j - 7 == i ? 1.0 : 0.0);
  for (int c = 0; c < 7; ++c) {
    int p = c;
    for (int r = c + 1; r < 7; ++r)
      if (fabs(M[14 * r + c]) > fabs(M[14 * p + c])) p = r;
    if (M[14 * p + c] == 0.0) return false;
    if (p != c)
      for (int j = 0; j < 14; ++j) { const double x = M[14 * c + j]; M[14 * c + j] = M[14 * p + j]; M[14 * p + j] = x; }
    const double d = 1.0 / M[14 * c + c];
    for (int j = 0; j < 14; ++j) M[14 * c + j] *= d;
    for (int r = 0; r < 7; ++r) {
      if (r == c) continue;
      const double f = M[14 * r + c];
      if (f != 0.0)
        for (int j = 0; j < 14; ++j) M[14 * r + j] -= f * M[14 * c + j];
    }
  }
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j) X[7 * i + j] = M[14 * i + 7 + j];
  return true;
}

}  // namespace s3a
