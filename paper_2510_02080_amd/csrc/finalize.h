// FP64 per-pair finalize of the alignment passes (Sec. III-C.2, eq. (sim3);
// Huber IRLS): from a pair's summed statistics, the weighted Umeyama start or
// one Gauss-Newton step, run by one lane. Shared by the multi-launch and the
// persistent schedules.
#pragma once

#include "align_kernels.h"

namespace s3a {

__device__ inline void store_sim3(s3a_sim3* o, const Sim3d& S) {
  for (int i = 0; i < 9; ++i) o->R[i] = S.R[i];
  for (int i = 0; i < 3; ++i) o->t[i] = S.t[i];
  o->s = S.s;
  o->pad[0] = o->pad[1] = o->pad[2] = 0.0;
}

__device__ inline Sim3d load_sim3(const s3a_sim3* o) {
  Sim3d S;
  for (int i = 0; i < 9; ++i) S.R[i] = o->R[i];
  for (int i = 0; i < 3; ++i) S.t[i] = o->t[i];
  S.s = o->s;
  return S;
}

__device__ inline bool sim3_finite(const Sim3d& S) {
  bool f = __builtin_isfinite(S.s) && S.s > 0.0;
  for (int i = 0; i < 9; ++i) f = f && __builtin_isfinite(S.R[i]);
  for (int i = 0; i < 3; ++i) f = f && __builtin_isfinite(S.t[i]);
  return f;
}

__device__ inline void publish(PointParams* P, const Sim3d& S, const double* c, int active, int nonfinite = 1) {
  PointParams p;
  for (int i = 0; i < 9; ++i) { p.M[i] = S.s * S.R[i]; p.Mf[i] = (float)p.M[i]; }
  for (int i = 0; i < 3; ++i) {
    p.t[i] = S.t[i];
    p.c[i] = c[i];
    p.tcf[i] = (float)(S.t[i] - c[i]);
    p.cf[i] = (float)c[i];
  }
  p.inv_C = 0.0f;
  p.scale = 0.0f;
  p.L = 0.0f;
  p.active = active;
  p.nonfinite = nonfinite;
  *P = p;
}

__device__ inline void write_outputs(const CallDesc* cd, int k, const PairState& st, double final_cost,
                                     int64_t final_inl) {
  const bool ok = st.status == S3A_PAIR_OK;
  const double nan = __builtin_nan("");
  store_sim3(cd->S_out + k, ok ? st.S : sim3_identity());
  if (cd->info) {
    s3a_align_info* I = cd->info + k;
    I->cost = ok ? st.cost_lin : nan;
    I->final_cost = ok ? final_cost : nan;
    I->weight_sum = st.C;
    for (int i = 0; i < 28; ++i) I->H[i] = ok ? st.H[i] : nan;
    for (int i = 0; i < 7; ++i) I->g[i] = ok ? st.g[i] : nan;
    I->n_valid = st.V;
    I->n_nonfinite = st.nnf;
    I->n_inliers = ok ? st.inl_lin : 0;
    I->final_inliers = ok ? final_inl : 0;
    I->status = st.status;
    I->iters = st.iters;
  }
}

// Packed lower triangle of H and g of the Gauss-Newton system with Jacobian
// [I, -[y]x, y] from the 17 sums (om, om y, om y y^T, om r, om y x r, om y.r):
//   H_rr = W I, H_rw = -[a]x, H_rs = a, H_ww = tr(B) I - B, H_ws = 0, H_ss = tr(B);
//   g = (b_r, b_x, b_d).
__device__ inline void assemble_gn_packed(const double* st, double* L, double* g) {
  const double A0 = st[0];
  const double a0 = st[1], a1 = st[2], a2 = st[3];
  const double Bxx = st[4], Bxy = st[5], Bxz = st[6], Byy = st[7], Byz = st[8], Bzz = st[9];
  const double trB = Bxx + Byy + Bzz;
  // row 0..6, columns 0..i
  L[0] = A0;
  L[1] = 0.0; L[2] = A0;
  L[3] = 0.0; L[4] = 0.0; L[5] = A0;
  L[6] = 0.0; L[7] = -a2; L[8] = a1; L[9] = trB - Bxx;
  L[10] = a2; L[11] = 0.0; L[12] = -a0; L[13] = -Bxy; L[14] = trB - Byy;
  L[15] = -a1; L[16] = a0; L[17] = 0.0; L[18] = -Bxz; L[19] = -Byz; L[20] = trB - Bzz;
  L[21] = a0; L[22] = a1; L[23] = a2; L[24] = 0.0; L[25] = 0.0; L[26] = 0.0; L[27] = trB;
  for (int i = 0; i < 7; ++i) g[i] = st[10 + i];
}

// Moments pass -> weighted Umeyama start (or the caller's), validity, centre.
__device__ inline void finalize_moments(const Shape& sh, const CallDesc* cd, Work& w, int k, const PairSched& sc,
                                        const double* s) {
  const double nan = __builtin_nan("");
  PairState* st = w.state + k;
  st->C = s[0];
  st->V = (int64_t)s[17];
  st->nnf = (int64_t)s[18];
  st->cost_lin = nan;
  for (int i = 0; i < 28; ++i) st->H[i] = nan;
  for (int i = 0; i < 7; ++i) st->g[i] = nan;
  st->inl_lin = 0;
  st->iters = 0;
  int status = S3A_PAIR_OK;
  double cq[3] = {0.0, 0.0, 0.0};
  Sim3d S = sim3_identity();
  if (sc.bad) {
    status = S3A_PAIR_BADRANGE;
  } else if (st->V == 0) {
    status = st->nnf > 0 ? S3A_PAIR_NONFINITE : S3A_PAIR_EMPTY;
  } else if (!(s[0] > 0.0)) {
    status = S3A_PAIR_DEGENERATE;
  } else {
    const int u = umeyama_from_moments(s[0], s + 1, s + 4, s[7], s + 8, &S, cq);
    if (cd->init) {
      S = load_sim3(cd->init + k);
      if (!sim3_finite(S)) status = S3A_PAIR_NONFINITE;
    } else if (u != UMEYAMA_OK) {
      status = u == UMEYAMA_EMPTY ? S3A_PAIR_EMPTY : S3A_PAIR_DEGENERATE;
    }
  }
  if (status != S3A_PAIR_OK) S = sim3_identity();
  st->S = S;
  for (int i = 0; i < 3; ++i) st->cq[i] = cq[i];
  st->status = status;
  const bool more = status == S3A_PAIR_OK && (sh.K > 0 || (sh.flags & S3A_FLAG_FINAL_COST));
  if (!more) write_outputs(cd, k, *st, nan, 0);
  publish(w.params + k, S, cq, more ? 1 : 0, st->nnf > 0 ? 1 : 0);
}

// Gauss-Newton pass `pass` (1..K): assemble H, g in centred coordinates from the
// 17 statistics, Cholesky solve, map the step back, S <- Exp(xi) S. The
// reported H, g are those of the uncentred Jacobian, rebuilt from the same
// statistics shifted back by the centre c (y = y_c + c).
__device__ inline void finalize_gn(const Shape& sh, const CallDesc* cd, Work& w, int k, int pass, const double* s) {
  PairState* st = w.state + k;
  if (st->status != S3A_PAIR_OK || !w.params[k].active) return;
  const double nan = __builtin_nan("");
  const double c[3] = {st->cq[0], st->cq[1], st->cq[2]};
  const double C = st->C;
  st->cost_lin = s[17] / C;  // the cost and inlier count at the linearisation point
  st->inl_lin = (int64_t)s[18];
  double Hp[28], g[7], x[7];
  assemble_gn_packed(s, Hp, g);
  for (int i = 0; i < 7; ++i) g[i] = -g[i];
  int status = S3A_PAIR_OK;
  if (cholesky_solve_packed<7>(Hp, g, x)) {
    // xi = Ad(translation c) xi': rho = rho' + c x omega - sigma c
    double xi[7];
    xi[0] = x[0] + (c[1] * x[5] - c[2] * x[4]) - x[6] * c[0];
    xi[1] = x[1] + (c[2] * x[3] - c[0] * x[5]) - x[6] * c[1];
    xi[2] = x[2] + (c[0] * x[4] - c[1] * x[3]) - x[6] * c[2];
    for (int i = 3; i < 7; ++i) xi[i] = x[i];
    const Sim3d Snew = sim3_compose(sim3_exp(xi), st->S);
    if (!sim3_finite(Snew)) {
      status = S3A_PAIR_NONFINITE;
    } else {
      st->S = Snew;
      st->iters = pass;
    }
    if (status == S3A_PAIR_OK && pass == sh.K) {
      // Reported with the last step only: uncentred statistics, y = y_c + c
      double u[17];
      const double A0 = s[0], a[3] = {s[1], s[2], s[3]}, br[3] = {s[10], s[11], s[12]};
      u[0] = A0;
      for (int i = 0; i < 3; ++i) u[1 + i] = a[i] + A0 * c[i];
      u[4] = s[4] + 2.0 * a[0] * c[0] + A0 * c[0] * c[0];
      u[5] = s[5] + a[0] * c[1] + c[0] * a[1] + A0 * c[0] * c[1];
      u[6] = s[6] + a[0] * c[2] + c[0] * a[2] + A0 * c[0] * c[2];
      u[7] = s[7] + 2.0 * a[1] * c[1] + A0 * c[1] * c[1];
      u[8] = s[8] + a[1] * c[2] + c[1] * a[2] + A0 * c[1] * c[2];
      u[9] = s[9] + 2.0 * a[2] * c[2] + A0 * c[2] * c[2];
      for (int i = 0; i < 3; ++i) u[10 + i] = br[i];
      u[13] = s[13] + (c[1] * br[2] - c[2] * br[1]);
      u[14] = s[14] + (c[2] * br[0] - c[0] * br[2]);
      u[15] = s[15] + (c[0] * br[1] - c[1] * br[0]);
      u[16] = s[16] + c[0] * br[0] + c[1] * br[1] + c[2] * br[2];
      assemble_gn_packed(u, Hp, g);
      // packed lower -> row-major upper triangle (same values, H symmetric)
      const double invC = 1.0 / C;
      int m = 0;
      for (int i = 0; i < 7; ++i)
        for (int j = i; j < 7; ++j) st->H[m++] = Hp[j * (j + 1) / 2 + i] * invC;
      for (int i = 0; i < 7; ++i) st->g[i] = g[i] * invC;
    }
  } else {
    status = S3A_PAIR_DEGENERATE;
  }
  st->status = status;
  const bool failed = status != S3A_PAIR_OK;
  const bool last = pass == sh.K;
  const bool final_pass = (sh.flags & S3A_FLAG_FINAL_COST) != 0;
  if (failed || (last && !final_pass)) write_outputs(cd, k, *st, nan, 0);
  publish(w.params + k, st->S, c, (failed || (last && !final_pass)) ? 0 : 1, st->nnf > 0 ? 1 : 0);
}

__device__ inline void finalize_final_cost(const CallDesc* cd, Work& w, int k, const double* s) {
  const PairState* st = w.state + k;
  if (st->status != S3A_PAIR_OK || !w.params[k].active) return;
  write_outputs(cd, k, *st, s[17] / st->C, (int64_t)s[18]);
  w.params[k].active = 0;
}

}  // namespace s3a
