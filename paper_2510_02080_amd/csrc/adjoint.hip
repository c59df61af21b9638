// Adjoint of the Huber alignment cost (the robust form of Sec. III-C.2,
// eq. (sim3)) with respect to points, confidences and the left tangent
// perturbation xi of S' = Exp(xi) S.
//
// One streaming pass per call: reads the seven planes, recomputes the Huber
// weight of every point (nothing is stored by the forward beyond L and C per
// pair), writes FP32 gradients for the pair's elements, and reduces the seven
// FP64 sums of dL/dxi per tile.
#include "align_kernels.h"
#include "align_launch.h"

namespace s3a {

template <int DT, int WG, int ITEMS>
__global__ __launch_bounds__(WG) void k_adjoint(Shape sh, const CallDesc* __restrict__ cd, Work w) {
  constexpr int VEC = Planes<DT>::VEC;
  __shared__ double red[WG / 64][NSTAT];
  const int total = *w.total_tiles;
  const void* pl[7];
  float* gout[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) { pl[j] = cd->planes[j]; gout[j] = cd->grad[j]; }
  const float tau = sh.tau, delta = sh.delta_f;
  for (int t = (int)blockIdx.x; t < total; t += (int)gridDim.x) {
    const TileDesc td = load_tile(w.tiles + t);
    const PointParams P = load_params(w.params + td.pair);
    double acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = 0.0;
#pragma unroll 1
    for (int it = 0; it < ITEMS; ++it) {
      const int64_t g0 = td.begin + (int64_t)(it * WG + (int)threadIdx.x) * VEC;
      if (g0 >= td.end) continue;
      float v[7][VEC];
      Planes<DT>::load(SrcCtx<DT>{pl}, g0, sh.n_points, v);
      float go[7][VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int64_t g = g0 + e;
        const bool in = (g >= td.lo) && (g < td.end);
        float x[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) x[j] = v[j][e];
        const bool valid = P.active && in && finite7(x) && x[6] >= tau;
        if (!valid) {
#pragma unroll
          for (int j = 0; j < 7; ++j) x[j] = 0.0f;
        }
        const double p0 = x[0], p1 = x[1], p2 = x[2];
        double y[3], r[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          y[i] = fma(P.M[3 * i], p0, fma(P.M[3 * i + 1], p1, fma(P.M[3 * i + 2], p2, P.t[i])));
          r[i] = y[i] - (double)x[3 + i];
        }
        const float rf[3] = {(float)r[0], (float)r[1], (float)r[2]};
        const float e2 = rf[0] * rf[0] + rf[1] * rf[1] + rf[2] * rf[2];
        float psi, rho;
        if (e2 <= delta * delta) {
          psi = 1.0f;
          rho = 0.5f * e2;
        } else {
          const float ie = rsqrtf(e2);
          psi = delta * ie;
          rho = delta * (e2 * ie - 0.5f * delta);
        }
        const float wgt = x[6] * P.inv_C;         // w_i (0 when invalid)
        const float f = P.scale * wgt * psi;      // gL w psi
        go[3][e] = -f * rf[0];
        go[4][e] = -f * rf[1];
        go[5][e] = -f * rf[2];
        // (s R)^T r
        go[0][e] = f * (P.Mf[0] * rf[0] + P.Mf[3] * rf[1] + P.Mf[6] * rf[2]);
        go[1][e] = f * (P.Mf[1] * rf[0] + P.Mf[4] * rf[1] + P.Mf[7] * rf[2]);
        go[2][e] = f * (P.Mf[2] * rf[0] + P.Mf[5] * rf[1] + P.Mf[8] * rf[2]);
        go[6][e] = valid ? P.scale * (rho - P.L) * P.inv_C : 0.0f;
        // dL/dxi sums (unnormalised omega = c psi; FP64)
        const double om = (double)x[6] * (double)psi;
        const double orr[3] = {om * r[0], om * r[1], om * r[2]};
        acc[0] += orr[0];
        acc[1] += orr[1];
        acc[2] += orr[2];
        acc[3] += y[1] * orr[2] - y[2] * orr[1];
        acc[4] += y[2] * orr[0] - y[0] * orr[2];
        acc[5] += y[0] * orr[1] - y[1] * orr[0];
        acc[6] += y[0] * orr[0] + y[1] * orr[1] + y[2] * orr[2];
      }
#pragma unroll
      for (int j = 0; j < 7; ++j) store_grad_vec(gout[j], g0, sh.n_points, go[j], VEC, td.lo, td.end);
    }
    block_store_f64<WG, 7>(acc, red, w.partials + (int64_t)t * NSTAT);
  }
}

// dL/dxi = gL J_l(xi)^T (1/C) sum om J^T r.
__global__ __launch_bounds__(64) void k_finalize_adjoint(Shape sh, const CallDesc* __restrict__ cd, Work w) {
  const int k = blockIdx.x;
  if (k >= sh.n_pairs) return;
  const PairSched sc = w.sched[k];
  double s[NSTAT];
  pair_sums(w, sc, 7, s);
  if (threadIdx.x != 0 || !cd->gxi) return;
  double* out = cd->gxi + 7 * k;
  const double C = cd->C_in[k];
  if (!(C > 0.0)) {
    for (int i = 0; i < 7; ++i) out[i] = 0.0;
    return;
  }
  const double f = cd->gL[k] / C;
  double g[7];
  for (int i = 0; i < 7; ++i) g[i] = f * s[i];
  if (cd->xi) {
    double J[49];
    sim3_jacobian(cd->xi + 7 * k, 1.0, J);
    for (int i = 0; i < 7; ++i) {
      double v = 0.0;
      for (int m = 0; m < 7; ++m) v += J[7 * m + i] * g[m];
      out[i] = v;
    }
  } else {
    for (int i = 0; i < 7; ++i) out[i] = g[i];
  }
}

template <int DT>
static hipError_t launch_adjoint_t(const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w, int grid,
                                   hipStream_t st) {
#define S3A_CASE(WGV, IT)                                                                \
  if (lc.wg == WGV && lc.items == IT) {                                                  \
    hipLaunchKernelGGL((k_adjoint<DT, WGV, IT>), dim3(grid), dim3(WGV), 0, st, sh, cd, w); \
    return hipGetLastError();                                                            \
  }
  S3A_CASE(256, 2) S3A_CASE(256, 4) S3A_CASE(256, 8) S3A_CASE(256, 16)
  S3A_CASE(512, 2) S3A_CASE(512, 4) S3A_CASE(512, 8)
#undef S3A_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w, int grid,
                          hipStream_t st) {
  return dtype == S3A_F32 ? launch_adjoint_t<S3A_F32>(lc, sh, cd, w, grid, st)
                          : launch_adjoint_t<S3A_BF16>(lc, sh, cd, w, grid, st);
}

hipError_t launch_finalize_adjoint(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st) {
  if (sh.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize_adjoint, dim3(sh.n_pairs), dim3(64), 0, st, sh, cd, w);
  return hipGetLastError();
}

}  // namespace s3a
