// Implicit derivative of the solved pose (Sec. III-C.2, eq. (sim3) with Huber
// weights): with F = dL/dxi and H = d^2 L/dxi^2 at the solution S* (exact
// Hessian, second-order terms of Exp included), the implicit function theorem
// gives dl/dtheta = -(dF/dtheta)^T v, v = H^{-1} g_S, for the points and
// confidences theta. One FP64 pass gathers H and F, one FP64 finalize per pair
// solves for v, and one pass writes the per-point terms.
#include "implicit.h"

#include "finalize.h"

namespace s3a {

// Per-tile sums of the Hessian pass (weights om = c psi, c-weighted; divided
// by C = sum m c in the finalize). y = S* p, r = y - q, all in FP64:
//   0 sum om, 1-3 sum om y, 4-9 sum om y y^T (xx xy xz yy yz zz),
//   10-12 sum om r, 13-21 sum om y_a r_b (row-major a, b),
//   22-49 sum over points outside delta of c psi / e^2 u u^T, u = (r, y x r, y . r)
//         (packed lower triangle, row i at i (i + 1) / 2),
//   50 C, 51 valid count.
constexpr int HSTAT = 52;

template <int WG>
__device__ inline void block_store_h(double (&acc)[HSTAT], double (*red)[HSTAT], double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  wave_totals_f64(acc);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < HSTAT; ++j) red[wv][j] = acc[j];
  }
  __syncthreads();
  if ((int)threadIdx.x < HSTAT) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < WG / 64; ++q) s += red[q][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// The per-tile pipelined walk over a run of consecutive tiles of one pair, taken
// as one stream: `items` (even, known only at run time) vectors per lane, lane
// l's item i at element (i * WG + l) * VEC from the run's first tile. Tiles of
// a pair lie end to end, so this visits each element of the run once, as the
// per-tile walks do; the next vector's loads are issued before the current one
// is worked on.
template <int WG, int VEC, typename Raw, typename Fetch, typename Body>
__device__ inline void pipelined_run(int items, int end_rel, Fetch&& fetch, Body&& body) {
  constexpr int STRIDE = WG * VEC;
  Raw A, B;
  const int first = (int)threadIdx.x * VEC;
  if (first >= end_rel) return;
  fetch(first, A);
#pragma unroll 1
  for (int it = 0; it < items; it += 2) {
    const int r0 = first + it * STRIDE;
    const int r1 = r0 + STRIDE;
    const bool more1 = r1 < end_rel;
    if (more1) fetch(r1, B);
    body(A, r0);
    if (!more1) break;
    const int r2 = r1 + STRIDE;
    const bool more2 = it + 2 < items && r2 < end_rel;
    if (more2) fetch(r2, A);
    body(B, r1);
    if (!more2) break;
  }
}

// Each workgroup takes a contiguous range of tiles and streams each run of
// consecutive tiles of one pair as one pipelined sweep: the per-lane sums and
// the load pipeline carry across the run's tile boundaries, and the 52-value
// block reduction runs once per run, not once per tile. The run's sums land in
// the slot of its first tile and its other slots are zeroed, so the finalize
// (which adds every slot of a pair) is unchanged. The grid changes only the
// summation order.
template <int DT, int WG, int ITEMS>
__global__ __launch_bounds__(WG) void k_hess(Shape sh, const CallDesc* __restrict__ cd, Work w, double* hpart) {
  constexpr int VEC = Planes<DT>::VEC;
  __shared__ double red[WG / 64][HSTAT];
  const int total = *w.total_tiles;
  const int t0 = (int)((int64_t)total * blockIdx.x / gridDim.x);
  const int t1 = (int)((int64_t)total * (blockIdx.x + 1) / gridDim.x);
  const void* pl[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) pl[j] = cd->planes[j];
  const SrcCtx<DT> src{pl};
  const float tau = sh.tau;
  const double delta = sh.delta;
#pragma unroll 1
  for (int t = t0; t < t1;) {
    const TileDesc td = load_tile(w.tiles + t);
    const PairSched sc = w.sched[td.pair];
    // tiles in this run, capped so that element offsets within it fit an int
    const int m = min(min(t1, sc.tile0 + sc.ntiles) - t, (int)((1ll << 30) / sh.tile_elems));
    const int64_t run_end = w.tiles[t + m - 1].end;
    const PointParams P = load_params(w.params + td.pair);
    double a[HSTAT];
#pragma unroll
    for (int j = 0; j < HSTAT; ++j) a[j] = 0.0;
    const int lo_rel = (int)(td.lo - td.begin), end_rel = (int)(run_end - td.begin);
    pipelined_run<WG, VEC, RawVec>(
        m * ITEMS, end_rel, [&](int rel, RawVec& r) { Planes<DT>::fetch(src, td.begin + rel, sh.n_points, r); },
        [&](const RawVec& raw, int rel0) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            float x[7];
#pragma unroll
            for (int j = 0; j < 7; ++j) x[j] = Planes<DT>::elem(raw, j, e);
            const bool valid =
                P.active && rel0 + e >= lo_rel && rel0 + e < end_rel && finite7(x) && x[6] >= tau;
#pragma unroll
            for (int j = 0; j < 7; ++j) x[j] = valid ? x[j] : 0.0f;  // masked points add zeros
            double y[3], r[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              y[i] = fma(P.M[3 * i], (double)x[0],
                         fma(P.M[3 * i + 1], (double)x[1], fma(P.M[3 * i + 2], (double)x[2], P.t[i])));
              r[i] = y[i] - (double)x[3 + i];
            }
            const double c = x[6];
            const double e2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double ie = rsqrt(e2);  // 1 / |r|, used only outside delta (|r| > delta > 0)
            const bool outl = e2 > delta * delta;
            const double psi = outl ? delta * ie : 1.0;
            const double om = c * psi;
            a[0] += om;
#pragma unroll
            for (int i = 0; i < 3; ++i) a[1 + i] = fma(om, y[i], a[1 + i]);
            a[4] = fma(om * y[0], y[0], a[4]); a[5] = fma(om * y[0], y[1], a[5]); a[6] = fma(om * y[0], y[2], a[6]);
            a[7] = fma(om * y[1], y[1], a[7]); a[8] = fma(om * y[1], y[2], a[8]); a[9] = fma(om * y[2], y[2], a[9]);
#pragma unroll
            for (int i = 0; i < 3; ++i) a[10 + i] = fma(om, r[i], a[10 + i]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) a[13 + 3 * i + j] = fma(om * y[i], r[j], a[13 + 3 * i + j]);
            // rank-one correction of the Huber Hessian outside delta: c psi / e^2 u u^T
            const double k1 = outl ? om * ie * ie : 0.0;
            const double u[7] = {r[0], r[1], r[2], y[1] * r[2] - y[2] * r[1], y[2] * r[0] - y[0] * r[2],
                                 y[0] * r[1] - y[1] * r[0], y[0] * r[0] + y[1] * r[1] + y[2] * r[2]};
#pragma unroll
            for (int i = 0; i < 7; ++i) {
              const double ku = k1 * u[i];
#pragma unroll
              for (int j = 0; j <= i; ++j) a[22 + i * (i + 1) / 2 + j] = fma(ku, u[j], a[22 + i * (i + 1) / 2 + j]);
            }
            a[50] += c;
            a[51] += valid ? 1.0 : 0.0;
          }
        });
    block_store_h<WG>(a, red, hpart + (int64_t)t * HSTAT);
    for (int i = (int)threadIdx.x; i < (m - 1) * HSTAT; i += WG) hpart[(int64_t)(t + 1) * HSTAT + i] = 0.0;
    t += m;
  }
}

// Per pair: H and F from the sums, the upstream gradient in tangent form,
// v = H^{-1} g_S; published for the gradient pass (state: g = v, cost_lin =
// v^T F, C; params: active).
__global__ __launch_bounds__(64) void k_finalize_implicit(Shape sh, const CallDesc* __restrict__ cd, Work w,
                                                          const double* __restrict__ hpart, const double* __restrict__ gS,
                                                          uint32_t iflags, double* v_out, int32_t* status_out) {
  const int k = blockIdx.x;
  if (k >= sh.n_pairs) return;
  const PairSched sc = w.sched[k];
  const int lane = threadIdx.x & 63;
  double s[HSTAT];
#pragma unroll
  for (int j = 0; j < HSTAT; ++j) s[j] = 0.0;
  for (int t = sc.tile0 + lane; t < sc.tile0 + sc.ntiles; t += 64) {
    const double* p = hpart + (int64_t)t * HSTAT;
#pragma unroll
    for (int j = 0; j < HSTAT; ++j) s[j] += p[j];
  }
  wave_totals_f64(s);
  if (threadIdx.x != 0) return;
  const double nan = __builtin_nan("");
  const double C = s[50];
  int status = S3A_PAIR_OK;
  double v[7];
  for (int i = 0; i < 7; ++i) v[i] = nan;
  double vF = 0.0;
  if (sc.bad) {
    status = S3A_PAIR_BADRANGE;
  } else if (!(C > 0.0)) {
    status = S3A_PAIR_EMPTY;
  } else {
    const double iC = 1.0 / C;
    double st[50];
    for (int j = 0; j < 50; ++j) st[j] = s[j] * iC;
    const double A0 = st[0], av[3] = {st[1], st[2], st[3]};
    const double B[9] = {st[4], st[5], st[6], st[5], st[7], st[8], st[6], st[8], st[9]};
    const double trB = st[4] + st[7] + st[9];
    const double R[3] = {st[10], st[11], st[12]};
    const double* N = st + 13;  // N[3a + b] = sum om y_a r_b / C
    const double trN = N[0] + N[4] + N[8];
    const double yxr[3] = {N[5] - N[7], N[6] - N[2], N[1] - N[3]};
    double H[49];
    for (int i = 0; i < 49; ++i) H[i] = 0.0;
    // Gauss-Newton part sum om J^T J, J = [I, -[y]x, y]
    for (int i = 0; i < 3; ++i) {
      H[7 * i + i] = A0;
      H[7 * i + 6] = H[7 * 6 + i] = av[i];
    }
    const double ax[9] = {0.0, -av[2], av[1], av[2], 0.0, -av[0], -av[1], av[0], 0.0};  // [a]x
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        H[7 * i + 3 + j] = -ax[3 * i + j];  // rho-omega: -[a]x
        H[7 * (3 + j) + i] = -ax[3 * i + j];
        H[7 * (3 + i) + 3 + j] = (i == j ? trB : 0.0) - B[3 * i + j];
      }
    H[48] = trB;
    // minus the rank-one terms of the points outside delta
    for (int i = 0; i < 7; ++i)
      for (int j = 0; j <= i; ++j) {
        const double x = st[22 + i * (i + 1) / 2 + j];
        H[7 * i + j] -= x;
        if (j != i) H[7 * j + i] -= x;
      }
    // second-order terms of Exp: omega-rho -[R]x / 2, sigma-rho R / 2,
    // omega-omega (N + N^T) / 2 - tr(N) I, sigma-omega sum om y x r, sigma-sigma tr(N)
    const double Rx[9] = {0.0, -R[2], R[1], R[2], 0.0, -R[0], -R[1], R[0], 0.0};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        H[7 * (3 + a) + b] -= 0.5 * Rx[3 * a + b];
        H[7 * b + 3 + a] -= 0.5 * Rx[3 * a + b];
        H[7 * (3 + a) + 3 + b] += 0.5 * (N[3 * a + b] + N[3 * b + a]) - (a == b ? trN : 0.0);
      }
    for (int b = 0; b < 3; ++b) {
      H[7 * 6 + b] += 0.5 * R[b];
      H[7 * b + 6] += 0.5 * R[b];
      H[7 * 6 + 3 + b] += yxr[b];
      H[7 * (3 + b) + 6] += yxr[b];
    }
    H[48] += trN;
    const double F[7] = {R[0], R[1], R[2], yxr[0], yxr[1], yxr[2], trN};
    // upstream gradient as a left-perturbation gradient
    double g[7];
    if (iflags & S3A_IMPLICIT_TANGENT) {
      for (int i = 0; i < 7; ++i) g[i] = gS[7 * k + i];
    } else {
      const double* gm = gS + 16 * k;  // s3a_sim3 layout: R[9] (row-major), t[3], s
      const s3a_sim3& S = cd->S_in[k];
      double om[3] = {S.t[1] * gm[11] - S.t[2] * gm[10], S.t[2] * gm[9] - S.t[0] * gm[11],
                      S.t[0] * gm[10] - S.t[1] * gm[9]};
      for (int j = 0; j < 3; ++j) {  // column j of R and of d/dR
        const double c0 = S.R[j], c1 = S.R[3 + j], c2 = S.R[6 + j];
        const double d0 = gm[j], d1 = gm[3 + j], d2 = gm[6 + j];
        om[0] += c1 * d2 - c2 * d1;
        om[1] += c2 * d0 - c0 * d2;
        om[2] += c0 * d1 - c1 * d0;
      }
      g[0] = gm[9]; g[1] = gm[10]; g[2] = gm[11];
      g[3] = om[0]; g[4] = om[1]; g[5] = om[2];
      g[6] = S.s * gm[12] + S.t[0] * gm[9] + S.t[1] * gm[10] + S.t[2] * gm[11];
    }
    double x[7];
    if (cholesky_solve<7>(H, g, x)) {
      for (int i = 0; i < 7; ++i) {
        v[i] = x[i];
        vF += x[i] * F[i];
      }
    } else {
      status = S3A_PAIR_DEGENERATE;
    }
  }
  const bool ok = status == S3A_PAIR_OK;
  PairState* st = w.state + k;
  for (int i = 0; i < 7; ++i) st->g[i] = ok ? v[i] : 0.0;
  st->cost_lin = ok ? vF : 0.0;
  st->C = C;
  st->status = status;
  w.params[k].active = ok ? 1 : 0;
  if (v_out)
    for (int i = 0; i < 7; ++i) v_out[7 * k + i] = v[i];
  if (status_out) status_out[k] = status;
}

// Per point: a = v_rho + v_omega x y + v_sigma y, b = Q a (the Huber Hessian
// in r applied to a), and
//   dl/dq = (c/C) b,  dl/dp = -(c/C) (s R)^T (b + psi (r x v_omega + v_sigma r)),
//   dl/dc = -(psi a . r - v^T F) / C;  zero for masked points.
template <int DT, int WG, int ITEMS>
__global__ __launch_bounds__(WG) void k_igrad(Shape sh, const CallDesc* __restrict__ cd, Work w) {
  constexpr int VEC = Planes<DT>::VEC;
  const int total = *w.total_tiles;
  const void* pl[7];
  float* gout[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) { pl[j] = cd->planes[j]; gout[j] = cd->grad[j]; }
  const float tau = sh.tau;
  const double delta = sh.delta;
  for (int t = (int)blockIdx.x; t < total; t += (int)gridDim.x) {
    const TileDesc td = load_tile(w.tiles + t);
    const PointParams P = load_params(w.params + td.pair);
    const PairState* S = w.state + td.pair;
    double vv[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) vv[i] = S->g[i];
    const double vF = S->cost_lin, iC = P.active ? 1.0 / S->C : 0.0;
    const int lo_rel = (int)(td.lo - td.begin), end_rel = (int)(td.end - td.begin);
#pragma unroll 1
    for (int it = 0; it < ITEMS; ++it) {
      const int rel0 = (it * WG + (int)threadIdx.x) * VEC;
      if (rel0 >= end_rel) break;
      float v[7][VEC];
      Planes<DT>::load(SrcCtx<DT>{pl}, td.begin + rel0, sh.n_points, v);
      float go[7][VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        float x[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) x[j] = v[j][e];
        const bool valid = P.active && rel0 + e >= lo_rel && rel0 + e < end_rel && finite7(x) && x[6] >= tau;
#pragma unroll
        for (int j = 0; j < 7; ++j) x[j] = valid ? x[j] : 0.0f;
        double y[3], r[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          y[i] = fma(P.M[3 * i], (double)x[0], fma(P.M[3 * i + 1], (double)x[1], fma(P.M[3 * i + 2], (double)x[2], P.t[i])));
          r[i] = y[i] - (double)x[3 + i];
        }
        const double e2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double en = sqrt(e2);
        const bool outl = en > delta;
        const double psi = outl ? delta / en : 1.0;
        const double av[3] = {vv[0] + vv[4] * y[2] - vv[5] * y[1] + vv[6] * y[0],
                              vv[1] + vv[5] * y[0] - vv[3] * y[2] + vv[6] * y[1],
                              vv[2] + vv[3] * y[1] - vv[4] * y[0] + vv[6] * y[2]};
        const double ar = av[0] * r[0] + av[1] * r[1] + av[2] * r[2];
        const double kk = outl ? ar / e2 : 0.0;  // (a . r^) r^ = (a . r) r / e^2
        double b[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) b[i] = psi * (av[i] - kk * r[i]);
        const double wc = (double)x[6] * iC;
        // b + psi (r x v_omega + v_sigma r)
        const double z[3] = {b[0] + psi * (r[1] * vv[5] - r[2] * vv[4] + vv[6] * r[0]),
                             b[1] + psi * (r[2] * vv[3] - r[0] * vv[5] + vv[6] * r[1]),
                             b[2] + psi * (r[0] * vv[4] - r[1] * vv[3] + vv[6] * r[2])};
        go[3][e] = (float)(wc * b[0]);
        go[4][e] = (float)(wc * b[1]);
        go[5][e] = (float)(wc * b[2]);
        go[0][e] = (float)(-wc * (P.M[0] * z[0] + P.M[3] * z[1] + P.M[6] * z[2]));
        go[1][e] = (float)(-wc * (P.M[1] * z[0] + P.M[4] * z[1] + P.M[7] * z[2]));
        go[2][e] = (float)(-wc * (P.M[2] * z[0] + P.M[5] * z[1] + P.M[8] * z[2]));
        go[6][e] = valid ? (float)(-(psi * ar - vF) * iC) : 0.0f;
      }
      const int64_t g0 = td.begin + rel0;
#pragma unroll
      for (int j = 0; j < 7; ++j) store_grad_vec(gout[j], g0, sh.n_points, go[j], VEC, td.lo, td.end);
    }
  }
}

// Workgroups of a kernel that one compute unit holds at once (at least 1).
template <typename K>
static int resident_per_cu(K kernel, int wg) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, wg, 0) != hipSuccess) n = 1;
  return std::max(n, 1);
}

template <int DT>
static hipError_t launch_implicit_t(const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                                    double* hpart, const double* gS, uint32_t iflags, double* v_out, int32_t* status_out,
                                    int grid, int64_t max_tiles, int n_cu, hipStream_t st) {
#define S3A_CASE(WGV, IT)                                                                                   \
  if (lc.wg == WGV && lc.items == IT) {                                                                     \
    static const int per_cu = resident_per_cu(k_hess<DT, WGV, IT>, WGV);                                  \
    const int64_t hgrid = std::max<int64_t>(1, std::min<int64_t>(max_tiles, (int64_t)per_cu * n_cu));      \
    hipError_t e;                                                                                           \
    hipLaunchKernelGGL((k_hess<DT, WGV, IT>), dim3(hgrid), dim3(WGV), 0, st, sh, cd, w, hpart);            \
    if ((e = hipGetLastError()) != hipSuccess) return e;                                                    \
    hipLaunchKernelGGL(k_finalize_implicit, dim3(sh.n_pairs), dim3(64), 0, st, sh, cd, w, hpart, gS, iflags, \
                       v_out, status_out);                                                                  \
    if ((e = hipGetLastError()) != hipSuccess) return e;                                                    \
    hipLaunchKernelGGL((k_igrad<DT, WGV, IT>), dim3(grid), dim3(WGV), 0, st, sh, cd, w);                   \
    return hipGetLastError();                                                                               \
  }
  S3A_CASE(256, 2) S3A_CASE(256, 4) S3A_CASE(256, 8) S3A_CASE(256, 16)
  S3A_CASE(512, 2) S3A_CASE(512, 4) S3A_CASE(512, 8)
#undef S3A_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_implicit(int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                           double* hpart, const double* gS, uint32_t iflags, double* v_out, int32_t* status_out,
                           int grid, int64_t max_tiles, int n_cu, hipStream_t st) {
  if (sh.n_pairs == 0) return hipSuccess;
  return dtype == S3A_F32
             ? launch_implicit_t<S3A_F32>(lc, sh, cd, w, hpart, gS, iflags, v_out, status_out, grid, max_tiles, n_cu, st)
             : launch_implicit_t<S3A_BF16>(lc, sh, cd, w, hpart, gS, iflags, v_out, status_out, grid, max_tiles, n_cu, st);
}

}  // namespace s3a
