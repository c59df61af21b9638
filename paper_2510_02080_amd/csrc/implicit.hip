// Implicit derivative of the solved pose (Sec. III-C.2, eq. (sim3) with Huber
// weights): with F = dL/dxi and H = d^2 L/dxi^2 at the solution S* (exact
// Hessian, second-order terms of Exp included), the implicit function theorem
// gives dl/dtheta = -(dF/dtheta)^T v, v = H^{-1} g_S, for the points and
// confidences theta. One FP64 pass gathers H and F, one FP64 finalize per pair
// solves for v, and one pass writes the per-point terms.
#include "implicit.h"

#include "finalize.h"

namespace s3a {

// Sums of the Hessian pass, per run of a workgroup's rows within one pair
// (weights om = c psi, c-weighted; divided by C = sum m c in the finalize).
// y = S* p, r = y - q, all in FP64 (the rank-one sums in FP32, see below):
//   0 sum om, 1-3 sum om y, 4-9 sum om y y^T (xx xy xz yy yz zz),
//   10-12 sum om r, 13-21 sum om y_a r_b (row-major a, b),
//   22-49 sum over points outside delta of c psi / e^2 u u^T, u = (r, y x r, y . r)
//         (packed lower triangle, row i at i (i + 1) / 2),
//   50 C, 51 unused (zero; 52 values halve evenly in the reduction).
constexpr int HSTAT = 52;

// One FP64 value's two halves through a lane-swap builtin pair.
template <bool HALF16>
__device__ inline void swap_f64(double& x, double& y) {
  const unsigned long long a = (unsigned long long)__double_as_longlong(x);
  const unsigned long long b = (unsigned long long)__double_as_longlong(y);
  unsigned alo = (unsigned)a, ahi = (unsigned)(a >> 32), blo = (unsigned)b, bhi = (unsigned)(b >> 32);
  if constexpr (HALF16) {
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    alo = l[0]; blo = l[1]; ahi = h[0]; bhi = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    alo = l[0]; blo = l[1]; ahi = h[0]; bhi = h[1];
  }
  x = __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo));
  y = __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
}

// Sums of the HSTAT per-lane values over the workgroup, stored to out. Within
// a wavefront the values are halved twice by lane swaps: swapping lanes 32-63
// of value j with lanes 0-31 of value j + 26 and adding leaves lanes 0-31 with
// value j and lanes 32-63 with value j + 26, each summed over two lanes; the
// same with 16-lane swaps within each half leaves lane l with values
// 13 (l / 16) + s, s < 13, summed over four lanes. A butterfly over each row of
// 16 lanes finishes them (about a third of the instructions of reducing all 52
// values over 64 lanes), then one lane per row stores its 13 totals to LDS.
template <int WG>
__device__ inline void block_store_h(double (&acc)[HSTAT], double (*red)[HSTAT], double* out) {
  static_assert(HSTAT == 52, "the lane halving takes 52 values");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double z[26];
#pragma unroll
  for (int j = 0; j < 26; ++j) {
    double x = acc[j], y = acc[j + 26];
    swap_f64<false>(x, y);
    z[j] = x + y;
  }
  double q[13];
#pragma unroll
  for (int j = 0; j < 13; ++j) {
    double x = z[j], y = z[j + 13];
    swap_f64<true>(x, y);
    q[j] = x + y;
  }
#pragma unroll
  for (int j = 0; j < 13; ++j) q[j] += dpp_f64<0xb1, 0xf>(q[j]);   // quad_perm [1,0,3,2]
#pragma unroll
  for (int j = 0; j < 13; ++j) q[j] += dpp_f64<0x4e, 0xf>(q[j]);   // quad_perm [2,3,0,1]
#pragma unroll
  for (int j = 0; j < 13; ++j) q[j] += dpp_f64<0x141, 0xf>(q[j]);  // row_half_mirror
#pragma unroll
  for (int j = 0; j < 13; ++j) q[j] += dpp_f64<0x140, 0xf>(q[j]);  // row_mirror
  if ((lane & 15) == 0) {
#pragma unroll
    for (int j = 0; j < 13; ++j) red[wv][13 * (lane >> 4) + j] = q[j];
  }
  __syncthreads();
  if ((int)threadIdx.x < HSTAT) {
    double s = 0.0;
#pragma unroll
    for (int w4 = 0; w4 < WG / 64; ++w4) s += red[w4][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// The Hessian pass reads 8-byte vectors per plane (2 FP32 or 4 BF16 points):
// its per-lane sums take 74 registers, and half-width raw buffers and fewer
// points in flight per lane let three wavefronts share a SIMD.
typedef unsigned int s3a_u2 __attribute__((ext_vector_type(2)));
template <int DT>
struct HalfVec;
template <>
struct HalfVec<S3A_F32> {
  static constexpr int VEC = 2;
  typedef s3a_u2 Raw[7];
  __device__ static inline void fetch(const SrcCtx<S3A_F32>& src, int64_t g0, int64_t n, Raw& r) {
    if (g0 + 2 <= n) {
#pragma unroll
      for (int j = 0; j < 7; ++j)
        r[j] = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u2*)(static_cast<const uint32_t*>(src.pl[j]) + g0));
    } else {
#pragma unroll
      for (int j = 0; j < 7; ++j)
#pragma unroll
        for (int e = 0; e < 2; ++e) r[j][e] = (g0 + e < n) ? static_cast<const uint32_t*>(src.pl[j])[g0 + e] : 0u;
    }
  }
  __device__ static inline float elem(const Raw& r, int j, int e) { return __uint_as_float(r[j][e]); }
};
template <>
struct HalfVec<S3A_BF16> {
  static constexpr int VEC = 4;
  typedef s3a_u2 Raw[7];
  __device__ static inline void fetch(const SrcCtx<S3A_BF16>& src, int64_t g0, int64_t n, Raw& r) {
    if (g0 + 4 <= n) {
#pragma unroll
      for (int j = 0; j < 7; ++j)
        r[j] = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u2*)(static_cast<const uint16_t*>(src.pl[j]) + g0));
    } else {
#pragma unroll
      for (int j = 0; j < 7; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const uint16_t* hp = static_cast<const uint16_t*>(src.pl[j]);
          const uint32_t a = (g0 + 2 * i < n) ? hp[g0 + 2 * i] : 0u;
          const uint32_t b = (g0 + 2 * i + 1 < n) ? hp[g0 + 2 * i + 1] : 0u;
          r[j][i] = a | (b << 16);
        }
    }
  }
  __device__ static inline float elem(const Raw& r, int j, int e) {
    const uint32_t u = r[j][e >> 1];
    return __uint_as_float((e & 1) ? (u & 0xffff0000u) : (u << 16));
  }
};

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

// Rows of the Hessian pass: a tile of the call holds HessRows<DT, ITEMS> rows
// of WG x HalfVec<DT>::VEC elements; global row r of tile t is r - t * RPT of
// that tile. Workgroup g of G sweeps the rows [R g / G, R (g + 1) / G) of the
// R = tiles x RPT rows, so every workgroup has the same share up to one row.
template <int DT, int ITEMS>
struct HessRows {
  static constexpr int RPT = ITEMS * Planes<DT>::VEC / HalfVec<DT>::VEC;
};

// The workgroup whose rows hold global row r.
__host__ __device__ inline int hess_wg_of_row(int64_t r, int64_t R, int G) { return (int)(((r + 1) * G - 1) / R); }

// Each workgroup streams each run of its rows that belongs to one pair as one
// pipelined sweep (rows of consecutive tiles lie end to end) and reduces its
// per-lane sums once per run, into slot g + k for workgroup g and pair k (the
// runs are ordered by workgroup and pair, so the slots are distinct; the
// finalize adds the slots of the workgroups that cover the pair's rows). The
// grid changes only the summation order.
template <int DT, int WG, int ITEMS>
__global__ __launch_bounds__(WG) void k_hess(Shape sh, const CallDesc* __restrict__ cd, Work w, double* hpart) {
  using HV = HalfVec<DT>;
  constexpr int VEC = HV::VEC;
  constexpr int RPT = HessRows<DT, ITEMS>::RPT;
  constexpr int STRIDE = WG * VEC;
  __shared__ double red[WG / 64][HSTAT];
  const int64_t R = (int64_t)(*w.total_tiles) * RPT;
  const int G = (int)gridDim.x, g = (int)blockIdx.x;
  const int64_t r0 = R * g / G, r1 = R * (g + 1) / G;
  const void* pl[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) pl[j] = cd->planes[j];
  const SrcCtx<DT> src{pl};
  const float tau = sh.tau;
  const double delta = sh.delta;
#pragma unroll 1
  for (int64_t row = r0; row < r1;) {
    const int t = (int)(row / RPT);
    const TileDesc td = load_tile(w.tiles + t);
    const PairSched sc = w.sched[td.pair];
    const int64_t re = min(r1, (int64_t)(sc.tile0 + sc.ntiles) * RPT);  // this run: rows [row, re)
    const int64_t base = td.begin + (row - (int64_t)t * RPT) * STRIDE;   // element of the run's first row
    const int64_t stop = min(w.tiles[(re - 1) / RPT].end, base + (re - row) * STRIDE);
    const PointParams P = load_params(w.params + td.pair);
    double a[HSTAT];
#pragma unroll
    for (int j = 0; j < HSTAT; ++j) a[j] = 0.0;
    float b[28];  // the rank-one sums (22-49), per lane in FP32
#pragma unroll
    for (int j = 0; j < 28; ++j) b[j] = 0.0f;
    const int64_t lo64 = td.lo - base;
    const int lo_rel = lo64 < 0 ? 0 : (int)lo64;
    const int end_rel = (int)(stop > base ? stop - base : 0);
    pipelined_run<WG, VEC, typename HV::Raw>(
        (int)(re - row), end_rel, [&](int rel, typename HV::Raw& q) { HV::fetch(src, base + rel, sh.n_points, q); },
        [&](const typename HV::Raw& raw, int rel0) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            float x[7];
#pragma unroll
            for (int j = 0; j < 7; ++j) x[j] = HV::elem(raw, j, e);
            // elements outside the pair (a run's first and last vectors) are zeroed on a
            // branch the other vectors skip: they add nothing, whatever they hold
            const bool in = P.active && rel0 + e >= lo_rel && rel0 + e < end_rel;
            if (!in) {
#pragma unroll
              for (int j = 0; j < 7; ++j) x[j] = 0.0f;
            }
            double y[3], r[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              y[i] = fma(P.M[3 * i], (double)x[0],
                         fma(P.M[3 * i + 1], (double)x[1], fma(P.M[3 * i + 2], (double)x[2], P.t[i])));
              r[i] = y[i] - (double)x[3 + i];
            }
            double e2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            // a NaN/Inf in p or q makes e2 NaN/Inf (FP64 sums of FP32 values cannot
            // overflow), so two checks find every non-finite point; such a point is
            // zeroed on a branch that wavefronts without one skip
            bool valid = in && x[6] >= tau;
            if (!(__builtin_isfinite(e2) && __builtin_isfinite(x[6]))) {
              valid = false;
#pragma unroll
              for (int i = 0; i < 3; ++i) y[i] = r[i] = 0.0;
              e2 = 0.0;
            }
            const double c = valid ? (double)x[6] : 0.0;  // invalid points weigh nothing
            // 1 / |r|, used only outside delta (|r| > delta > 0): the hardware
            // estimate and one Newton step (relative error near 1e-14)
            double ie = __builtin_amdgcn_rsq(e2);
            ie = ie * fma(-0.5 * e2 * ie, ie, 1.5);
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
            // rank-one correction of the Huber Hessian outside delta: c psi / e^2 u u^T,
            // in FP32: it is the Hessian of the few down-weighted points (psi =
            // delta / |r| < 1), a small share of H, so FP32 products and per-lane
            // sums leave H's relative error near 1e-9
            const float k1 = outl ? (float)(om * ie * ie) : 0.0f;
            const float yf[3] = {(float)y[0], (float)y[1], (float)y[2]};
            const float rf[3] = {(float)r[0], (float)r[1], (float)r[2]};
            const float u[7] = {rf[0], rf[1], rf[2], yf[1] * rf[2] - yf[2] * rf[1], yf[2] * rf[0] - yf[0] * rf[2],
                                yf[0] * rf[1] - yf[1] * rf[0], yf[0] * rf[0] + yf[1] * rf[1] + yf[2] * rf[2]};
#pragma unroll
            for (int i = 0; i < 7; ++i) {
              const float ku = k1 * u[i];
#pragma unroll
              for (int j = 0; j <= i; ++j) b[i * (i + 1) / 2 + j] = fmaf(ku, u[j], b[i * (i + 1) / 2 + j]);
            }
            a[50] += c;
          }
        });
#pragma unroll
    for (int j = 0; j < 28; ++j) a[22 + j] = (double)b[j];
    block_store_h<WG>(a, red, hpart + (int64_t)(g + td.pair) * HSTAT);
    row = re;
  }
}

// Per pair: H and F from the sums, the upstream gradient in tangent form,
// v = H^{-1} g_S; published for the gradient pass (state: g = v, cost_lin =
// v^T F, C; params: active).
__global__ __launch_bounds__(64) void k_finalize_implicit(Shape sh, const CallDesc* __restrict__ cd, Work w,
                                                          const double* __restrict__ hpart, int rpt, int hess_grid,
                                                          const double* __restrict__ gS, uint32_t iflags, double* v_out,
                                                          int32_t* status_out) {
  const int k = blockIdx.x;
  if (k >= sh.n_pairs) return;
  const PairSched sc = w.sched[k];
  const int lane = threadIdx.x & 63;
  double s[HSTAT];
#pragma unroll
  for (int j = 0; j < HSTAT; ++j) s[j] = 0.0;
  const int64_t R = (int64_t)(*w.total_tiles) * rpt;
  const int g_lo = hess_wg_of_row((int64_t)sc.tile0 * rpt, R, hess_grid);
  const int g_hi = hess_wg_of_row((int64_t)(sc.tile0 + sc.ntiles) * rpt - 1, R, hess_grid);
  for (int g = g_lo + lane; g <= g_hi; g += 64) {
    if (R * (g + 1) / hess_grid == R * g / hess_grid) continue;  // a workgroup with no rows wrote no slot
    const double* p = hpart + (int64_t)(g + k) * HSTAT;
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
    hipLaunchKernelGGL(k_finalize_implicit, dim3(sh.n_pairs), dim3(64), 0, st, sh, cd, w, hpart,            \
                       HessRows<DT, IT>::RPT, (int)hgrid, gS, iflags, v_out, status_out);                   \
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
