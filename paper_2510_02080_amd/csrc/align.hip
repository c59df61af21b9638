// Dense Sim(3) alignment kernels: tile scheduling, point passes, and the FP64
// per-pair finalize (Sec. III-C.2, eq. (sim3); Huber IRLS refinement).
//
// A call runs 1 + K (+1) passes over every pair: the moments pass of the
// weighted Umeyama closed form, K Gauss-Newton passes, and optionally a cost
// pass at the final iterate. Between passes each pair's tile partials are
// summed in a fixed order and its 7x7 (or 3x3 / 4x4) system is solved in FP64.
#include "align_kernels.h"
#include "align_launch.h"

namespace s3a {

// ------------------------------------------------------------------ schedule

// One workgroup. Checks every pair's range; if any pair is malformed, every
// pair is marked bad (so a malformed offsets array cannot make the tile table
// larger than the host-side bound). Then an exclusive scan of tile counts.
__global__ __launch_bounds__(1024) void k_sched(Shape sh, const CallDesc* __restrict__ cd, Work w) {
  __shared__ int32_t buf[1024];
  __shared__ int32_t carry;
  const int n = sh.n_pairs;
  const int64_t T = sh.tile_elems;
  int bad_local = 0;
  for (int k = threadIdx.x; k < n; k += 1024) {
    const int64_t a = cd->offsets[k], b = cd->offsets[k + 1];
    bad_local |= !(a >= 0 && a <= b && b <= sh.n_points);
  }
  const int any_bad = __syncthreads_or(bad_local);
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int k = base + threadIdx.x;
    int32_t nt = 0;
    PairSched s{};
    if (k < n) {
      int64_t a = cd->offsets[k], b = cd->offsets[k + 1];
      s.bad = any_bad;
      if (any_bad) { a = 0; b = 0; }
      s.a = a;
      s.b = b;
      const int64_t b0 = a & ~(TILE_ALIGN - 1);
      nt = (b > a) ? (int32_t)((b - b0 + T - 1) / T) : 1;
      s.ntiles = nt;
    }
    buf[threadIdx.x] = nt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int32_t x = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += x;
      __syncthreads();
    }
    if (k < n) {
      s.tile0 = carry + buf[threadIdx.x] - nt;
      w.sched[k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *w.total_tiles = carry;
}

__global__ void k_sched_fill(Shape sh, Work w) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= sh.n_pairs) return;
  const PairSched s = w.sched[k];
  const int64_t b0 = s.a & ~(TILE_ALIGN - 1);
  for (int j = 0; j < s.ntiles; ++j) {
    TileDesc t;
    t.pair = k;
    t.pad = 0;
    if (s.b > s.a) {
      t.begin = b0 + (int64_t)j * sh.tile_elems;
      t.end = t.begin + sh.tile_elems < s.b ? t.begin + sh.tile_elems : s.b;
      t.lo = s.a;
    } else {
      t.begin = t.end = t.lo = s.a;
    }
    w.tiles[s.tile0 + j] = t;
  }
}

// ------------------------------------------------------------------ point passes

template <int DT, int MODE, int WG, int ITEMS>
__global__ __launch_bounds__(WG) void k_pass(Shape sh, const CallDesc* __restrict__ cd, Work w,
                                              int32_t tile_lo, int32_t tile_hi) {
  __shared__ double red[WG / 64][NSTAT];
  const int total = tile_hi >= 0 ? tile_hi : *w.total_tiles;
  const void* pl[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) pl[j] = cd->planes[j];
  for (int t = tile_lo + (int)blockIdx.x; t < total; t += (int)gridDim.x) {
    const TileDesc td = w.tiles[t];
    const PointParams P = w.params[td.pair];
    tile_body<DT, MODE, WG, ITEMS>(sh, pl, td, P, red, w.partials + (int64_t)t * NSTAT);
  }
}

// ------------------------------------------------------------------ finalize

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

__device__ inline void publish(PointParams* P, const Sim3d& S, const double* c, int active) {
  PointParams p;
  for (int i = 0; i < 9; ++i) { p.M[i] = S.s * S.R[i]; p.Mf[i] = (float)p.M[i]; }
  for (int i = 0; i < 3; ++i) { p.t[i] = S.t[i]; p.c[i] = c[i]; }
  p.inv_C = 0.0f;
  p.scale = 0.0f;
  p.L = 0.0f;
  p.active = active;
  p.pad = 0;
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

// Moments pass -> weighted Umeyama start (or the caller's), validity, centre.
__device__ void finalize_moments(const Shape& sh, const CallDesc* cd, Work& w, int k, const PairSched& sc,
                                 const double* s) {
  const double nan = __builtin_nan("");
  PairState st;
  st.S = sim3_identity();
  st.C = s[0];
  st.V = (int64_t)s[17];
  st.nnf = (int64_t)s[18];
  st.cost_lin = nan;
  for (int i = 0; i < 28; ++i) st.H[i] = nan;
  for (int i = 0; i < 7; ++i) st.g[i] = nan;
  st.inl_lin = 0;
  st.iters = 0;
  st.status = S3A_PAIR_OK;
  st.cq[0] = st.cq[1] = st.cq[2] = 0.0;
  if (sc.bad) {
    st.status = S3A_PAIR_BADRANGE;
  } else if (st.V == 0) {
    st.status = st.nnf > 0 ? S3A_PAIR_NONFINITE : S3A_PAIR_EMPTY;
  } else if (!(st.C > 0.0)) {
    st.status = S3A_PAIR_DEGENERATE;
  } else {
    Sim3d S0;
    const int u = umeyama_from_moments(s[0], s + 1, s + 4, s[7], s + 8, &S0, st.cq);
    if (cd->init) {
      st.S = load_sim3(cd->init + k);
      if (!sim3_finite(st.S)) st.status = S3A_PAIR_NONFINITE;
    } else if (u != UMEYAMA_OK) {
      st.status = u == UMEYAMA_EMPTY ? S3A_PAIR_EMPTY : S3A_PAIR_DEGENERATE;
    } else {
      st.S = S0;
    }
  }
  const bool more = st.status == S3A_PAIR_OK && (sh.K > 0 || (sh.flags & S3A_FLAG_FINAL_COST));
  if (!more) write_outputs(cd, k, st, nan, 0);
  publish(w.params + k, st.S, st.cq, more ? 1 : 0);
  w.state[k] = st;
}

// Gauss-Newton pass `pass` (1..K): assemble H, g in centred coordinates from the
// 17 statistics, Cholesky solve, map the step back, S <- Exp(xi) S.
__device__ void finalize_gn(const Shape& sh, const CallDesc* cd, Work& w, int k, int pass, const double* s) {
  PairState st = w.state[k];
  if (st.status != S3A_PAIR_OK || !w.params[k].active) return;
  const double nan = __builtin_nan("");
  const double* c = st.cq;
  // centred system (y_c = y - c): J' = [I, -[y_c]x, y_c]
  const double A0 = s[0], a[3] = {s[1], s[2], s[3]};
  const double Bxx = s[4], Bxy = s[5], Bxz = s[6], Byy = s[7], Byz = s[8], Bzz = s[9];
  const double trB = Bxx + Byy + Bzz;
  double H[49];
  for (int i = 0; i < 49; ++i) H[i] = 0.0;
  for (int i = 0; i < 3; ++i) H[8 * i] = A0;
  // rho-omega block: -[a]x
  H[0 * 7 + 4] = a[2];  H[0 * 7 + 5] = -a[1];
  H[1 * 7 + 3] = -a[2]; H[1 * 7 + 5] = a[0];
  H[2 * 7 + 3] = a[1];  H[2 * 7 + 4] = -a[0];
  for (int i = 0; i < 3; ++i) H[7 * i + 6] = a[i];
  const double B[9] = {Bxx, Bxy, Bxz, Bxy, Byy, Byz, Bxz, Byz, Bzz};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) H[7 * (3 + i) + 3 + j] = (i == j ? trB : 0.0) - B[3 * i + j];
  H[48] = trB;
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < i; ++j) H[7 * i + j] = H[7 * j + i];
  const double gs[7] = {s[10], s[11], s[12], s[13], s[14], s[15], s[16]};
  st.cost_lin = s[17] / st.C;
  st.inl_lin = (int64_t)s[18];
  double Hc[49], mg[7], x[7];
  for (int i = 0; i < 49; ++i) Hc[i] = H[i];
  for (int i = 0; i < 7; ++i) mg[i] = -gs[i];
  bool ok = cholesky_solve<7>(Hc, mg, x);
  if (ok) {
    // xi = Ad(translation c) xi': rho = rho' + c x omega - sigma c
    double xi[7];
    xi[0] = x[0] + (c[1] * x[5] - c[2] * x[4]) - x[6] * c[0];
    xi[1] = x[1] + (c[2] * x[3] - c[0] * x[5]) - x[6] * c[1];
    xi[2] = x[2] + (c[0] * x[4] - c[1] * x[3]) - x[6] * c[2];
    for (int i = 3; i < 7; ++i) xi[i] = x[i];
    const Sim3d Snew = sim3_compose(sim3_exp(xi), st.S);
    if (!sim3_finite(Snew)) {
      st.status = S3A_PAIR_NONFINITE;
    } else {
      st.S = Snew;
      st.iters = pass;
      // report H, g in the uncentred tangent: H = A^-T H' A^-1, g = A^-T g',
      // A^-1 = [[I, -[c]x, c], [0, I, 0], [0, 0, 1]], normalised by C.
      double Ai[49];
      for (int i = 0; i < 49; ++i) Ai[i] = (i % 8 == 0) ? 1.0 : 0.0;
      Ai[0 * 7 + 4] = c[2];  Ai[0 * 7 + 5] = -c[1];
      Ai[1 * 7 + 3] = -c[2]; Ai[1 * 7 + 5] = c[0];
      Ai[2 * 7 + 3] = c[1];  Ai[2 * 7 + 4] = -c[0];
      Ai[0 * 7 + 6] = c[0];  Ai[1 * 7 + 6] = c[1];  Ai[2 * 7 + 6] = c[2];
      double T1[49];
      for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 7; ++j) {
          double v = 0.0;
          for (int m = 0; m < 7; ++m) v += H[7 * i + m] * Ai[7 * m + j];
          T1[7 * i + j] = v;
        }
      int u = 0;
      for (int i = 0; i < 7; ++i)
        for (int j = i; j < 7; ++j) {
          double v = 0.0;
          for (int m = 0; m < 7; ++m) v += Ai[7 * m + i] * T1[7 * m + j];
          st.H[u++] = v / st.C;
        }
      for (int i = 0; i < 7; ++i) {
        double v = 0.0;
        for (int m = 0; m < 7; ++m) v += Ai[7 * m + i] * gs[m];
        st.g[i] = v / st.C;
      }
    }
  } else {
    st.status = S3A_PAIR_DEGENERATE;
  }
  const bool failed = st.status != S3A_PAIR_OK;
  const bool last = pass == sh.K;
  const bool final_pass = (sh.flags & S3A_FLAG_FINAL_COST) != 0;
  if (failed || (last && !final_pass)) write_outputs(cd, k, st, nan, 0);
  publish(w.params + k, st.S, st.cq, (failed || (last && !final_pass)) ? 0 : 1);
  w.state[k] = st;
}

__device__ void finalize_final_cost(const CallDesc* cd, Work& w, int k, const double* s) {
  const PairState st = w.state[k];
  if (st.status != S3A_PAIR_OK || !w.params[k].active) return;
  write_outputs(cd, k, st, s[17] / st.C, (int64_t)s[18]);
  w.params[k].active = 0;
}

// kind: 0 moments, 1 Gauss-Newton, 2 final cost.
__global__ __launch_bounds__(64) void k_finalize(Shape sh, const CallDesc* __restrict__ cd, Work w, int kind,
                                                 int pass, int32_t pair_lo) {
  const int k = pair_lo + (int)blockIdx.x;
  if (k >= sh.n_pairs) return;
  const PairSched sc = w.sched[k];
  double s[NSTAT];
  pair_sums(w, sc, NSTAT, s);
  if (threadIdx.x != 0) return;
  if (kind == 0) finalize_moments(sh, cd, w, k, sc, s);
  else if (kind == 1) finalize_gn(sh, cd, w, k, pass, s);
  else finalize_final_cost(cd, w, k, s);
}

// ------------------------------------------------------------------ cost / adjoint prep

// S' = Exp(xi) S per pair; the adjoint also needs 1/C, gL and L.
__global__ void k_prep(Shape sh, const CallDesc* __restrict__ cd, Work w, int adjoint) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= sh.n_pairs) return;
  Sim3d S = load_sim3(cd->S_in + k);
  if (cd->xi) S = sim3_compose(sim3_exp(cd->xi + 7 * k), S);
  const double c0[3] = {0.0, 0.0, 0.0};
  int active = 1;
  if (adjoint) active = cd->C_in[k] > 0.0;
  publish(w.params + k, S, c0, active);
  if (adjoint) {
    w.params[k].inv_C = active ? (float)(1.0 / cd->C_in[k]) : 0.0f;
    w.params[k].scale = (float)cd->gL[k];
    w.params[k].L = (float)cd->L_in[k];
  }
}

__global__ __launch_bounds__(64) void k_finalize_cost(Shape sh, const CallDesc* __restrict__ cd, Work w) {
  const int k = blockIdx.x;
  if (k >= sh.n_pairs) return;
  const PairSched sc = w.sched[k];
  double s[NSTAT];
  pair_sums(w, sc, 3, s);
  if (threadIdx.x != 0) return;
  const double C = s[0];
  cd->C_out[k] = C;
  cd->L_out[k] = C > 0.0 ? s[1] / C : __builtin_nan("");
}

}  // namespace s3a

// ------------------------------------------------------------------ launchers

namespace s3a {

template <int DT, int MODE>
static hipError_t launch_pass_t(const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                                int32_t tile_lo, int32_t tile_hi, int grid, hipStream_t st) {
#define S3A_CASE(WGV, IT)                                                                                   \
  if (lc.wg == WGV && lc.items == IT) {                                                                     \
    hipLaunchKernelGGL((k_pass<DT, MODE, WGV, IT>), dim3(grid), dim3(WGV), 0, st, sh, cd, w, tile_lo, tile_hi); \
    return hipGetLastError();                                                                               \
  }
  S3A_CASE(256, 2) S3A_CASE(256, 4) S3A_CASE(256, 8) S3A_CASE(512, 2) S3A_CASE(512, 4) S3A_CASE(512, 8)
#undef S3A_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_pass(int dtype, int mode, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd,
                       const Work& w, int32_t tile_lo, int32_t tile_hi, int grid, hipStream_t st) {
  if (dtype == S3A_F32) {
    if (mode == MODE_MOMENTS) return launch_pass_t<S3A_F32, MODE_MOMENTS>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN) return launch_pass_t<S3A_F32, MODE_GN>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_COST) return launch_pass_t<S3A_F32, MODE_COST>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
  } else {
    if (mode == MODE_MOMENTS) return launch_pass_t<S3A_BF16, MODE_MOMENTS>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN) return launch_pass_t<S3A_BF16, MODE_GN>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_COST) return launch_pass_t<S3A_BF16, MODE_COST>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sched(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st) {
  hipLaunchKernelGGL(k_sched, dim3(1), dim3(1024), 0, st, sh, cd, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || sh.n_pairs == 0) return e;
  hipLaunchKernelGGL(k_sched_fill, dim3((sh.n_pairs + 255) / 256), dim3(256), 0, st, sh, w);
  return hipGetLastError();
}

hipError_t launch_finalize(int kind, const Shape& sh, const CallDesc* cd, const Work& w, int pass, int32_t pair_lo,
                           int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(n), dim3(64), 0, st, sh, cd, w, kind, pass, pair_lo);
  return hipGetLastError();
}

hipError_t launch_prep(const Shape& sh, const CallDesc* cd, const Work& w, int adjoint, hipStream_t st) {
  if (sh.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3((sh.n_pairs + 127) / 128), dim3(128), 0, st, sh, cd, w, adjoint);
  return hipGetLastError();
}

hipError_t launch_finalize_cost(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st) {
  if (sh.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize_cost, dim3(sh.n_pairs), dim3(64), 0, st, sh, cd, w);
  return hipGetLastError();
}

}  // namespace s3a
