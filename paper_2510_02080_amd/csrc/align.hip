// Dense Sim(3) alignment kernels: tile scheduling, point passes, and the FP64
// per-pair finalize (Sec. III-C.2, eq. (sim3); Huber IRLS refinement).
//
// A call runs 1 + K (+1) passes over every pair: the moments pass of the
// weighted Umeyama closed form, K Gauss-Newton passes, and optionally a cost
// pass at the final iterate. Between passes each pair's tile partials are
// summed in a fixed order and its 7x7 (or 3x3 / 4x4) system is solved in FP64.
#include "align_kernels.h"
#include "align_launch.h"
#include "finalize.h"

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
    const TileDesc td = load_tile(w.tiles + t);
    const PointParams P = load_params(w.params + td.pair);
    const SrcCtx<DT> src = make_src<DT>(pl, w, td);
    tile_body<DT, MODE, WG, ITEMS>(sh, src, td, P, red, w.partials + (int64_t)t * NSTAT);
  }
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
  S3A_CASE(256, 2) S3A_CASE(256, 4) S3A_CASE(256, 8) S3A_CASE(256, 16)
  S3A_CASE(512, 2) S3A_CASE(512, 4) S3A_CASE(512, 8)
#undef S3A_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_pass(int dtype, int mode, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd,
                       const Work& w, int32_t tile_lo, int32_t tile_hi, int grid, hipStream_t st) {
  if (dtype == DT_DEPTH_F32) {
    if (mode == MODE_MOMENTS) return launch_pass_t<DT_DEPTH_F32, MODE_MOMENTS>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN) return launch_pass_t<DT_DEPTH_F32, MODE_GN>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN_NC) return launch_pass_t<DT_DEPTH_F32, MODE_GN_NC>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    return hipErrorInvalidValue;
  }
  if (dtype == DT_DEPTH_BF16) {
    if (mode == MODE_MOMENTS) return launch_pass_t<DT_DEPTH_BF16, MODE_MOMENTS>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN) return launch_pass_t<DT_DEPTH_BF16, MODE_GN>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN_NC) return launch_pass_t<DT_DEPTH_BF16, MODE_GN_NC>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    return hipErrorInvalidValue;
  }
  if (dtype == S3A_F32) {
    if (mode == MODE_MOMENTS) return launch_pass_t<S3A_F32, MODE_MOMENTS>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN) return launch_pass_t<S3A_F32, MODE_GN>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN_NC) return launch_pass_t<S3A_F32, MODE_GN_NC>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_COST) return launch_pass_t<S3A_F32, MODE_COST>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
  } else {
    if (mode == MODE_MOMENTS) return launch_pass_t<S3A_BF16, MODE_MOMENTS>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN) return launch_pass_t<S3A_BF16, MODE_GN>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
    if (mode == MODE_GN_NC) return launch_pass_t<S3A_BF16, MODE_GN_NC>(lc, sh, cd, w, tile_lo, tile_hi, grid, st);
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

// Depth input: the caller's cameras in pass form (reciprocal focal lengths,
// offsets), geometry checked and sanitised; a pair with invalid geometry, or
// with more elements than its frames hold, is marked bad (BADRANGE).
__global__ void k_depth_prep(Shape sh, const CallDesc* __restrict__ cd, Work w) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= sh.n_pairs) return;
  const s3a_depth_pair& src = cd->depth[k];
  int W = src.width, HW = src.frame_pixels, nf = src.n_frames;
  bool ok = W >= 1 && HW >= W && HW % W == 0 && nf >= 1 && nf <= DEPTH_MAX_FRAMES && src.reserved == 0;
  const PairSched sc = w.sched[k];
  if (ok && !sc.bad) ok = sc.b - sc.a <= (int64_t)nf * HW;
  if (!ok) {
    W = 1;
    HW = 1;
    nf = 1;
  }
  DepthPair dp;
  dp.width = W;
  dp.rows = HW / W;
  dp.frame_pixels = HW;
  dp.n_frames = nf;
  dp.inv_width = 1.0f / (float)W;
  dp.inv_frame = 1.0f / (float)HW;
  dp.pad[0] = dp.pad[1] = 0;
  for (int f = 0; f < DEPTH_MAX_FRAMES; ++f) {
    const s3a_camera* in[2] = {src.p + f, src.q + f};
    DepthCam* out[2] = {dp.p + f, dp.q + f};
    for (int side = 0; side < 2; ++side) {
      const s3a_camera& c = *in[side];
      DepthCam& o = *out[side];
      o.ifx = 1.0f / c.fx;
      o.ify = 1.0f / c.fy;
      o.ox = -c.cx / c.fx;
      o.oy = -c.cy / c.fy;
      for (int i = 0; i < 9; ++i) o.R[i] = c.R[i];
      for (int i = 0; i < 3; ++i) o.t[i] = c.t[i];
    }
  }
  w.dpairs[k] = dp;
  if (!ok) w.sched[k].bad = 1;
}

hipError_t launch_depth_prep(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st) {
  if (sh.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_depth_prep, dim3((sh.n_pairs + 63) / 64), dim3(64), 0, st, sh, cd, w);
  return hipGetLastError();
}

hipError_t launch_finalize_cost(const Shape& sh, const CallDesc* cd, const Work& w, hipStream_t st) {
  if (sh.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize_cost, dim3(sh.n_pairs), dim3(64), 0, st, sh, cd, w);
  return hipGetLastError();
}

}  // namespace s3a
