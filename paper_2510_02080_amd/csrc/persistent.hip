// Batched alignment in one persistent launch.
//
// Work items are (pass, tile) tickets handed out by one atomic counter in
// pass-major order: every tile of pass k comes before any tile of pass k+1.
// A tile of pass k >= 1 of pair j waits until pair j's pass k-1 has been
// finalized; that depends only on tickets smaller than its own, all of which
// were taken earlier by running workgroups, so the smallest unfinished ticket
// can always proceed (no deadlock, whatever the number of resident
// workgroups). The last tile of a pair to arrive in a pass sums the pair's
// partials in a fixed order, runs the FP64 finalize, and publishes the next
// iterate with a release store; waiting tiles acquire it. Waits are bounded:
// a wait that exceeds its limit raises a global abort word, every workgroup
// then drains, and the pairs left unfinished keep the ABORTED status written
// before the launch.
#include <algorithm>

#include "align_kernels.h"
#include "align_launch.h"
#include "finalize.h"

namespace s3a {

constexpr int CTL_TICKET = 0;  // 64-bit ticket counter in counters[0..1]
constexpr int CTL_ABORT = 2;
constexpr int ARRIVE_BASE = 64;
constexpr uint32_t SPIN_LIMIT = 1u << 23;  // ~0.5 s of polling

__global__ void k_fill_zero(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_fill_zero(uint32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// Outputs of a batched call start as ABORTED (identity, NaN cost); every pair
// that completes overwrites them.
__global__ void k_init_outputs(Shape sh, const CallDesc* __restrict__ cd) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= sh.n_pairs) return;
  store_sim3(cd->S_out + k, sim3_identity());
  if (cd->info) {
    s3a_align_info* I = cd->info + k;
    const double nan = __builtin_nan("");
    I->cost = nan;
    I->final_cost = nan;
    I->weight_sum = nan;
    for (int i = 0; i < 28; ++i) I->H[i] = nan;
    for (int i = 0; i < 7; ++i) I->g[i] = nan;
    I->n_valid = I->n_nonfinite = I->n_inliers = I->final_inliers = 0;
    I->status = S3A_PAIR_ABORTED;
    I->iters = 0;
  }
}

__device__ inline uint32_t ld_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DT, int WG, int ITEMS>
__global__ __launch_bounds__(WG, 2) void k_persistent(Shape sh, const CallDesc* __restrict__ cd, Work w) {
  __shared__ double red[WG / 64][NSTAT];
  __shared__ unsigned long long s_ticket;
  __shared__ int s_flag;
  const int npass = 1 + sh.K + ((sh.flags & S3A_FLAG_FINAL_COST) ? 1 : 0);
  const int64_t total_tiles = *w.total_tiles;
  const uint64_t total_tickets = (uint64_t)total_tiles * (uint64_t)npass;
  unsigned long long* ticket = reinterpret_cast<unsigned long long*>(w.counters + CTL_TICKET);
  uint32_t* abort_word = w.counters + CTL_ABORT;
  uint32_t* arrive = w.counters + ARRIVE_BASE;
  const void* pl[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) pl[j] = cd->planes[j];

  for (;;) {
    if (threadIdx.x == 0) s_ticket = atomicAdd(ticket, 1ull);
    __syncthreads();
    const uint64_t x = s_ticket;
    if (x >= total_tickets) break;
    const int pass = (int)(x / (uint64_t)total_tiles);
    const int t = (int)(x % (uint64_t)total_tiles);
    const TileDesc td = load_tile(w.tiles + t);
    const int j = td.pair;
    if (pass > 0) {
      if (threadIdx.x == 0) {
        int stop = 0;
        uint32_t n = 0;
        while (ld_acquire(w.flags + j) < (uint32_t)pass) {
          if (ld_acquire(abort_word) != 0u) { stop = 1; break; }
          if (++n > SPIN_LIMIT) {
            __hip_atomic_store(abort_word, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            stop = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        s_flag = stop;
      }
      __syncthreads();
      if (s_flag) break;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const PointParams P = load_params(w.params + j);
    double* out = w.partials + (int64_t)t * NSTAT;
    if (pass == 0) tile_body<DT, MODE_MOMENTS, WG, ITEMS>(sh, SrcCtx<DT>{pl}, td, P, red, out);
    else if (pass < sh.K) tile_body<DT, MODE_GN_NC, WG, ITEMS>(sh, SrcCtx<DT>{pl}, td, P, red, out);
    else tile_body<DT, MODE_GN, WG, ITEMS>(sh, SrcCtx<DT>{pl}, td, P, red, out);
    if (threadIdx.x == 0) {
      __threadfence();  // partials before the arrival
      const uint32_t old = atomicAdd(arrive + j, 1u);
      s_flag = (old + 1u == (uint32_t)w.sched[j].ntiles);
    }
    __syncthreads();
    if (s_flag) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (threadIdx.x < 64) {
        const PairSched sc = w.sched[j];
        double s[NSTAT];
        pair_sums(w, sc, NSTAT, s);
        if (threadIdx.x == 0) {
          if (pass == 0) finalize_moments(sh, cd, w, j, sc, s);
          else if (pass <= sh.K) finalize_gn(sh, cd, w, j, pass, s);
          else finalize_final_cost(cd, w, j, s);
          arrive[j] = 0u;
          __threadfence();
          __hip_atomic_store(w.flags + j, (uint32_t)(pass + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
  }
}

template <int DT>
static hipError_t launch_persistent_t(const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                                      int grid, hipStream_t st) {
#define S3A_CASE(WGV, IT)                                                                   \
  if (lc.wg == WGV && lc.items == IT) {                                                     \
    hipLaunchKernelGGL((k_persistent<DT, WGV, IT>), dim3(grid), dim3(WGV), 0, st, sh, cd, w); \
    return hipGetLastError();                                                               \
  }
  S3A_CASE(256, 2) S3A_CASE(256, 4) S3A_CASE(256, 8) S3A_CASE(256, 16)
  S3A_CASE(512, 2) S3A_CASE(512, 4) S3A_CASE(512, 8)
#undef S3A_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_init_outputs(const Shape& sh, const CallDesc* cd, hipStream_t st) {
  if (sh.n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_outputs, dim3((sh.n_pairs + 127) / 128), dim3(128), 0, st, sh, cd);
  return hipGetLastError();
}

hipError_t launch_persistent(int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* cd, const Work& w,
                             int grid, hipStream_t st) {
  return dtype == S3A_F32 ? launch_persistent_t<S3A_F32>(lc, sh, cd, w, grid, st)
                          : launch_persistent_t<S3A_BF16>(lc, sh, cd, w, grid, st);
}

}  // namespace s3a
