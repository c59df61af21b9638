// C ABI of the s3a library: handle, workspace, argument checks, launch
// sequences (plain per-pair and batched), graph capture, autotuning.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "align_launch.h"
#include "pgo.h"
#include "points.h"
#include "implicit.h"

using namespace s3a;

namespace {

struct GraphKey {
  int dtype, n_pairs, K, wg, items, occupancy, window, persistent;
  int64_t n_points;
  uint32_t flags;
  float tau;
  double delta;
  const void* ptrs[12];
  bool operator==(const GraphKey& o) const { return memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
  uint64_t used;
};

struct TuneEntry {
  int dtype;
  int size_class;
  LaunchCfg cfg;
};

}  // namespace

struct s3a_handle {
  int device = 0;
  int n_cu = 256;
  int last_hip = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t cap_tiles = 0;
  int cap_pairs = 0;
  Work w{};
  hipStream_t capture_stream = nullptr;
  std::vector<GraphEntry> graphs;
  uint64_t clock = 0;
  bool forced[2] = {false, false};
  LaunchCfg forced_cfg[2];
  std::vector<TuneEntry> tuned;
  PgoWorkspace* pgo = nullptr;
  CallDesc* desc = nullptr;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
  int32_t* flags_dev = nullptr;  // small device scratch (offset-check flag of the point transform)
  double* hpart = nullptr;       // per-run sums of the implicit-derivative pass
  int64_t hpart_tiles = 0;       // slots of 52 doubles
  // issue order of calls across streams (they share the workspace)
  hipEvent_t order_ev = nullptr;
  hipStream_t order_stream = nullptr;
  bool order_valid = false;
};

namespace {

int hip_fail(s3a_handle* h, hipError_t e) {
  if (h) h->last_hip = (int)e;
  return e == hipErrorOutOfMemory ? S3A_ENOMEM : S3A_EHIP;
}

#define S3A_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(h, e_); \
  } while (0)

// Event pair around one launch of a call's dominant kernel (timing mode).
struct TimedLaunch {
  s3a_handle* h;
  hipStream_t st;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  TimedLaunch(s3a_handle* hh, hipStream_t s) : h(hh), st(s) {
    if (!h || !h->timing) return;
    if (!h->ev_free.empty()) {
      ev = h->ev_free.back();
      h->ev_free.pop_back();
    } else {
      (void)hipEventCreate(&ev.first);
      (void)hipEventCreate(&ev.second);
    }
    (void)hipEventRecord(ev.first, st);
  }
  ~TimedLaunch() {
    if (!ev.first) return;
    (void)hipEventRecord(ev.second, st);
    h->ev_used.push_back(ev);
  }
};

// Calls through one handle share its workspace (descriptor slot, tile table,
// partials, per-pair state), so they must run in issue order. A call on a
// stream other than the previous call's first makes its stream wait, on the
// device, for everything the previous call enqueued; on leaving, it records
// where its own work ends. Calls on one stream are ordered by the stream.
struct StreamOrder {
  s3a_handle* h;
  hipStream_t st;
  hipError_t err = hipSuccess;
  StreamOrder(s3a_handle* hh, hipStream_t s) : h(hh), st(s) {
    if (h->order_valid && h->order_stream != st) err = hipStreamWaitEvent(st, h->order_ev, 0);
  }
  ~StreamOrder() {
    if (hipEventRecord(h->order_ev, st) == hipSuccess) {
      h->order_stream = st;
      h->order_valid = true;
    } else {
      // no marker for this call's end: drain it instead, so no later call can overtake it
      (void)hipStreamSynchronize(st);
      h->order_valid = false;
    }
  }
};

#define S3A_ORDERED(h, st)              \
  StreamOrder order_(h, st);            \
  if (order_.err != hipSuccess) return hip_fail(h, order_.err)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void clear_graphs(s3a_handle* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int ensure_workspace(s3a_handle* h, int n_pairs, int64_t tiles) {
  if (n_pairs <= h->cap_pairs && tiles <= h->cap_tiles && h->ws) return S3A_OK;
  const int np = std::max(n_pairs, std::max(h->cap_pairs, 64));
  const int64_t nt = std::max<int64_t>(tiles, std::max<int64_t>(h->cap_tiles, 1024));
  size_t off = 0;
  const size_t o_tiles = off; off = align_up(off + sizeof(TileDesc) * nt);
  const size_t o_part = off;  off = align_up(off + sizeof(double) * NSTAT * nt);
  const size_t o_sched = off; off = align_up(off + sizeof(PairSched) * np);
  const size_t o_par = off;   off = align_up(off + sizeof(PointParams) * np);
  const size_t o_state = off; off = align_up(off + sizeof(PairState) * np);
  const size_t o_cnt = off;   off = align_up(off + sizeof(uint32_t) * (np + 64));
  const size_t o_flag = off;  off = align_up(off + sizeof(uint32_t) * (np + 64));
  const size_t o_tot = off;   off = align_up(off + sizeof(int32_t) * 64);
  const size_t o_desc = off;  off = align_up(off + sizeof(CallDesc));
  const size_t o_dpair = off; off = align_up(off + sizeof(DepthPair) * np);
  clear_graphs(h);
  if (h->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(h->ws);
    h->ws = nullptr;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, off);
  if (e != hipSuccess) {
    h->cap_pairs = 0;
    h->cap_tiles = 0;
    return hip_fail(h, e);
  }
  h->ws = p;
  h->ws_bytes = off;
  char* b = static_cast<char*>(p);
  h->w.tiles = reinterpret_cast<TileDesc*>(b + o_tiles);
  h->w.partials = reinterpret_cast<double*>(b + o_part);
  h->w.sched = reinterpret_cast<PairSched*>(b + o_sched);
  h->w.params = reinterpret_cast<PointParams*>(b + o_par);
  h->w.state = reinterpret_cast<PairState*>(b + o_state);
  h->w.counters = reinterpret_cast<uint32_t*>(b + o_cnt);
  h->w.flags = reinterpret_cast<uint32_t*>(b + o_flag);
  h->w.total_tiles = reinterpret_cast<int32_t*>(b + o_tot);
  h->w.scan_tmp = nullptr;
  h->desc = reinterpret_cast<CallDesc*>(b + o_desc);
  h->w.dpairs = reinterpret_cast<DepthPair*>(b + o_dpair);
  h->cap_pairs = np;
  h->cap_tiles = nt;
  return S3A_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_desc(const s3a_align_desc* d) {
  if (!d) return S3A_EINVAL;
  if (d->dtype != S3A_F32 && d->dtype != S3A_BF16) return S3A_EINVAL;
  if (d->n_pairs < 0 || d->n_points < 0 || d->n_pairs > (1 << 24)) return S3A_EINVAL;
  if (d->n_pairs > 0 && !d->offsets) return S3A_EINVAL;
  const void* pl[7] = {d->px, d->py, d->pz, d->qx, d->qy, d->qz, d->conf};
  for (const void* p : pl)
    if (d->n_points > 0 && (!p || !aligned16(p))) return S3A_EINVAL;
  if (!(d->conf_threshold >= 0.0f)) return S3A_EINVAL;  // rejects NaN
  if (d->irls_iters < 0 || d->irls_iters > 10000) return S3A_EINVAL;
  if (!(d->huber_delta > 0.0)) return S3A_EINVAL;
  if (d->flags & ~(S3A_FLAG_PLAIN | S3A_FLAG_FINAL_COST | S3A_FLAG_NO_GRAPH | S3A_FLAG_PERSISTENT))
    return S3A_EINVAL;
  if (d->reserved != 0) return S3A_EINVAL;
  return S3A_OK;
}

int size_class(int64_t n_points) {
  int c = 0;
  while (n_points > 65536 && c < 12) {
    n_points >>= 2;
    ++c;
  }
  return c;
}

// Untuned shapes. Depth-map input does about seven times the arithmetic per
// byte of stored points and runs best with one workgroup per (longer) tile.
LaunchCfg default_cfg(int dtype) {
  LaunchCfg c;
  c.wg = 256;
  if (dtype == DT_DEPTH_F32 || dtype == DT_DEPTH_BF16) {
    c.items = 16;
    c.occupancy = 0;
  } else {
    c.items = (dtype & 1) ? 2 : 4;
    c.occupancy = 4;
  }
  c.window = 0;
  return c;
}

// A forced shape applies to plane and depth-map input of its plane type; tuned
// shapes are kept per input kind (plane or depth map, FP32 or BF16) and size
// class.
LaunchCfg pick_cfg(s3a_handle* h, int dtype, int64_t n_points) {
  if (h->forced[dtype & 1]) return h->forced_cfg[dtype & 1];
  const int sc = size_class(n_points);
  for (auto& t : h->tuned)
    if (t.dtype == dtype && t.size_class == sc) return t.cfg;
  return default_cfg(dtype);
}

bool valid_cfg(const LaunchCfg& c) {
  return (c.wg == 256 || c.wg == 512) && (c.items == 2 || c.items == 4 || c.items == 8 || (c.items == 16 && c.wg == 256)) &&
         c.occupancy >= 0 &&
         c.occupancy <= 8 && c.window >= 0;
}

Shape make_shape(const s3a_align_desc* d, const LaunchCfg& lc) {
  Shape sh;
  sh.n_points = d->n_points;
  sh.n_pairs = d->n_pairs;
  sh.K = d->irls_iters;
  sh.tau = d->conf_threshold;
  sh.delta = d->huber_delta;
  sh.delta_f = (float)d->huber_delta;
  sh.flags = d->flags;
  sh.tile_elems = (int32_t)tile_elems(d->dtype, lc);
  return sh;
}

CallDesc make_call(const s3a_align_desc* d) {
  CallDesc c;
  memset(&c, 0, sizeof(c));
  c.planes[0] = d->px; c.planes[1] = d->py; c.planes[2] = d->pz;
  c.planes[3] = d->qx; c.planes[4] = d->qy; c.planes[5] = d->qz;
  c.planes[6] = d->conf;
  c.offsets = d->offsets;
  return c;
}

// The CallDesc travels to the device inside the workspace: copied on the
// stream just before the kernels that read it.
CallDesc* desc_slot(s3a_handle* h) { return h->desc; }

// Occupancy 0: one workgroup per tile (the hardware balances the tail);
// otherwise a fixed number of workgroups per compute unit loops over the tiles.
int grid_for(s3a_handle* h, const LaunchCfg& lc, int64_t tiles) {
  const int64_t g = lc.occupancy == 0 ? tiles
                                      : std::min<int64_t>(tiles, (int64_t)lc.occupancy * h->n_cu * (256 / std::min(lc.wg, 256)));
  return (int)std::max<int64_t>(g, 1);
}

// Multi-launch batched sequence: schedule, then per pass one streaming launch
// over every tile of every pair and one finalize launch.
hipError_t enqueue_batched_multi(s3a_handle* h, int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* dcd,
                                 hipStream_t st) {
  hipError_t e = launch_sched(sh, dcd, h->w, st);
  if (e != hipSuccess) return e;
  if (dtype == DT_DEPTH_F32 || dtype == DT_DEPTH_BF16) {
    e = launch_depth_prep(sh, dcd, h->w, st);
    if (e != hipSuccess) return e;
  }
  const int64_t mt = max_tiles(sh.n_points, sh.n_pairs, sh.tile_elems);
  const int grid = grid_for(h, lc, mt);
  const int npass = 1 + sh.K + ((sh.flags & S3A_FLAG_FINAL_COST) ? 1 : 0);
  for (int pass = 0; pass < npass; ++pass) {
    const int mode = pass_mode(pass, sh.K);
    {
      TimedLaunch tl(h, st);
      e = launch_pass(dtype, mode, lc, sh, dcd, h->w, 0, -1, grid, st);
    }
    if (e != hipSuccess) return e;
    const int kind = pass == 0 ? 0 : (pass <= sh.K ? 1 : 2);
    e = launch_finalize(kind, sh, dcd, h->w, pass, 0, sh.n_pairs, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_batched(s3a_handle* h, int dtype, const LaunchCfg& lc, const Shape& sh, const CallDesc* dcd,
                           bool persistent, hipStream_t st) {
  if (!persistent) return enqueue_batched_multi(h, dtype, lc, sh, dcd, st);
  hipError_t e = launch_sched(sh, dcd, h->w, st);
  if (e != hipSuccess) return e;
  e = launch_fill_zero(h->w.counters, (int64_t)sh.n_pairs + 64, st);
  if (e != hipSuccess) return e;
  e = launch_fill_zero(h->w.flags, (int64_t)sh.n_pairs, st);
  if (e != hipSuccess) return e;
  e = launch_init_outputs(sh, dcd, st);
  if (e != hipSuccess) return e;
  const int grid = (lc.occupancy > 0 ? lc.occupancy : 4) * h->n_cu;
  TimedLaunch tl(h, st);
  return launch_persistent(dtype, lc, sh, dcd, h->w, grid, st);
}

}  // namespace

extern "C" {

int s3a_version(void) { return 100; }

const char* s3a_strerror(int code) {
  switch (code) {
    case S3A_OK: return "ok";
    case S3A_EINVAL: return "invalid argument";
    case S3A_EHIP: return "HIP runtime error";
    case S3A_ENOMEM: return "out of device memory";
    case S3A_ELIMIT: return "batch exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown error";
  }
}

int s3a_last_hip_error(const s3a_handle* h) { return h ? h->last_hip : 0; }

int s3a_create(s3a_handle** out, int device) {
  if (!out) return S3A_EINVAL;
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return S3A_EHIP;
  if (device < 0 || device >= n) return S3A_EINVAL;
  s3a_handle* h = new s3a_handle();
  h->device = device;
  DeviceGuard g(device);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete h;
    return S3A_EHIP;
  }
  h->n_cu = prop.multiProcessorCount;
  e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete h;
    return S3A_EHIP;
  }
  e = hipEventCreateWithFlags(&h->order_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(h->capture_stream);
    delete h;
    return S3A_EHIP;
  }
  *out = h;
  return S3A_OK;
}

int s3a_destroy(s3a_handle* h) {
  if (!h) return S3A_EINVAL;
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  clear_graphs(h);
  if (h->ws) (void)hipFree(h->ws);
  if (h->flags_dev) (void)hipFree(h->flags_dev);
  if (h->hpart) (void)hipFree(h->hpart);
  pgo_free(h->pgo);
  for (auto& ev : h->ev_used) { (void)hipEventDestroy(ev.first); (void)hipEventDestroy(ev.second); }
  for (auto& ev : h->ev_free) { (void)hipEventDestroy(ev.first); (void)hipEventDestroy(ev.second); }
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  if (h->order_ev) (void)hipEventDestroy(h->order_ev);
  delete h;
  return S3A_OK;
}

}  // extern "C"

namespace {

// The alignment driver of s3a_align_pairs and s3a_align_depth_pairs: d holds
// a checked descriptor whose dtype may be an internal depth type (planes px,
// py, pz = d_p, d_q, c), with the caller's cameras in depth.
int align_run(s3a_handle* h, const s3a_align_desc* d, const s3a_depth_pair* depth, const s3a_sim3* init,
              s3a_sim3* S_out, s3a_align_info* info, s3a_stream stream) {
  int rc = S3A_OK;
  DeviceGuard g(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  S3A_ORDERED(h, st);
  const LaunchCfg lc = pick_cfg(h, d->dtype, d->n_points);
  const Shape sh = make_shape(d, lc);
  const int64_t mt = max_tiles(sh.n_points, sh.n_pairs, sh.tile_elems);
  if (mt >= (1ll << 31)) return S3A_EINVAL;
  rc = ensure_workspace(h, d->n_pairs, mt);
  if (rc) return rc;
  CallDesc c = make_call(d);
  c.init = init;
  c.S_out = S_out;
  c.info = info;
  c.depth = depth;
  CallDesc* dcd = desc_slot(h);

  if (d->flags & S3A_FLAG_PLAIN) {
    // one pair at a time: read the schedule back, then 1 + K (+1) passes per pair
    S3A_TRY(hipMemcpyAsync(dcd, &c, sizeof(c), hipMemcpyHostToDevice, st));
    S3A_TRY(launch_sched(sh, dcd, h->w, st));
    if (depth) S3A_TRY(launch_depth_prep(sh, dcd, h->w, st));
    std::vector<PairSched> sched(d->n_pairs);
    S3A_TRY(hipMemcpyAsync(sched.data(), h->w.sched, sizeof(PairSched) * d->n_pairs, hipMemcpyDeviceToHost, st));
    S3A_TRY(hipStreamSynchronize(st));
    const int npass = 1 + sh.K + ((sh.flags & S3A_FLAG_FINAL_COST) ? 1 : 0);
    for (int k = 0; k < d->n_pairs; ++k) {
      const PairSched& s = sched[k];
      for (int pass = 0; pass < npass; ++pass) {
        const int mode = pass_mode(pass, sh.K);
        {
          TimedLaunch tl(h, st);
          S3A_TRY(launch_pass(d->dtype, mode, lc, sh, dcd, h->w, s.tile0, s.tile0 + s.ntiles, s.ntiles, st));
        }
        const int kind = pass == 0 ? 0 : (pass <= sh.K ? 1 : 2);
        S3A_TRY(launch_finalize(kind, sh, dcd, h->w, pass, k, 1, st));
      }
    }
    return S3A_OK;
  }

  const bool persistent = (d->flags & S3A_FLAG_PERSISTENT) != 0;
  if ((d->flags & S3A_FLAG_NO_GRAPH) || h->timing) {
    S3A_TRY(hipMemcpyAsync(dcd, &c, sizeof(c), hipMemcpyHostToDevice, st));
    S3A_TRY(enqueue_batched(h, d->dtype, lc, sh, dcd, persistent, st));
    return S3A_OK;
  }

  // graph path: the descriptor copy stays outside the graph; the graph is keyed
  // on the shape and launch configuration (pointers reach the kernels through
  // the descriptor, so a graph serves every call of that shape)
  GraphKey key;
  memset(&key, 0, sizeof(key));
  key.dtype = d->dtype;
  key.n_pairs = d->n_pairs;
  key.K = sh.K;
  key.wg = lc.wg;
  key.items = lc.items;
  key.occupancy = lc.occupancy;
  key.window = lc.window;
  key.persistent = persistent;
  key.n_points = d->n_points;
  key.flags = d->flags;
  key.tau = d->conf_threshold;
  key.delta = d->huber_delta;
  key.ptrs[0] = h->ws;
  hipGraphExec_t exec = nullptr;
  for (auto& ge : h->graphs)
    if (ge.key == key) {
      exec = ge.exec;
      ge.used = ++h->clock;
    }
  if (!exec) {
    hipGraph_t graph = nullptr;
    S3A_TRY(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_batched(h, d->dtype, lc, sh, dcd, persistent, h->capture_stream);
    hipError_t e2 = hipStreamEndCapture(h->capture_stream, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(h, e);
    }
    if (e2 != hipSuccess) return hip_fail(h, e2);
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(h, e);
    if (h->graphs.size() >= 16) {
      auto it = std::min_element(h->graphs.begin(), h->graphs.end(),
                                 [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
      (void)hipGraphExecDestroy(it->exec);
      h->graphs.erase(it);
    }
    h->graphs.push_back(GraphEntry{key, exec, ++h->clock});
  }
  S3A_TRY(hipMemcpyAsync(dcd, &c, sizeof(c), hipMemcpyHostToDevice, st));
  S3A_TRY(hipGraphLaunch(exec, st));
  return S3A_OK;
}

}  // namespace

// ------------------------------------------------------------------ allocation-free alignment
//
// s3a_align_pairs_noalloc runs the batched sequence (schedule, then per pass
// one streaming launch and one finalize launch) with every temporary in one
// fixed device array per device, laid out below. Its launch shape is fixed,
// so no autotuning state is needed either.

namespace {

constexpr size_t align_c(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int NA_PAIRS = S3A_NOALLOC_MAX_PAIRS;
constexpr int64_t NA_TILES = S3A_NOALLOC_MAX_TILES;
constexpr size_t NA_O_DESC = 0;
constexpr size_t NA_O_TOTAL = align_c(NA_O_DESC + sizeof(CallDesc));
constexpr size_t NA_O_SCHED = align_c(NA_O_TOTAL + sizeof(int32_t) * 64);
constexpr size_t NA_O_PARAMS = align_c(NA_O_SCHED + sizeof(PairSched) * NA_PAIRS);
constexpr size_t NA_O_STATE = align_c(NA_O_PARAMS + sizeof(PointParams) * NA_PAIRS);
constexpr size_t NA_O_TILES = align_c(NA_O_STATE + sizeof(PairState) * NA_PAIRS);
constexpr size_t NA_O_PART = align_c(NA_O_TILES + sizeof(TileDesc) * NA_TILES);
constexpr size_t NA_BYTES = align_c(NA_O_PART + sizeof(double) * NSTAT * NA_TILES);
static_assert(NA_BYTES <= S3A_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds its stated size");

}  // namespace

// The scratch array: one copy per device, held until the process ends. Host
// code never names it in a launch or copy; it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[S3A_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
unsigned char* na_ptr[NA_MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up once per device).
int noalloc_scratch(unsigned char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return S3A_EHIP;
  if (dev >= NA_MAX_DEVICES) return S3A_EINVAL;
  std::lock_guard<std::mutex> lock(na_mutex);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return S3A_EHIP;
    na_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = na_ptr[dev];
  return S3A_OK;
}

// The call's descriptor reaches the device as a kernel argument (no host copy).
__global__ void k_store_desc(CallDesc c, CallDesc* dst) {
  if (threadIdx.x == 0) *dst = c;
}

// Fixed launch shapes: 8192-element tiles, one workgroup per tile.
LaunchCfg noalloc_cfg(int dtype) {
  LaunchCfg c;
  c.wg = dtype == S3A_F32 ? 512 : 256;
  c.items = 4;
  c.occupancy = 0;
  c.window = 0;
  return c;
}

}  // namespace

extern "C" {

int s3a_align_pairs_noalloc(const s3a_align_desc* d, const s3a_sim3* init, s3a_sim3* S_out,
                            s3a_align_info* info, s3a_stream stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->flags & (S3A_FLAG_PLAIN | S3A_FLAG_PERSISTENT)) return S3A_EINVAL;
  if (d->n_pairs > 0 && !S_out) return S3A_EINVAL;
  if (d->n_pairs == 0) return S3A_OK;
  const LaunchCfg lc = noalloc_cfg(d->dtype);
  const Shape sh = make_shape(d, lc);
  const int64_t mt = max_tiles(sh.n_points, sh.n_pairs, sh.tile_elems);
  if (d->n_pairs > NA_PAIRS || mt > NA_TILES) return S3A_ELIMIT;
  unsigned char* base = nullptr;
  rc = noalloc_scratch(&base);
  if (rc) return rc;
  Work w{};
  w.tiles = reinterpret_cast<TileDesc*>(base + NA_O_TILES);
  w.partials = reinterpret_cast<double*>(base + NA_O_PART);
  w.sched = reinterpret_cast<PairSched*>(base + NA_O_SCHED);
  w.params = reinterpret_cast<PointParams*>(base + NA_O_PARAMS);
  w.state = reinterpret_cast<PairState*>(base + NA_O_STATE);
  w.total_tiles = reinterpret_cast<int32_t*>(base + NA_O_TOTAL);
  w.counters = nullptr;  // persistent launch only
  w.flags = nullptr;
  w.scan_tmp = nullptr;
  w.dpairs = nullptr;    // depth input only
  CallDesc c = make_call(d);
  c.init = init;
  c.S_out = S_out;
  c.info = info;
  CallDesc* dcd = reinterpret_cast<CallDesc*>(base + NA_O_DESC);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_store_desc, dim3(1), dim3(64), 0, st, c, dcd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(nullptr, e);
  // every scratch word a kernel reads is written earlier in the same call:
  // the schedule and tile table by k_sched/k_sched_fill, each tile's partials
  // by its pass, each pair's state and parameters by the moments finalize
  e = launch_sched(sh, dcd, w, st);
  if (e != hipSuccess) return hip_fail(nullptr, e);
  const int grid = (int)std::max<int64_t>(mt, 1);
  const int npass = 1 + sh.K + ((sh.flags & S3A_FLAG_FINAL_COST) ? 1 : 0);
  for (int pass = 0; pass < npass; ++pass) {
    e = launch_pass(d->dtype, pass_mode(pass, sh.K), lc, sh, dcd, w, 0, -1, grid, st);
    if (e != hipSuccess) return hip_fail(nullptr, e);
    e = launch_finalize(pass == 0 ? 0 : (pass <= sh.K ? 1 : 2), sh, dcd, w, pass, 0, sh.n_pairs, st);
    if (e != hipSuccess) return hip_fail(nullptr, e);
  }
  return S3A_OK;
}

}  // extern "C"

extern "C" {

int s3a_align_pairs(s3a_handle* h, const s3a_align_desc* d, const s3a_sim3* init, s3a_sim3* S_out,
                    s3a_align_info* info, s3a_stream stream) {
  if (!h) return S3A_EINVAL;
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->n_pairs > 0 && !S_out) return S3A_EINVAL;
  if (d->n_pairs == 0) return S3A_OK;
  return align_run(h, d, nullptr, init, S_out, info, stream);
}

}  // extern "C"

// The internal descriptor of a depth-map call (the three planes stand in for
// the seven, which the descriptor check wants non-null), after checking it.
static int depth_call_desc(const s3a_depth_desc* dd, s3a_align_desc* d) {
  if (dd->dtype != S3A_F32 && dd->dtype != S3A_BF16) return S3A_EINVAL;
  if (dd->flags & S3A_FLAG_PERSISTENT) return S3A_EINVAL;
  if (dd->n_pairs > 0 && !dd->pairs) return S3A_EINVAL;
  memset(d, 0, sizeof(*d));
  d->dtype = dd->dtype == S3A_F32 ? DT_DEPTH_F32 : DT_DEPTH_BF16;
  d->n_pairs = dd->n_pairs;
  d->n_points = dd->n_points;
  d->offsets = dd->offsets;
  d->px = dd->depth_p; d->py = dd->depth_q; d->pz = dd->conf;
  d->qx = dd->depth_p; d->qy = dd->depth_q; d->qz = dd->conf; d->conf = dd->conf;
  d->conf_threshold = dd->conf_threshold;
  d->irls_iters = dd->irls_iters;
  d->huber_delta = dd->huber_delta;
  d->flags = dd->flags;
  d->reserved = dd->reserved;
  s3a_align_desc chk = *d;
  chk.dtype = dd->dtype;
  return check_desc(&chk);
}

extern "C" {

int s3a_align_depth_pairs(s3a_handle* h, const s3a_depth_desc* dd, const s3a_sim3* init, s3a_sim3* S_out,
                          s3a_align_info* info, s3a_stream stream) {
  if (!h || !dd) return S3A_EINVAL;
  if (dd->n_pairs > 0 && !S_out) return S3A_EINVAL;
  s3a_align_desc d;
  const int rc = depth_call_desc(dd, &d);
  if (rc) return rc;
  if (d.n_pairs == 0) return S3A_OK;
  return align_run(h, &d, dd->pairs, init, S_out, info, stream);
}

int s3a_align_cost(s3a_handle* h, const s3a_align_desc* d, const s3a_sim3* S, const double* xi, double* L_out,
                   double* C_out, s3a_stream stream) {
  if (!h) return S3A_EINVAL;
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->n_pairs > 0 && (!S || !L_out || !C_out)) return S3A_EINVAL;
  if (d->n_pairs == 0) return S3A_OK;
  DeviceGuard g(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  S3A_ORDERED(h, st);
  const LaunchCfg lc = pick_cfg(h, d->dtype, d->n_points);
  const Shape sh = make_shape(d, lc);
  const int64_t mt = max_tiles(sh.n_points, sh.n_pairs, sh.tile_elems);
  if (mt >= (1ll << 31)) return S3A_EINVAL;
  rc = ensure_workspace(h, d->n_pairs, mt);
  if (rc) return rc;
  CallDesc c = make_call(d);
  c.S_in = S;
  c.xi = xi;
  c.L_out = L_out;
  c.C_out = C_out;
  CallDesc* dcd = desc_slot(h);
  S3A_TRY(hipMemcpyAsync(dcd, &c, sizeof(c), hipMemcpyHostToDevice, st));
  S3A_TRY(launch_sched(sh, dcd, h->w, st));
  S3A_TRY(launch_prep(sh, dcd, h->w, 0, st));
  {
    TimedLaunch tl(h, st);
    S3A_TRY(launch_pass(d->dtype, MODE_COST, lc, sh, dcd, h->w, 0, -1, grid_for(h, lc, mt), st));
  }
  S3A_TRY(launch_finalize_cost(sh, dcd, h->w, st));
  return S3A_OK;
}

int s3a_align_pairs_backward(s3a_handle* h, const s3a_align_desc* d, const s3a_sim3* S, const double* xi,
                             const double* L, const double* C, const double* gL, float* gpx, float* gpy, float* gpz,
                             float* gqx, float* gqy, float* gqz, float* gc, double* gxi, s3a_stream stream) {
  if (!h) return S3A_EINVAL;
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->n_pairs > 0 && (!S || !L || !C || !gL)) return S3A_EINVAL;
  float* gr[7] = {gpx, gpy, gpz, gqx, gqy, gqz, gc};
  for (float* p : gr)
    if (p && !aligned16(p)) return S3A_EINVAL;
  if (d->n_pairs == 0) return S3A_OK;
  DeviceGuard g(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  S3A_ORDERED(h, st);
  const LaunchCfg lc = pick_cfg(h, d->dtype, d->n_points);
  const Shape sh = make_shape(d, lc);
  const int64_t mt = max_tiles(sh.n_points, sh.n_pairs, sh.tile_elems);
  if (mt >= (1ll << 31)) return S3A_EINVAL;
  rc = ensure_workspace(h, d->n_pairs, mt);
  if (rc) return rc;
  CallDesc c = make_call(d);
  c.S_in = S;
  c.xi = xi;
  c.L_in = L;
  c.C_in = C;
  c.gL = gL;
  for (int j = 0; j < 7; ++j) c.grad[j] = gr[j];
  c.gxi = gxi;
  CallDesc* dcd = desc_slot(h);
  S3A_TRY(hipMemcpyAsync(dcd, &c, sizeof(c), hipMemcpyHostToDevice, st));
  S3A_TRY(launch_sched(sh, dcd, h->w, st));
  S3A_TRY(launch_prep(sh, dcd, h->w, 1, st));
  {
    TimedLaunch tl(h, st);
    S3A_TRY(launch_adjoint(d->dtype, lc, sh, dcd, h->w, grid_for(h, lc, mt), st));
  }
  S3A_TRY(launch_finalize_adjoint(sh, dcd, h->w, st));
  return S3A_OK;
}

int s3a_align_pairs_implicit_backward(s3a_handle* h, const s3a_align_desc* d, const s3a_sim3* S, const double* gS,
                                      uint32_t iflags, float* gpx, float* gpy, float* gpz, float* gqx, float* gqy,
                                      float* gqz, float* gc, double* v_out, int32_t* status_out, s3a_stream stream) {
  if (!h) return S3A_EINVAL;
  int rc = check_desc(d);
  if (rc) return rc;
  if (iflags & ~S3A_IMPLICIT_TANGENT) return S3A_EINVAL;
  if (d->n_pairs > 0 && (!S || !gS)) return S3A_EINVAL;
  float* gr[7] = {gpx, gpy, gpz, gqx, gqy, gqz, gc};
  for (float* p : gr)
    if (p && !aligned16(p)) return S3A_EINVAL;
  if (d->n_pairs == 0) return S3A_OK;
  DeviceGuard g(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  S3A_ORDERED(h, st);
  const LaunchCfg lc = pick_cfg(h, d->dtype, d->n_points);
  const Shape sh = make_shape(d, lc);
  const int64_t mt = max_tiles(sh.n_points, sh.n_pairs, sh.tile_elems);
  if (mt >= (1ll << 31)) return S3A_EINVAL;
  rc = ensure_workspace(h, d->n_pairs, mt);
  if (rc) return rc;
  const int64_t hslots = mt + d->n_pairs;  // the Hessian pass's slots: at most one per workgroup and pair run
  if (h->hpart_tiles < hslots) {
    if (h->hpart) {
      S3A_TRY(hipStreamSynchronize(st));
      (void)hipFree(h->hpart);
      h->hpart = nullptr;
      h->hpart_tiles = 0;
    }
    S3A_TRY(hipMalloc(&h->hpart, sizeof(double) * 52 * (size_t)hslots));
    h->hpart_tiles = hslots;
  }
  CallDesc c = make_call(d);
  c.S_in = S;
  c.xi = nullptr;
  for (int j = 0; j < 7; ++j) c.grad[j] = gr[j];
  CallDesc* dcd = desc_slot(h);
  S3A_TRY(hipMemcpyAsync(dcd, &c, sizeof(c), hipMemcpyHostToDevice, st));
  S3A_TRY(launch_sched(sh, dcd, h->w, st));
  S3A_TRY(launch_prep(sh, dcd, h->w, 0, st));
  TimedLaunch tl(h, st);
  S3A_TRY(launch_implicit(d->dtype, lc, sh, dcd, h->w, h->hpart, gS, iflags, v_out, status_out, grid_for(h, lc, mt), mt,
                          h->n_cu, st));
  return S3A_OK;
}

int s3a_set_timing(s3a_handle* h, int on) {
  if (!h) return S3A_EINVAL;
  h->timing = on != 0;
  return S3A_OK;
}

int s3a_kernel_time(s3a_handle* h, double* ms, int32_t* launches) {
  if (!h || !ms || !launches) return S3A_EINVAL;
  DeviceGuard g(h->device);
  double total = 0.0;
  int rc = S3A_OK;
  for (auto& ev : h->ev_used) {
    hipError_t e = hipEventSynchronize(ev.second);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev.first, ev.second);
    if (e != hipSuccess) rc = hip_fail(h, e);
    total += t;
  }
  *launches = (int32_t)h->ev_used.size();
  *ms = total;
  h->ev_free.insert(h->ev_free.end(), h->ev_used.begin(), h->ev_used.end());
  h->ev_used.clear();
  return rc;
}

int s3a_set_tuning(s3a_handle* h, int32_t dtype, const s3a_tuning* t) {
  if (!h || (dtype != S3A_F32 && dtype != S3A_BF16)) return S3A_EINVAL;
  if (!t) {
    h->forced[dtype] = false;
    return S3A_OK;
  }
  LaunchCfg c;
  c.wg = t->wg;
  c.items = t->items;
  c.occupancy = t->occupancy;
  c.window = t->window;
  if (!valid_cfg(c)) return S3A_EINVAL;
  h->forced[dtype] = true;
  h->forced_cfg[dtype] = c;
  return S3A_OK;
}

int s3a_get_tuning(s3a_handle* h, int32_t dtype, int64_t n_points, s3a_tuning* t) {
  if (!h || !t || (dtype != S3A_F32 && dtype != S3A_BF16)) return S3A_EINVAL;
  const LaunchCfg c = pick_cfg(h, dtype, n_points);
  t->wg = c.wg;
  t->items = c.items;
  t->occupancy = c.occupancy;
  t->window = c.window;
  return S3A_OK;
}

}  // extern "C"

// Time the candidate launch shapes on one call (plane or depth-map input; the
// caller's descriptor is already checked) and keep the fastest for its (input
// kind, size class).
static int autotune_run(s3a_handle* h, const s3a_align_desc* d, const s3a_depth_pair* depth, s3a_tuning* best,
                        s3a_stream stream) {
  if (d->n_pairs == 0) return S3A_OK;
  DeviceGuard g(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  S3A_ORDERED(h, st);
  // scratch outputs
  s3a_sim3* S = nullptr;
  S3A_TRY(hipMalloc(&S, sizeof(s3a_sim3) * d->n_pairs));
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int plane = d->dtype & 1;  // the forced shape is per plane type
  const bool was_forced = h->forced[plane];
  const LaunchCfg was_cfg = h->forced_cfg[plane];
  LaunchCfg bestc = default_cfg(d->dtype);
  float best_ms = 1e30f;
  const int wgs[2] = {256, 512};
  const int its[4] = {2, 4, 8, 16};
  const int occs[4] = {0, 2, 4, 8};
  const bool persistent = (d->flags & S3A_FLAG_PERSISTENT) && !(d->flags & S3A_FLAG_PLAIN);
  s3a_align_desc dd = *d;
  dd.flags &= ~S3A_FLAG_PLAIN;
  for (int wg : wgs)
    for (int it : its)
      for (int oc : occs) {
        if (wg == 512 && (oc > 4 || it > 8)) continue;
        if (persistent ? oc == 0 : (oc != 0 && oc != 4)) continue;
        LaunchCfg c;
        c.wg = wg;
        c.items = it;
        c.occupancy = oc;
        c.window = 0;
        h->forced[plane] = true;
        h->forced_cfg[plane] = c;
        float ms = 1e30f;
        bool ok = true;
        for (int rep = 0; rep < 4 && ok; ++rep) {
          if (align_run(h, &dd, depth, nullptr, S, nullptr, stream) != S3A_OK) ok = false;
          if (rep == 0) {  // warm-up (and graph capture)
            if (hipStreamSynchronize(st) != hipSuccess) ok = false;
            continue;
          }
          (void)hipEventRecord(e0, st);
          if (align_run(h, &dd, depth, nullptr, S, nullptr, stream) != S3A_OK) ok = false;
          (void)hipEventRecord(e1, st);
          if (hipEventSynchronize(e1) != hipSuccess) ok = false;
          float t = 0.0f;
          (void)hipEventElapsedTime(&t, e0, e1);
          ms = std::min(ms, t);
        }
        if (ok && ms < best_ms) {
          best_ms = ms;
          bestc = c;
        }
      }
  h->forced[plane] = was_forced;
  h->forced_cfg[plane] = was_cfg;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(S);
  const int sc = size_class(d->n_points);
  bool found = false;
  for (auto& t : h->tuned)
    if (t.dtype == d->dtype && t.size_class == sc) {
      t.cfg = bestc;
      found = true;
    }
  if (!found) h->tuned.push_back(TuneEntry{d->dtype, sc, bestc});
  if (best) {
    best->wg = bestc.wg;
    best->items = bestc.items;
    best->occupancy = bestc.occupancy;
    best->window = bestc.window;
  }
  return S3A_OK;
}

extern "C" {

int s3a_autotune(s3a_handle* h, const s3a_align_desc* d, s3a_tuning* best, s3a_stream stream) {
  if (!h) return S3A_EINVAL;
  const int rc = check_desc(d);
  if (rc) return rc;
  return autotune_run(h, d, nullptr, best, stream);
}

int s3a_autotune_depth(s3a_handle* h, const s3a_depth_desc* dd, s3a_tuning* best, s3a_stream stream) {
  if (!h || !dd) return S3A_EINVAL;
  s3a_align_desc d;
  const int rc = depth_call_desc(dd, &d);
  if (rc) return rc;
  return autotune_run(h, &d, dd->pairs, best, stream);
}

int s3a_transform_points(s3a_handle* h, int32_t dtype, int64_t n_points, int32_t n_submaps, const int64_t* offsets,
                         const s3a_sim3* T, const void* x, const void* y, const void* z, float* out_x, float* out_y,
                         float* out_z, int32_t* status, s3a_stream stream) {
  if (!h || (dtype != S3A_F32 && dtype != S3A_BF16) || n_points < 0 || n_submaps < 0 || !offsets) return S3A_EINVAL;
  if (n_submaps > 0 && !T) return S3A_EINVAL;
  if (n_points > 0 && (!x || !y || !z || !out_x || !out_y || !out_z)) return S3A_EINVAL;
  const void* planes[6] = {x, y, z, out_x, out_y, out_z};
  for (const void* q : planes)
    if (((uintptr_t)q & 15) != 0) return S3A_EINVAL;
  DeviceGuard g(h->device);
  hipStream_t st = (hipStream_t)stream;
  S3A_ORDERED(h, st);
  if (!h->flags_dev) S3A_TRY(hipMalloc(&h->flags_dev, 256));
  S3A_TRY(launch_check_offsets(n_points, n_submaps, offsets, h->flags_dev, status, st));
  TimedLaunch tl(h, st);
  S3A_TRY(launch_transform(dtype, n_points, n_submaps, offsets, T, x, y, z, out_x, out_y, out_z, h->flags_dev, st));
  return S3A_OK;
}

int s3a_correct_points(s3a_handle* h, int64_t n_corr, const int64_t* src, const int64_t* dst, int64_t n_world,
                       const float* wx, const float* wy, const float* wz, int64_t n_sparse, float* sx, float* sy,
                       float* sz, unsigned long long* n_skipped, s3a_stream stream) {
  if (!h || n_corr < 0 || n_world < 0 || n_sparse < 0) return S3A_EINVAL;
  if (n_corr > 0 && (!src || !dst)) return S3A_EINVAL;
  if (n_world > 0 && (!wx || !wy || !wz)) return S3A_EINVAL;
  if (n_sparse > 0 && (!sx || !sy || !sz)) return S3A_EINVAL;
  DeviceGuard g(h->device);
  hipStream_t st = (hipStream_t)stream;
  S3A_ORDERED(h, st);
  TimedLaunch tl(h, st);
  S3A_TRY(launch_correct(n_corr, src, dst, n_world, wx, wy, wz, n_sparse, sx, sy, sz, n_skipped, st));
  return S3A_OK;
}

int s3a_edges_from_alignment(s3a_handle* h, int32_t n_edges, const s3a_sim3* S, const s3a_align_info* info,
                             double info_scale, s3a_sim3* T_meas, double* omega, int32_t* edge_status,
                             s3a_stream stream) {
  if (!h || n_edges < 0) return S3A_EINVAL;
  if (!(info_scale > 0.0) || !(info_scale < __builtin_inf())) return S3A_EINVAL;
  if (n_edges > 0 && (!S || !info || !T_meas || !omega)) return S3A_EINVAL;
  if (n_edges == 0) return S3A_OK;
  DeviceGuard g(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  S3A_ORDERED(h, st);
  S3A_TRY(launch_edges_from_alignment(n_edges, S, info, info_scale, T_meas, omega, edge_status, st));
  return S3A_OK;
}

int s3a_pose_graph_solve(s3a_handle* h, int32_t n_nodes, int32_t n_edges, const int32_t* ij, const s3a_sim3* T_meas,
                         const double* omega, s3a_sim3* T, const s3a_pgo_params* params, s3a_pgo_report* report,
                         s3a_stream stream) {
  if (!h) return S3A_EINVAL;
  DeviceGuard g(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  S3A_ORDERED(h, st);
  return pgo_solve(&h->pgo, &h->last_hip, n_nodes, n_edges, ij, T_meas, omega, T, params, report, st);
}

}  // extern "C"
