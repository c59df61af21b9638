// Internal device-side data structures of the s3a library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "s3a.h"
#include "dmath.h"

namespace s3a {

// Statistics reduced per tile and per pair. Every point pass reduces NSTAT
// values: the alignment passes the 17 sufficient statistics of the Umeyama or
// Gauss-Newton system plus two counters, the cost pass 3, the adjoint pass 7.
constexpr int NSTAT = 19;

// Moments pass (closed-form start), weights w = m c:
//   0 W, 1-3 sum w p, 4-6 sum w q, 7 sum w |p|^2, 8-16 sum w q_a p_b,
//   17 valid count V, 18 non-finite count.
// Gauss-Newton pass at S, centre c, y_c = S p - c, r = S p - q, om = w psi:
//   0 sum om, 1-3 sum om y_c, 4-9 sum om y_c y_c^T (xx xy xz yy yz zz),
//   10-12 sum om r, 13-15 sum om y_c x r, 16 sum om y_c . r,
//   17 sum w rho, 18 inlier count.
// MODE_GN_NC: a Gauss-Newton pass whose cost and inlier count (17, 18) are not
// needed (every pass but the one at the last linearisation point): left zero.
enum PassMode { MODE_MOMENTS = 0, MODE_GN = 1, MODE_COST = 2, MODE_ADJOINT = 3, MODE_GN_NC = 4 };

// Mode of pass `pass` (0: moments, 1..K: Gauss-Newton, K+1: final cost) of a call with K steps.
__host__ __device__ inline int pass_mode(int pass, int K) {
  return pass == 0 ? MODE_MOMENTS : (pass < K ? MODE_GN_NC : MODE_GN);
}

// A pair's first tile starts at a multiple of 64 elements (its head is masked),
// and tiles hold a multiple of 64 elements, so every tile boundary inside a pair
// falls on a 128-byte line of each plane (FP32: 256 B, BF16: 128 B) and no line is
// fetched by two tiles of the same pair; 16-byte vector loads stay aligned.
constexpr int64_t TILE_ALIGN = 64;

// Internal source types of the point passes: stored xyz (the public S3A_F32,
// S3A_BF16) or depth maps unprojected on the fly (Sec. III-C.1, submaps from
// depth and camera parameters), FP32 or BF16 planes.
constexpr int DT_DEPTH_F32 = 2;
constexpr int DT_DEPTH_BF16 = 3;
constexpr int DEPTH_MAX_FRAMES = 4;

// A camera as the point passes use it: x_submap = R (d ((u, v) * inv_f + o, 1)) + t.
struct DepthCam {
  float ifx, ify, ox, oy;  // 1/fx, 1/fy, -cx/fx, -cy/fy
  float R[9];
  float t[3];
};

// Per pair: frame geometry (sanitised: width, rows >= 1) and the two submaps'
// cameras of each shared frame.
struct DepthPair {
  int32_t width, rows, frame_pixels, n_frames;
  float inv_width, inv_frame;  // 1/width, 1/frame_pixels (division estimates, corrected exactly)
  int32_t pad[2];
  DepthCam p[DEPTH_MAX_FRAMES];
  DepthCam q[DEPTH_MAX_FRAMES];
};

struct TileDesc {
  int64_t begin;  // first element loaded (multiple of TILE_ALIGN)
  int64_t end;    // one past the last element of this tile
  int64_t lo;     // first element of the pair (elements in [begin, lo) are masked)
  int32_t pair;
  int32_t pad;
};

struct PairSched {
  int64_t a, b;     // element range of the pair
  int32_t tile0;    // first tile
  int32_t ntiles;   // >= 1 (an empty or bad pair gets one empty tile)
  int32_t bad;      // offsets out of order or out of range
  int32_t pad;
};

// Per-pair parameters read by the point passes.
struct PointParams {
  double M[9];   // s R (FP64), y = M p + t
  double t[3];
  double c[3];   // centre of the Gauss-Newton statistics
  float Mf[9];   // s R (FP32)
  float tcf[3];  // t - c (FP32): centred model point y_c = Mf p + tcf
  float cf[3];   // c (FP32): centred target q_c = q - cf
  float inv_C;   // 1 / C (adjoint)
  float scale;   // gL (adjoint)
  float L;       // cost (adjoint)
  int32_t active;// 0: skip (pair failed or finished)
  int32_t nonfinite; // the pair holds NaN/Inf values (validity then checks finiteness)
};

// FP64 master state per pair.
struct PairState {
  Sim3d S;
  double C;
  double cq[3];
  double cost_lin;
  double H[28];
  double g[7];
  int64_t V;
  int64_t nnf;
  int64_t inl_lin;
  int32_t status;
  int32_t iters;
};

// Per-call pointers read by every kernel of a call.
struct CallDesc {
  const void* planes[7];
  const int64_t* offsets;
  const s3a_sim3* init;  // or null
  s3a_sim3* S_out;
  s3a_align_info* info;
  // cost / adjoint
  const s3a_sim3* S_in;
  const double* xi;
  const double* L_in;
  const double* C_in;
  const double* gL;
  double* L_out;
  double* C_out;
  float* grad[7];
  double* gxi;
  const s3a_depth_pair* depth;  // caller's per-pair cameras (depth input), or null
};

// Shape of a call (passed by value).
struct Shape {
  int64_t n_points;
  int32_t n_pairs;
  int32_t K;
  float tau;
  float delta_f;
  double delta;
  uint32_t flags;
  int32_t tile_elems;
};

// Workspace pointers (device).
struct Work {
  TileDesc* tiles;
  PairSched* sched;
  PointParams* params;
  PairState* state;
  double* partials;    // [max_tiles][NSTAT]
  int32_t* total_tiles;
  uint32_t* counters;  // [n_pairs] arrivals, then 4 scheduling words
  uint32_t* flags;     // [n_pairs] per-pair published pass (persistent launch)
  int32_t* scan_tmp;
  DepthPair* dpairs;   // [n_pairs] cameras in pass form (depth input)
};

}  // namespace s3a
