/*
 * s3a: dense confidence-weighted Sim(3) alignment of submap pointmaps, its
 * cost adjoint, and the Sim(3) pose-graph solve, on one AMD Instinct MI355X
 * (gfx950). C ABI: plain pointers and sizes only.
 *
 * The problem statement follows EC3R-SLAM (arXiv 2510.02080):
 *   - Sec. III-C.2, eq. (sim3): given corresponding points P = {p_i} (current
 *     submap) and Q = {q_i} (another submap, same pixels of a shared keyframe)
 *     and confidence-derived weights w_i, find S = {s, R, t} in Sim(3)
 *     minimising sum_i w_i |s R p_i + t - q_i|^2, solved by the weighted
 *     Umeyama closed form; S becomes a relative Sim(3) edge of the pose graph.
 *   - Sec. III-E: nodes T_t in Sim(3), edge residual
 *     e_ij = Log(T_ij^{-1} T_i^{-1} T_j), energy sum e_ij^T Omega_ij e_ij,
 *     poses initialised by chaining the relative transforms.
 *
 * This library refines the closed-form start with Huber IRLS: K Gauss-Newton
 * steps on sum_i w_i rho_delta(|S p_i - q_i|), each reducing per-point
 * residuals and Jacobians to 7x7 normal equations (solved in FP64).
 *
 * Conventions
 *   - A similarity {s, R, t} maps x -> s R x + t. R is row-major.
 *   - Tangent vectors xi = (rho[3], omega[3], sigma): translation, rotation,
 *     log-scale; perturbations act on the left: S' = Exp(xi) S.
 *   - Mask and weights: point i of a pair is valid iff p_i, q_i, c_i are all
 *     finite and c_i >= conf_threshold; w_i = m_i c_i / C, C = sum m_j c_j.
 *
 * Memory and streams
 *   - "device" pointers are HIP device memory on the handle's device; "host"
 *     pointers are ordinary host memory. The caller owns every array passed
 *     in; the library keeps no pointer past the call.
 *   - Calls enqueue work on the given stream (a hipStream_t; NULL = the null
 *     stream) and return; device outputs are valid once the stream has
 *     reached that point. Calls that say they synchronise do so on that
 *     stream before returning.
 *   - A handle owns its workspace (grown on demand), captured graphs and
 *     autotuning results. A handle must not be used by two threads at once.
 *   - Calls through one handle share that workspace, so they execute in the
 *     order they were issued, whatever streams they are given: a call on a
 *     stream other than the previous call's makes its stream wait (on the
 *     device, hipStreamWaitEvent) for all work of the previous call. Work
 *     through one handle therefore never overlaps; for concurrent work on
 *     several streams, use one handle per stream.
 *
 * Errors
 *   - Every call returns S3A_OK (0) or a negative code (s3a_strerror).
 *     S3A_EINVAL: a bad argument (null pointer, negative count, unknown dtype,
 *     delta <= 0 or NaN, tau < 0 or NaN, iters < 0, misaligned plane).
 *     S3A_EHIP: a HIP runtime error (code kept, s3a_last_hip_error).
 *     S3A_ENOMEM: workspace allocation failed.
 *     S3A_ELIMIT: the batch is larger than s3a_align_pairs_noalloc's fixed
 *     scratch holds.
 *   - Problems of one pair do not fail the call: they are reported in that
 *     pair's status (S3A_PAIR_*), and the pair's outputs are the identity with
 *     cost NaN. Other pairs are unaffected, with one exception: invalid
 *     offsets (any offsets[k] > offsets[k+1], or any offset outside
 *     [0, n_points]) are detected on the device and mark EVERY pair of the
 *     call S3A_PAIR_BADRANGE, since the work split over tiles is derived from
 *     the whole offsets array.
 */
#ifndef S3A_H
#define S3A_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct s3a_handle s3a_handle;
typedef void* s3a_stream; /* hipStream_t */

/* Similarity x -> s R x + t; 128 bytes, FP64. */
typedef struct {
  double R[9]; /* row-major rotation */
  double t[3];
  double s; /* > 0 */
  double pad[3];
} s3a_sim3;

enum { S3A_F32 = 0, S3A_BF16 = 1 };

enum { S3A_OK = 0, S3A_EINVAL = -1, S3A_EHIP = -2, S3A_ENOMEM = -3, S3A_ELIMIT = -4 };

/* Per-pair status. */
enum {
  S3A_PAIR_OK = 0,
  S3A_PAIR_EMPTY = 1,      /* no valid point (or all weights zero with tau = 0) */
  S3A_PAIR_DEGENERATE = 2, /* coincident or collinear points, or a non-SPD normal matrix */
  S3A_PAIR_NONFINITE = 3,  /* no valid point and some were dropped for NaN/Inf, or a non-finite solve */
  S3A_PAIR_BADRANGE = 4,   /* the call's offsets are invalid (every pair gets it), or a depth pair's geometry is */
  S3A_PAIR_ABORTED = 5     /* the batched launch stopped waiting for this pair (internal error) */
};

/* Flags of s3a_align_desc.flags. */
#define S3A_FLAG_PLAIN 0x1u        /* one pair at a time, one launch per pass */
#define S3A_FLAG_FINAL_COST 0x2u   /* one more pass: cost and inliers at the final iterate */
#define S3A_FLAG_NO_GRAPH 0x4u     /* batched: launch directly, do not capture/replay a graph */
#define S3A_FLAG_PERSISTENT 0x8u   /* batched: one persistent launch for all passes (see s3a_align_pairs) */

/*
 * A batch of pairs in structure-of-arrays form: seven planes (px, py, pz,
 * qx, qy, qz, conf) of n_points elements each, all of one dtype (FP32, or
 * BF16 bit patterns as uint16), in device memory, each 16-byte aligned.
 * Pair k owns elements [offsets[k], offsets[k+1]).
 */
typedef struct {
  int32_t dtype;          /* S3A_F32 or S3A_BF16 */
  int32_t n_pairs;        /* >= 0 */
  int64_t n_points;       /* elements per plane, >= 0 */
  const int64_t* offsets; /* device, n_pairs + 1 entries */
  const void* px;
  const void* py;
  const void* pz; /* source points P (current submap) */
  const void* qx;
  const void* qy;
  const void* qz; /* target points Q (other submap) */
  const void* conf;     /* per-correspondence confidence */
  float conf_threshold; /* tau >= 0; valid iff conf >= tau */
  int32_t irls_iters;   /* K >= 0 Gauss-Newton steps after the closed form */
  double huber_delta;   /* delta > 0 (metres in the target frame); +inf = least squares */
  uint32_t flags;       /* S3A_FLAG_* */
  int32_t reserved;     /* 0 */
} s3a_align_desc;

/* Per-pair diagnostics of s3a_align_pairs (device array of n_pairs). */
typedef struct {
  double cost;       /* L at the last linearisation point S_{K-1}; NaN if K = 0 or failed */
  double final_cost; /* L at S_K with S3A_FLAG_FINAL_COST, else NaN */
  double weight_sum; /* C = sum m_i c_i */
  double H[28];      /* upper triangle (row-major) of the last Gauss-Newton matrix, normalised weights */
  double g[7];       /* and its gradient: L's derivative w.r.t. xi at S_{K-1} */
  int64_t n_valid;   /* V = number of valid points */
  int64_t n_nonfinite;  /* points dropped for a NaN/Inf value */
  int64_t n_inliers;    /* valid points with residual <= delta at S_{K-1} */
  int64_t final_inliers;/* the same at S_K (with S3A_FLAG_FINAL_COST) */
  int32_t status;       /* S3A_PAIR_* */
  int32_t iters;        /* Gauss-Newton steps taken */
} s3a_align_info;

int s3a_create(s3a_handle** out, int device);
int s3a_destroy(s3a_handle* h);

/*
 * Align every pair of a batch (Sec. III-C.2, eq. (sim3), refined by Huber IRLS).
 *   init:   device, n_pairs similarities used instead of the closed-form start,
 *           or NULL for the weighted Umeyama closed form.
 *   S_out:  device, n_pairs results (the K-th Gauss-Newton iterate).
 *   info:   device, n_pairs diagnostics, or NULL.
 * Batched (default): all pairs together; each pass is one launch over every
 * tile of every pair plus one FP64 finalize launch, the whole sequence
 * captured once in a graph and replayed on later calls of the same shape.
 * S3A_FLAG_PERSISTENT: all passes in one persistent launch that hands out
 * (pass, tile) work items in pass-major order and finalizes each pair when
 * its last tile of a pass arrives (its per-item cross-workgroup release and
 * acquire make it slower on multi-die parts; kept as an option).
 * S3A_FLAG_PLAIN: one pair at a time, one launch per pass; synchronises the
 * stream once to read the pair sizes.
 */
int s3a_align_pairs(s3a_handle* h, const s3a_align_desc* desc, const s3a_sim3* init,
                    s3a_sim3* S_out, s3a_align_info* info, s3a_stream stream);

/*
 * Allocation-free variant of s3a_align_pairs, for callers that cannot
 * allocate device memory: code being captured into a HIP graph, tight serving
 * loops, hosts that forbid allocation after start-up. It takes no handle,
 * allocates nothing and makes no host-device copy: it only enqueues kernels.
 *   - It runs on the calling thread's current device; `stream` must belong to
 *     that device. Arguments, outputs and per-pair statuses are those of
 *     s3a_align_pairs (batched path).
 *   - Every temporary lives in one fixed scratch array of
 *     S3A_NOALLOC_SCRATCH_BYTES per device, held by the library until the
 *     process ends. Limits: n_pairs <= S3A_NOALLOC_MAX_PAIRS, and the batch's
 *     tile bound n_points / 8192 + 2 n_pairs + 1 <= S3A_NOALLOC_MAX_TILES
 *     (about 260 million points); beyond them the call returns S3A_ELIMIT and
 *     enqueues nothing.
 *   - Launch shape fixed at tiles of 8192 elements, one workgroup per tile
 *     (FP32: 512 threads x 4 vectors; BF16: 256 x 4). The results equal, bit
 *     for bit, s3a_align_pairs' with that launch shape.
 *   - Flags: S3A_FLAG_FINAL_COST; S3A_FLAG_NO_GRAPH is accepted and changes
 *     nothing; S3A_FLAG_PLAIN and S3A_FLAG_PERSISTENT return S3A_EINVAL.
 *   - All calls on one device share that device's scratch array, which keeps
 *     the last call's contents (each call writes every word it reads before
 *     reading it). Calls that can overlap on one device (two streams, or two
 *     threads) race on it and must be serialised by the caller. Calls through
 *     a handle do not use it.
 */
#define S3A_NOALLOC_MAX_PAIRS 4096
#define S3A_NOALLOC_MAX_TILES 32768
#define S3A_NOALLOC_SCRATCH_BYTES (12u << 20)
int s3a_align_pairs_noalloc(const s3a_align_desc* desc, const s3a_sim3* init, s3a_sim3* S_out,
                            s3a_align_info* info, s3a_stream stream);

/*
 * Depth-map input (Sec. III-C.1: a submap is its keyframes' predicted depth
 * and confidence maps unprojected with the predicted camera parameters).
 * Pair k shares n_frames keyframes between its source submap (P side) and its
 * target submap (Q side); its stored elements offsets[k] .. offsets[k+1]-1 are
 * those frames' pixels, frame after frame, row-major (pixel j of the pair:
 * frame f = j / frame_pixels, column j mod width, row (j mod frame_pixels) /
 * width). Element i carries the two submaps' depths d_p, d_q of that pixel and
 * one confidence c, and the pair's points are
 *   p_i = R_p,f (d_p ((col - cx)/fx, (row - cy)/fy, 1)) + t_p,f   (camera p of frame f),
 *   q_i = R_q,f (d_q ((col - cx)/fx, (row - cy)/fy, 1)) + t_q,f   (camera q of frame f),
 * after which the alignment is exactly s3a_align_pairs' on (p_i, q_i, c_i).
 * Reading 3 planes instead of 7 moves 12 bytes per pixel (FP32) instead of 28
 * per stored point.
 */
typedef struct {
  float fx, fy, cx, cy; /* pinhole intrinsics in pixels */
  float R[9];           /* camera-to-submap rotation, row-major */
  float t[3];           /* camera centre in the submap frame */
} s3a_camera;           /* 64 bytes */

typedef struct {
  int32_t width;        /* pixels per row (>= 1) */
  int32_t frame_pixels; /* pixels per frame: width x rows (a multiple of width) */
  int32_t n_frames;     /* shared frames, 1..4; the pair holds at most n_frames x frame_pixels elements */
  int32_t reserved;     /* 0 */
  s3a_camera p[4];      /* source submap's camera of frame f */
  s3a_camera q[4];      /* target submap's camera of frame f */
} s3a_depth_pair;       /* 528 bytes */

typedef struct {
  int32_t dtype;          /* S3A_F32 or S3A_BF16: the type of the three planes */
  int32_t n_pairs;
  int64_t n_points;       /* elements of each plane */
  const int64_t* offsets; /* device, n_pairs + 1, as in s3a_align_desc */
  const void* depth_p;    /* device plane: source submap depth */
  const void* depth_q;    /* device plane: target submap depth */
  const void* conf;       /* device plane: confidence */
  const s3a_depth_pair* pairs; /* device, n_pairs */
  float conf_threshold;
  int32_t irls_iters;
  double huber_delta;
  uint32_t flags;         /* S3A_FLAG_PLAIN, S3A_FLAG_FINAL_COST, S3A_FLAG_NO_GRAPH */
  int32_t reserved;
} s3a_depth_desc;

/*
 * s3a_align_pairs on depth-map input: same outputs, statuses and tolerances.
 * A pair whose geometry is invalid (width < 1, frame_pixels not a positive
 * multiple of width, n_frames outside 1..4, nonzero reserved, or more
 * elements than n_frames x frame_pixels) gets S3A_PAIR_BADRANGE.
 */
int s3a_align_depth_pairs(s3a_handle* h, const s3a_depth_desc* desc, const s3a_sim3* init, s3a_sim3* S_out,
                          s3a_align_info* info, s3a_stream stream);

/*
 * Forward of the differentiable alignment cost, per pair:
 *   L_k = sum_i w_i rho_delta(|S'_k p_i - q_i|),  S'_k = Exp(xi_k) S_k,
 * the Huber form of eq. (sim3).
 *   S:  device, n_pairs; xi: device, 7 * n_pairs doubles, or NULL (xi = 0).
 *   L_out, C_out: device, n_pairs doubles (C = sum m_i c_i; L = NaN if C = 0).
 */
int s3a_align_cost(s3a_handle* h, const s3a_align_desc* desc, const s3a_sim3* S, const double* xi,
                   double* L_out, double* C_out, s3a_stream stream);

/*
 * Adjoint of s3a_align_cost: given gL_k = d(loss)/dL_k, writes
 *   dL/dq_i = -w_i psi_i r_i,  dL/dp_i = w_i psi_i (s'R')^T r_i,
 *   dL/dc_i = m_i (rho_i - L) / C,  dL/dxi = J_l(xi)^T sum_i w_i psi_i J_i^T r_i,
 * each scaled by gL_k (r_i = S' p_i - q_i, psi_i = rho'(e_i)/e_i, J_i = [I, -[y_i]x, y_i]).
 * Huber weights are recomputed, not stored. L and C are the forward's outputs.
 *   gpx..gqz, gc: device FP32 arrays of n_points (NULL = not wanted); entries
 *                 outside every pair's range are left untouched.
 *   gxi: device, 7 * n_pairs doubles, or NULL.
 */
int s3a_align_pairs_backward(s3a_handle* h, const s3a_align_desc* desc, const s3a_sim3* S,
                             const double* xi, const double* L, const double* C, const double* gL,
                             float* gpx, float* gpy, float* gpz, float* gqx, float* gqy, float* gqz,
                             float* gc, double* gxi, s3a_stream stream);

/*
 * Implicit derivative of the solved pose (differentiating through the
 * alignment): S_k is taken as a stationary point of the Huber cost
 * L_k(xi) = sum_i w_i rho_delta(|Exp(xi) S_k p_i - q_i|) at xi = 0. With
 * F = dL/dxi and H = d^2 L/dxi^2 there (the exact Hessian: Huber curvature
 * and the second-order terms of Exp included, not the Gauss-Newton matrix),
 * the implicit function theorem gives, for a loss l(S),
 *   dl/dtheta = -(dF/dtheta)^T v,  v = H^{-1} dl/dxi,
 * over theta = (p_i, q_i, c_i). Per valid point, with y = S p, r = y - q,
 * psi = rho'(e)/e, a = J(y) v = v_rho + v_omega x y + v_sigma y and
 * b = psi (a - [e > delta] (a . r/e) r/e):
 *   dl/dq_i = (c_i/C) b,  dl/dp_i = -(c_i/C) (sR)^T (b + psi (r x v_omega + v_sigma r)),
 *   dl/dc_i = -(psi a . r - v^T F) / C;  zero for masked points.
 *   S:     device, n_pairs solutions (typically s3a_align_pairs' output).
 *   gS:    device, dl/dS per pair: 16 doubles in s3a_sim3 layout (d/dR row-major,
 *          d/dt, d/ds; pad ignored), or with S3A_IMPLICIT_TANGENT 7 doubles
 *          d l/d xi of a left perturbation S -> Exp(xi) S.
 *   gpx..gc: device FP32 planes of n_points, 16-byte aligned (NULL = not
 *          wanted); entries outside every pair's range are left untouched.
 *   v_out: device, 7 * n_pairs doubles (v, NaN for a failed pair), or NULL.
 *   status_out: device, n_pairs int32 (S3A_PAIR_OK, EMPTY, DEGENERATE when H is
 *          not positive definite, BADRANGE), or NULL. Failed pairs get zero
 *          gradients.
 */
#define S3A_IMPLICIT_TANGENT 0x1u
int s3a_align_pairs_implicit_backward(s3a_handle* h, const s3a_align_desc* desc, const s3a_sim3* S,
                                      const double* gS, uint32_t flags, float* gpx, float* gpy, float* gpz,
                                      float* gqx, float* gqy, float* gqz, float* gc, double* v_out,
                                      int32_t* status_out, s3a_stream stream);

/* Pose-graph options. */
#define S3A_PGO_INIT_CHAIN 0x1u /* ignore T on input: chain the edges from the gauge node */
#define S3A_PGO_LM 0x2u         /* Levenberg-Marquardt (Sec. III-E) instead of fixed-damping Gauss-Newton */

typedef struct {
  int32_t iters;      /* outer iterations (20): Gauss-Newton steps, or LM steps kept */
  int32_t gauge;      /* node held fixed (0) */
  double huber_delta; /* Huber threshold on sqrt(e^T Omega e); +inf = none */
  double lambda;      /* damping along diag(H): fixed for Gauss-Newton (0 = none), the
                         starting value for LM (0 = 1e-4) */
  uint32_t flags;     /* S3A_PGO_* */
  int32_t max_rejects;/* LM: rejected trials in a row before the solve stops (0 = 10) */
} s3a_pgo_params;

typedef struct {
  double chi2[64];        /* sum e^T Omega e at each linearisation point (first 64): Gauss-Newton,
                             before step k; LM, at the start and after each kept step */
  double final_chi2;      /* at the returned poses */
  int32_t iters;          /* iterations run (LM: steps kept) */
  int32_t status;         /* 0 ok, 2 factorisation failed (graph not connected to the gauge) */
  int64_t factor_nnz_blocks; /* 7x7 blocks in the Cholesky factor (after fill) */
  double lambda_final;    /* LM: damping after the last trial */
  int32_t rejected;       /* LM: trials rejected */
  int32_t stalled;        /* LM: 1 if max_rejects trials in a row were rejected (no lower energy found) */
} s3a_pgo_report;

/*
 * Sim(3) pose-graph optimisation (Sec. III-E) with Huber edge weights and a
 * 7x7-block sparse Cholesky factorisation in FP64 on the GPU (minimum-degree
 * order; a dense trailing clique, with the columns before it that fit in its
 * padding, up to 73 nodes, is factored as one dense block on the matrix cores).
 * Gauss-Newton (default): exactly iters steps of (H + lambda diag(H)) dx = -g.
 * S3A_PGO_LM, Levenberg-Marquardt: each trial solves the same system with the
 * current lambda; it is kept when the energy F = sum rho(sqrt(e^T Omega e))
 * falls (rho the Huber loss, r^2/2 inside delta), and lambda then scales by
 * max(1/3, 1 - (2 rho - 1)^3) with rho = (F - F_trial) / predicted reduction
 * (nu = 2); otherwise the poses are restored, lambda *= nu and nu doubles. The
 * solve stops after iters kept steps, after max_rejects rejections in a row
 * (stalled), or when a trial's predicted reduction is at most 1e-15 F
 * (converged). The host reads back each trial's energy (one synchronisation
 * per trial).
 *   ij:     host, 2 * n_edges node indices (i, j) per edge; T_ij maps frame j to
 *           frame i, so a consistent graph has T_j = T_i T_ij.
 *   T_meas: device, n_edges relative similarities T_ij.
 *   omega:  device, 49 * n_edges row-major information matrices, or NULL (I).
 *   T:      device, n_nodes poses; initial values on input (unless
 *           S3A_PGO_INIT_CHAIN), optimised poses on output.
 *   report: host, or NULL.
 * Synchronises the stream (the report is host memory).
 */
int s3a_pose_graph_solve(s3a_handle* h, int32_t n_nodes, int32_t n_edges, const int32_t* ij,
                         const s3a_sim3* T_meas, const double* omega, s3a_sim3* T,
                         const s3a_pgo_params* params, s3a_pgo_report* report, s3a_stream stream);

/*
 * Pose-graph edges from pairwise alignments (Sec. III-C.2's registration result
 * becomes a Sec. III-E edge; the paper leaves the information matrix open).
 * Pair e of an s3a_align_pairs call aligned source points of submap j onto
 * target points of submap i; its result S_e is the edge's measurement
 * T_ij = S_e, and its last Gauss-Newton matrix H_e (s3a_align_info.H, for left
 * perturbations S -> Exp(xi) S, normalised weights) gives the information
 *   Omega_e = info_scale * n_valid_e * Ad(S_e)^T H_e Ad(S_e),
 * since a relative pose T = Exp(xi) S_e has edge residual
 * e = Log(S_e^-1 T) = Ad(S_e^-1) xi, so 1/2 xi^T H xi = 1/2 e^T Ad^T H Ad e.
 * With info_scale = 1/sigma^2 that is the inverse covariance of an alignment
 * of n_valid equally weighted points with isotropic noise sigma.
 *   n_edges:     pairs (>= 0); pair e gives edge e.
 *   S, info:     device, n_edges each: s3a_align_pairs' outputs.
 *   info_scale:  > 0 and finite.
 *   T_meas:      device, n_edges similarities (may be S itself: in place).
 *   omega:       device, 49 * n_edges doubles, row-major 7x7, symmetric.
 *   edge_status: device, n_edges int32 (the pair's status), or NULL. A failed
 *                pair (status != S3A_PAIR_OK) gives T_meas = identity and
 *                Omega = 0: the edge then adds nothing to the pose graph.
 * The outputs feed s3a_pose_graph_solve's T_meas and omega directly.
 */
int s3a_edges_from_alignment(s3a_handle* h, int32_t n_edges, const s3a_sim3* S, const s3a_align_info* info,
                             double info_scale, s3a_sim3* T_meas, double* omega, int32_t* edge_status,
                             s3a_stream stream);

/*
 * Launch shape of the alignment kernels. The autotuner picks one per
 * (dtype, batch size class) by timing candidates on the caller's data;
 * s3a_set_tuning forces one (for tests and sweeps).
 */
typedef struct {
  int32_t wg;       /* workgroup size: 256 or 512 */
  int32_t items;    /* vector loads per thread per tile: 2, 4, 8, or 16 (with wg 256) */
  int32_t occupancy;/* workgroups per compute unit looping over the tiles: 1..8; 0 = one workgroup
                       per tile (not for the persistent launch, which then uses 4) */
  int32_t window;   /* pairs per scheduling window in the persistent launch (0 = all) */
} s3a_tuning;

/*
 * Point correction (Sec. III-C.3), step 1: submap points to the world frame.
 * Submap k owns rows offsets[k] .. offsets[k+1]-1 of three coordinate planes
 * (x, y, z; FP32 or BF16 per dtype), and each of its rows maps to
 * s_k R_k x + t_k, formed in FP64 and rounded once to FP32, in the three FP32
 * output planes. Rows outside every submap are copied through as FP32.
 *   offsets:  device, n_submaps + 1 int64, non-decreasing, offsets[0] >= 0,
 *             offsets[n_submaps] <= n_points. Otherwise nothing is
 *             transformed, every output is NaN and *status = 1.
 *   T:        device, n_submaps similarities.
 *   x, y, z:  device planes of n_points, 16-byte aligned; out_*: device FP32
 *             planes of n_points, 16-byte aligned. With dtype F32 the outputs
 *             may be the input planes (in place).
 *   status:   device int32, or NULL: 0, or 1 for invalid offsets.
 * Bad arguments (null planes, misalignment, negative sizes) return S3A_EINVAL.
 */
int s3a_transform_points(s3a_handle* h, int32_t dtype, int64_t n_points, int32_t n_submaps, const int64_t* offsets,
                         const s3a_sim3* T, const void* x, const void* y, const void* z, float* out_x, float* out_y,
                         float* out_z, int32_t* status, s3a_stream stream);

/*
 * Point correction, step 2: points of the tracker's sparse map that have a
 * dense counterpart take its world coordinates:
 *   sparse[dst[m]] = world[src[m]]   for m < n_corr with 0 <= src[m] < n_world
 *                                    and 0 <= dst[m] < n_sparse,
 * on all three FP32 planes (device). Other m are skipped and counted: the
 * count is added to *n_skipped (device, may be NULL). src, dst: device int64.
 * Destinations should be distinct; for a repeated one, which write survives
 * is unspecified.
 */
int s3a_correct_points(s3a_handle* h, int64_t n_corr, const int64_t* src, const int64_t* dst, int64_t n_world,
                       const float* wx, const float* wy, const float* wz, int64_t n_sparse, float* sx, float* sy,
                       float* sz, unsigned long long* n_skipped, s3a_stream stream);

/* Time candidate launch shapes on this batch and keep the fastest for its
 * (dtype, size class). Synchronises the stream. best may be NULL. */
int s3a_autotune(s3a_handle* h, const s3a_align_desc* desc, s3a_tuning* best, s3a_stream stream);
/* The same for depth-map input: the shape is kept for depth-map calls of this
 * plane type and size class, apart from stored-point calls (the pass kernels do
 * different work per byte). Errors as s3a_align_depth_pairs. */
int s3a_autotune_depth(s3a_handle* h, const s3a_depth_desc* desc, s3a_tuning* best, s3a_stream stream);
/* Force one shape for every call on planes of dtype, depth-map input included. */
int s3a_set_tuning(s3a_handle* h, int32_t dtype, const s3a_tuning* t); /* t = NULL: back to automatic */
int s3a_get_tuning(s3a_handle* h, int32_t dtype, int64_t n_points, s3a_tuning* t);

/*
 * Kernel timing (profiling aid). While on, calls launch directly (no graph
 * replay) and record HIP events on the caller's stream around every launch of
 * the call's dominant point kernel: the persistent kernel of a batched call,
 * the pass kernels of a plain or multi-launch call, the adjoint kernel of a
 * backward call, the cost kernel of a cost call. s3a_kernel_time synchronises
 * on those events and returns their summed duration (ms) and launch count
 * since the previous s3a_kernel_time, then clears them.
 */
int s3a_set_timing(s3a_handle* h, int on);
int s3a_kernel_time(s3a_handle* h, double* ms, int32_t* launches);

const char* s3a_strerror(int code);
int s3a_last_hip_error(const s3a_handle* h);
/* Library version as major * 10000 + minor * 100 + patch. */
int s3a_version(void);

#ifdef __cplusplus
}
#endif

#endif /* S3A_H */
