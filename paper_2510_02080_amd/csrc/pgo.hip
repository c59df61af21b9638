// Sim(3) pose-graph optimisation (Sec. III-E) on the GPU in FP64.
//
// Nodes are submap poses T_t; edge (i, j) carries T_ij and the residual
// e_ij = Log(T_ij^{-1} T_i^{-1} T_j). Each iteration is one Gauss-Newton step
// on sum_ij rho_pg(sqrt(e^T Omega e)) (Huber weights recomputed per
// iteration; plain chi^2 when delta_pg = inf), with left perturbations
// T <- Exp(xi) T and the gauge node held fixed:
//   de/dxi_j = J_r(e)^{-1} Ad(T_j^{-1}) =: A,   de/dxi_i = -A,
// so edge (i, j) adds M = psi A^T Omega A to the diagonal blocks of i and j,
// -M to the off-diagonal block (i, j), and -/+ psi A^T Omega e to g_i / g_j.
//
// Host (once per graph topology): minimum-degree ordering of the free nodes,
// symbolic block Cholesky (column structures, elimination tree, levels), and
// fixed-order lists: which edges assemble into which block, and which pairs of
// factor blocks update which target block.
// A failed factorisation (a pivot not positive) sets the solve's status. The
// kernels of the linearisation, the factorisation and the front run whatever the
// status (all they write is workspace, rewritten in full by the next iteration or
// trial; reading the status first would put a dependent load at the head of each
// launch); the chi^2 sum and the solves kernel, which write what the caller
// reads, check it.
// Device, per iteration: the edges are linearised and H and g assembled across
// the chip; the sparse columns are factored level by level, two launches per
// level spread over the chip (the columns of a level are independent), each
// column's forward solve with its factor; the dense front (the trailing clique
// and the columns that fit in its padding) is factored one panel per launch, its
// tiles across the chip on the matrix cores, with its forward solve; one
// workgroup runs the backward solves of L L^T dx = -g and applies T <- Exp(dx) T.
#include <string.h>

#include <algorithm>
#include <deque>
#include <set>
#include <vector>

#include "align_launch.h"
#include "finalize.h"
#include "pgo.h"

namespace s3a {

// ------------------------------------------------------------------ device data

struct PgoDev {
  int32_t n_nodes, n_edges, m, gauge;   // m = free nodes
  int32_t nblk;                         // off-diagonal factor blocks
  const int32_t* ei;                    // [E] node i
  const int32_t* ej;                    // [E] node j
  const int32_t* pos;                   // [n] node -> elimination position (-1: gauge)
  const int32_t* node;                  // [m] position -> node
  // off-diagonal blocks of L, column-major: column c owns blocks [col_ptr[c], col_ptr[c+1])
  const int32_t* col_ptr;               // [m+1]
  const int32_t* blk_row;               // [nblk] row position
  const int32_t* blk_col;               // [nblk] column position
  // assembly: diagonal of position c gets +M of edges dg_edge[dg_ptr[c]..]; block b gets -M of
  // edges ob_edge[ob_ptr[b]..]; g of position c gets sign * v of edges (gv_edge, gv_sign)
  const int32_t* dg_ptr; const int32_t* dg_edge;
  const int32_t* ob_ptr; const int32_t* ob_edge;
  const int32_t* gv_ptr; const int32_t* gv_edge; const int8_t* gv_sign;
  // updates: target t (0..m-1 diagonal of position t, m + b off-diagonal block b) gets
  // -= L_a L_b^T for (a, b) in up_a/up_b[up_ptr[t]..]; a, b index blocks (always off-diagonal)
  const int32_t* up_ptr; const int32_t* up_a; const int32_t* up_b;
  // schedule of the sparse part (columns below p0), for the factorisation and both
  // solves: the columns of level l are flev_col[flev_ptr[l] .. flev_ptr[l+1]); for the
  // column at schedule position j, its targets that receive updates (its diagonal c or
  // m + one of its off-diagonal blocks) lt_tgt[ct_ptr[j] .. ct_ptr[j+1]), its row
  // blocks fs_blk[fs_ptr[j]..] (forward solve) and its column blocks bs_blk[bs_ptr[j]..]
  // (backward solve)
  int32_t nflev;
  const int32_t* flev_ptr; const int32_t* flev_col;
  const int32_t* lt_tgt; const int32_t* ct_ptr;
  // the update pairs target by target in lt_tgt order: target at position i gets
  // -= L_a L_b^T for (a, b) in fu_a/fu_b[fu_ptr[i]..fu_ptr[i+1])
  const int32_t* fu_ptr; const int32_t* fu_a; const int32_t* fu_b;
  const int32_t* fs_ptr; const int32_t* fs_blk;
  const int32_t* bs_ptr; const int32_t* bs_blk;
  const int32_t* bs_row;  // row node of each bs_blk entry
  // per level, LVW entries: j0, j1 (schedule positions), Q0 = bs_ptr[j0], Q1 = bs_ptr[j1],
  // then, when bw is kept, the offsets in bw of the level's blocks and columns and their
  // strides NQ, NJ (the counts rounded up to a wavefront)
  const int32_t* lv;
  // the backward solve's copy of the factor, level by level, element-major: element e of
  // the level's block p at [lv[4] + e NQ + p]; of its column p, the lower triangle of
  // L_cc^{-1} by rows (e < 28) and y (28 + r) at [lv[5] + e NJ + p]. Null when not kept.
  double* bw;
  int64_t bw_size;
  // dense front: the trailing columns p0 .. m-1 (K of them: a clique, each column
  // holding every block below the diagonal, and the columns before it that fit in its
  // padding). Its blocks, with the updates of the sparse columns applied (dt lists),
  // form the dense front F (order nF = 7 K padded with identity to a multiple of the
  // update tile, column-major, lower triangle), factored in place; the lower blocks
  // outside the structure (fz_rc: front-relative node row and column) and the padding
  // are rewritten every iteration. Finv holds the inverses of the front's FB x FB
  // diagonal blocks (row-major) for the solves.
  int32_t K, p0, n_dt, nF, n_fz;
  const int32_t* dt_tgt; const int32_t* dt_ptr; const int32_t* dup_a; const int32_t* dup_b;
  const int32_t* fz_rc;
  double* F;
  double* Finv;
  double* Frd;    // [nF] 1 / L_jj of the front's factor
  double* yF;     // [nF] the front's right-hand side, updated panel by panel by the forward solve
  double* zF;     // [nF] the front's forward solve L_F z = y, block by block
  // rows of L: blocks (c, k), k < c (the front rows' right-hand side)
  const int32_t* row_ptr; const int32_t* row_blk;
  // chaining order: (node, parent, edge, dir) for nodes reached by breadth-first search
  const int32_t* chain; int32_t n_chain;
  // breadth-first depth levels of the chain: entries [chain_lev[l], chain_lev[l+1]) have depth l + 1
  const int32_t* chain_lev; int32_t n_chain_lev;
  // numeric storage
  double* Ld;     // [m][49] diagonal blocks (lower Cholesky factor after factorisation)
  double* Di;     // [m][49] inverses of the factored diagonal blocks of the sparse columns
  double* Lb;     // [nblk][49]
  double* g;      // [m][7]  gradient, then solution
  double* M;      // [E][49] per-edge psi A^T Omega A
  double* Aw;     // [E][56] per-edge Jacobian A and Om e (scratch of the linearisation)
  double* v;      // [E][7]  per-edge psi A^T Omega e
  double* r2;     // [E]     e^T Omega e
  double* chi2;   // [iters + 1]
  int32_t* status;
  // Levenberg-Marquardt: the undamped system of the last solve and its predicted reduction
  double* gsave;  // [m][7] right-hand side -g
  double* dsave;  // [m][7] diagonal of H
  double* pred;   // [1] dx^T (lambda diag(H) dx - g) / 2
};

__device__ inline Sim3d ld_pose(const s3a_sim3* p) { return load_sim3(p); }

// Breadth-first chaining from the gauge node: T_j = T_i T_ij (dir 0) or
// T_i = T_j T_ij^{-1} (dir 1), one workgroup, the entries of one depth level in
// parallel (each depends only on a parent of the level before).
constexpr int CHAIN_WG = 256;
__global__ __launch_bounds__(CHAIN_WG) void k_pgo_chain(PgoDev d, const s3a_sim3* __restrict__ Tm, s3a_sim3* T) {
  const int tid = threadIdx.x;
  for (int k = tid; k < d.n_nodes; k += CHAIN_WG) store_sim3(T + k, sim3_identity());
  __syncthreads();
  for (int l = 0; l < d.n_chain_lev; ++l) {
    for (int c = d.chain_lev[l] + tid; c < d.chain_lev[l + 1]; c += CHAIN_WG) {
      const int nd = d.chain[4 * c], par = d.chain[4 * c + 1], e = d.chain[4 * c + 2], dir = d.chain[4 * c + 3];
      const Sim3d Tp = ld_pose(T + par);
      const Sim3d Te = ld_pose(Tm + e);
      store_sim3(T + nd, dir == 0 ? sim3_compose(Tp, Te) : sim3_compose(Tp, sim3_inverse(Te)));
    }
    __syncthreads();
  }
}

// Orders the LDS writes of a wavefront's lanes before the reads that follow, for
// lanes that exchange values through LDS without a workgroup barrier.
__device__ inline void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Edges per wavefront in the linearisation (seven lanes each).
constexpr int LIN_EDGES = 9;

// Seven lanes per edge, lane i = row i: residual e = Log(T_ij^{-1} T_i^{-1} T_j),
// e^T Om e, and row i of the Jacobian A = J_r(e)^{-1} Ad(T_j^{-1}) into Aw (with
// Om e after it). Row i of J_r = sum_n (-ad e)^n / (n+1)! is formed by the lane
// alone; the inverse is Gauss-Jordan with partial pivoting on rows shared in LDS
// within the wavefront. M = psi A^T Om A and
// v = psi A^T Om e follow in k_pgo_edge_M.
__global__ __launch_bounds__(64) void k_pgo_linearize(PgoDev d, const s3a_sim3* __restrict__ Tm,
                                                     const double* __restrict__ omega, const s3a_sim3* __restrict__ T,
                                                     int r2_only) {
  __shared__ double aug[LIN_EDGES][7][14];
  const int lane = threadIdx.x, g = lane / 7, i = lane % 7;
  const int k = blockIdx.x * LIN_EDGES + g;
  if (g >= LIN_EDGES || k >= d.n_edges) return;
  const Sim3d Ti = ld_pose(T + d.ei[k]);
  const Sim3d Tj = ld_pose(T + d.ej[k]);
  const Sim3d Tij = ld_pose(Tm + k);
  const Sim3d Z = sim3_compose(sim3_compose(sim3_inverse(Tij), sim3_inverse(Ti)), Tj);
  double e[7];
  sim3_log(Z, e);
  const double* Om = omega ? omega + 49 * k : nullptr;
  double Oe[7];
  for (int a = 0; a < 7; ++a) {
    double s = 0.0;
    if (Om) for (int b = 0; b < 7; ++b) s += Om[7 * a + b] * e[b];
    else s = e[a];
    Oe[a] = s;
  }
  double q = 0.0;
  for (int a = 0; a < 7; ++a) q += e[a] * Oe[a];
  if (i == 0) d.r2[k] = q;
  if (r2_only) return;
  double* Ag = d.Aw + 56 * k;
  if (i == 0)
    for (int a = 0; a < 7; ++a) Ag[49 + a] = Oe[a];
  double row[14];
  {
    double A[49];
    sim3_ad(e, A);
    double P[7];
    for (int j = 0; j < 7; ++j) {
      P[j] = j == i ? 1.0 : 0.0;
      row[j] = P[j];
    }
    for (int n = 1; n < 80; ++n) {
      double Q[7], mx = 0.0;
      for (int j = 0; j < 7; ++j) {
        double v = 0.0;
        for (int c = 0; c < 7; ++c) v -= P[c] * A[7 * c + j];
        Q[j] = v / (double)(n + 1);
      }
      for (int j = 0; j < 7; ++j) {
        P[j] = Q[j];
        row[j] += Q[j];
        const double x = fabs(Q[j]);
        mx = x > mx ? x : mx;
      }
      if (mx < 1e-18) break;
    }
  }
  for (int j = 0; j < 7; ++j) row[7 + j] = j == i ? 1.0 : 0.0;
  double(*M)[14] = aug[g];
  for (int j = 0; j < 14; ++j) M[i][j] = row[j];
  wave_sync();
  bool ok = true;
  for (int c = 0; c < 7; ++c) {
    int p = c;
    for (int r = c + 1; r < 7; ++r)
      if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
    ok = ok && M[p][c] != 0.0;
    if (p != c && (i == c || i == p)) {  // exchange rows c and p
      const int o = i == c ? p : c;
      for (int j = 0; j < 14; ++j) row[j] = M[o][j];
      wave_sync();
      for (int j = 0; j < 14; ++j) M[i][j] = row[j];
    }
    wave_sync();
    const double dv = ok ? 1.0 / M[c][c] : 0.0;
    const double f = i == c ? 0.0 : M[i][c];
    for (int j = 0; j < 14; ++j) row[j] = i == c ? M[c][j] * dv : M[i][j] - f * (M[c][j] * dv);
    wave_sync();
    for (int j = 0; j < 14; ++j) M[i][j] = row[j];
    wave_sync();
  }
  double Ad[49];
  sim3_Ad(sim3_inverse(Tj), Ad);
  for (int b = 0; b < 7; ++b) {
    double s = 0.0;
    for (int c = 0; c < 7; ++c) s += row[7 + c] * Ad[7 * c + b];
    Ag[7 * i + b] = ok ? s : __builtin_nan("");
  }
}

// M = psi A^T (Om A) and v = psi A^T (Om e) per edge, one thread per element,
// over the whole chip.
__global__ __launch_bounds__(256) void k_pgo_edge_M(PgoDev d, const double* __restrict__ omega, double huber) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (int64_t)d.n_edges * 56) return;
  const int k = (int)(x / 56), t = (int)(x % 56);
  const double q = d.r2[k];
  const double r = sqrt(q > 0.0 ? q : 0.0);
  const double psi = r <= huber ? 1.0 : huber / r;
  const double* A = d.Aw + 56 * k;
  if (t >= 49) {
    const int b = t - 49;
    double s = 0.0;
    for (int a = 0; a < 7; ++a) s += A[7 * a + b] * A[49 + a];
    d.v[7 * k + b] = psi * s;
    return;
  }
  const int a = t / 7, b = t % 7;
  const double* Om = omega ? omega + 49 * k : nullptr;
  double s = 0.0;
  for (int c = 0; c < 7; ++c) {
    double oab = A[7 * c + b];  // (Om A)[c][b]
    if (Om) {
      oab = 0.0;
      for (int u = 0; u < 7; ++u) oab += Om[7 * c + u] * A[7 * u + b];
    }
    s += A[7 * c + a] * oab;
  }
  d.M[49 * k + 7 * a + b] = psi * s;
}

// Per-edge linearisation at T into d (r2 only, or r2, v and M).
hipError_t launch_linearize(const PgoDev& d, const s3a_sim3* Tm, const double* omega, const s3a_sim3* T, double huber,
                            int r2_only, hipStream_t st) {
  if (d.n_edges == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pgo_linearize, dim3((d.n_edges + LIN_EDGES - 1) / LIN_EDGES), dim3(64), 0, st, d, Tm, omega, T,
                     r2_only);
  if (!r2_only) {
    const int64_t nx = (int64_t)d.n_edges * 56;
    hipLaunchKernelGGL(k_pgo_edge_M, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, d, omega, huber);
  }
  return hipGetLastError();
}

constexpr int PGO_WG = 1024;

// Deterministic workgroup sum of per-lane doubles (fixed tree) over WG threads.
template <int WG>
__device__ inline double wg_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < WG / 64; ++q) s += sh[q];
    sh[WG / 64] = s;
  }
  __syncthreads();
  s = sh[WG / 64];
  __syncthreads();
  return s;
}

// Dense front of the trailing columns: at most PGO_KMAX node columns; panels of FB
// columns, trailing updates in FT x FT tiles.
constexpr int PGO_KMAX = 73;
constexpr int FB = 32;
constexpr int FT = 64;
constexpr int FRONT_MAX = 512;
typedef double d4 __attribute__((ext_vector_type(4)));
static_assert((7 * PGO_KMAX + FT - 1) / FT * FT <= FRONT_MAX, "front order");
constexpr int FIN_WG = 512;  // solves: 256 registers per lane
static_assert(FIN_WG % FB == 0 && (FIN_WG / FB) <= 64 && ((FIN_WG / FB) & (FIN_WG / FB - 1)) == 0, "row slots per front column");

// Element `lane` of factor block `target` (diagonal c, or m + off-diagonal block).
__device__ inline double* target_elem(const PgoDev& d, int target, int lane) {
  const int e = lane < 49 ? lane : 0;
  return target < d.m ? d.Ld + 49 * target + e : d.Lb + 49 * (target - d.m) + e;
}

// S -= sum_q L_a L_b^T over one target's update list [q0, q1) (blocks a = ua[q], b = ub[q]),
// by one wavefront, lane = element (r, s) of the 7x7 block, in list order. The block
// indices are fetched 64 at a time, one per lane, and read back from lanes (uniform),
// so the only dependent loads left are the blocks; four updates are in flight.
// The lane's element is read from `src` and the result written to `dst`.
__device__ inline void update_target(const PgoDev& d, const double* src, double* dst, int q0, int q1,
                                     const int32_t* ua, const int32_t* ub, int lane) {
  const int r = lane < 49 ? lane / 7 : 0, s = lane < 49 ? lane % 7 : 0;
  const double old = *src;  // issued first: its latency overlaps the update loads
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  for (int qb = q0; qb < q1; qb += 64) {
    const int nq = min(64, q1 - qb);
    const int ia = lane < nq ? ua[qb + lane] : 0;
    const int ib = lane < nq ? ub[qb + lane] : 0;
    int u = 0;
    for (; u + 4 <= nq; u += 4) {
      const double* A0 = d.Lb + 49 * __shfl(ia, u, 64) + 7 * r;
      const double* B0 = d.Lb + 49 * __shfl(ib, u, 64) + 7 * s;
      const double* A1 = d.Lb + 49 * __shfl(ia, u + 1, 64) + 7 * r;
      const double* B1 = d.Lb + 49 * __shfl(ib, u + 1, 64) + 7 * s;
      const double* A2 = d.Lb + 49 * __shfl(ia, u + 2, 64) + 7 * r;
      const double* B2 = d.Lb + 49 * __shfl(ib, u + 2, 64) + 7 * s;
      const double* A3 = d.Lb + 49 * __shfl(ia, u + 3, 64) + 7 * r;
      const double* B3 = d.Lb + 49 * __shfl(ib, u + 3, 64) + 7 * s;
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        acc0 += A0[k] * B0[k];
        acc1 += A1[k] * B1[k];
        acc2 += A2[k] * B2[k];
        acc3 += A3[k] * B3[k];
      }
    }
    for (; u < nq; ++u) {
      const double* A0 = d.Lb + 49 * __shfl(ia, u, 64) + 7 * r;
      const double* B0 = d.Lb + 49 * __shfl(ib, u, 64) + 7 * s;
#pragma unroll
      for (int k = 0; k < 7; ++k) acc0 += A0[k] * B0[k];
    }
  }
  if (lane < 49) *dst = old - ((acc0 + acc1) + (acc2 + acc3));
}

// In-place Cholesky of one 7x7 diagonal block by one lane (row by row), zeroing
// the upper triangle, and the inverse of the factor into Di (and its lower
// triangle, row by row, to copy[e * cstride] when given): each diagonal element is
// inverted once, so the triangular solves that use the block need no divisions.
// False if a pivot is not positive.
__device__ inline bool chol7_lane(double* D, double* Di, double* copy, int cstride) {
  double L[7][7];
  double rinv[7];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
#pragma unroll
    for (int k = 0; k <= i; ++k) {
      double v = D[7 * i + k];
#pragma unroll
      for (int q = 0; q < k; ++q) v -= L[i][q] * L[k][q];
      if (k == i) {
        ok = ok && v > 0.0;
        L[i][i] = sqrt(v > 0.0 ? v : 1.0);
        rinv[i] = 1.0 / L[i][i];
      } else {
        L[i][k] = v * rinv[k];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 7; ++i)
#pragma unroll
    for (int k = 0; k < 7; ++k) D[7 * i + k] = k <= i ? L[i][k] : 0.0;
  // column j of L^{-1} by forward substitution against e_j
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double v[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      if (i < j) {
        v[i] = 0.0;
      } else if (i == j) {
        v[i] = rinv[j];
      } else {
        double t = 0.0;
#pragma unroll
        for (int k = j; k < i; ++k) t += L[i][k] * v[k];
        v[i] = -t * rinv[i];
      }
      Di[7 * i + j] = v[i];
      if (copy && i >= j) copy[(i * (i + 1) / 2 + j) * cstride] = v[i];
    }
  }
  return ok;
}

// One row of L_ij = S_ij L_jj^{-T} in place, with Dinv = L_jj^{-1}; optionally
// copied to copy[j * cstride] as well.
__device__ inline void trsm_row(double* row, const double* Dinv, double* copy, int cstride) {
  double x[7], y[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) x[k] = row[k];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k <= j; ++k) v += x[k] * Dinv[7 * j + k];
    y[j] = v;
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) row[j] = y[j];
  if (copy)
#pragma unroll
    for (int j = 0; j < 7; ++j) copy[j * cstride] = y[j];
}

// Assembly of the normal equations from the per-edge linearisations:
// independent sums, spread over the whole chip.
__global__ __launch_bounds__(256) void k_pgo_assemble(PgoDev d, double lambda, int lm) {
  const int gt = blockIdx.x * blockDim.x + threadIdx.x, gs = gridDim.x * blockDim.x;
  // ---- assembly (diagonal blocks, off-diagonal blocks, gradient)
  for (int x = gt; x < d.m * 49; x += gs) {
    const int c = x / 49, a = x % 49;
    double s = 0.0;
    for (int q = d.dg_ptr[c]; q < d.dg_ptr[c + 1]; ++q) s += d.M[49 * d.dg_edge[q] + a];
    if (lm && a % 8 == 0) d.dsave[7 * c + a / 8] = s;
    if (lambda > 0.0 && a % 8 == 0) s += lambda * s;
    d.Ld[x] = s;
  }
  for (int x = gt; x < d.nblk * 49; x += gs) {
    const int b = x / 49, a = x % 49;
    double s = 0.0;
    for (int q = d.ob_ptr[b]; q < d.ob_ptr[b + 1]; ++q) s -= d.M[49 * d.ob_edge[q] + a];
    d.Lb[x] = s;
  }
  for (int x = gt; x < d.m * 7; x += gs) {
    const int c = x / 7, a = x % 7;
    double s = 0.0;
    for (int q = d.gv_ptr[c]; q < d.gv_ptr[c + 1]; ++q) s += (double)d.gv_sign[q] * d.v[7 * d.gv_edge[q] + a];
    d.g[x] = -s;  // right-hand side -g
    if (lm) d.gsave[x] = -s;
  }
}

// chi^2 at the linearisation point (fixed order), by one workgroup.
__global__ __launch_bounds__(PGO_WG) void k_pgo_chi2(PgoDev d, int it) {
  __shared__ double sh[PGO_WG / 64 + 1];
  if (*d.status != 0) return;
  double part = 0.0;
  for (int k = threadIdx.x; k < d.n_edges; k += PGO_WG) part += d.r2[k];
  const double c2 = wg_sum<PGO_WG>(part, sh);
  if (threadIdx.x == 0) d.chi2[it] = c2;
}

// One level of the sparse factorisation spread over the chip, in two launches
// (the columns of a level are independent):
//  k_pgo_level_updates: every target of the level's columns (a diagonal block or
//    an off-diagonal block that receives updates) takes its updates L_a L_b^T from
//    the factored columns below, one wavefront per target across the chip;
//  k_pgo_level_factor: a workgroup per column; one lane factors and inverts the
//    diagonal block, and one thread per row forms the off-diagonal rows
//    L_ij = S_ij L_jj^{-T}.
constexpr int LEV_WG = 256;
constexpr int LVW = 8;  // entries per level of the level table
// A level's entries of the table, passed to its factor launch by value.
struct LevelArg {
  int j0, j1, Q0, lb, dc, NQ, NJ;
};
// (The level's ranges come from the host as arguments: read from the index lists
// they would be a chain of dependent loads before any work.)
__global__ __launch_bounds__(LEV_WG) void k_pgo_level_updates(PgoDev d, int i0, int i1) {
  const int lane = threadIdx.x & 63;
  const int waves = (int)gridDim.x * (LEV_WG / 64);
  for (int i = i0 + (int)blockIdx.x * (LEV_WG / 64) + ((int)threadIdx.x >> 6); i < i1; i += waves) {
    double* e = target_elem(d, d.lt_tgt[i], lane);
    update_target(d, e, e, d.fu_ptr[i], d.fu_ptr[i + 1], d.fu_a, d.fu_b, lane);
  }
}

__global__ __launch_bounds__(LEV_WG) void k_pgo_level_factor(PgoDev d, int l, LevelArg la) {
  __shared__ int s_fail;
  __shared__ double part[LEV_WG / 64][7];
  __shared__ double sDi[49];  // L_cc^{-1}: read by the forward solve and the panel rows from LDS
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = la.j0 + (int)blockIdx.x; j < la.j1; j += (int)gridDim.x) {
    const int col = d.flev_col[j];
    // the backward solve's copy of this column (level-major, element-major: one
    // coalesced read per element for a level's columns and blocks)
    const int pj = j - la.j0, NJ = la.NJ;
    double* bwc = d.bw ? d.bw + la.dc + pj : nullptr;
    if (threadIdx.x == 0) s_fail = chol7_lane(d.Ld + 49 * col, sDi, bwc, NJ) ? 0 : 1;
    // forward solve of this column, y_c = L_cc^{-1} (y_c - sum_k L_ck y_k): its row blocks
    // (c, k) lie in factored columns of lower levels, whose y_k are final; per-thread
    // sums over the blocks (strided), then a fixed tree
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int q = d.fs_ptr[j] + (int)threadIdx.x; q < d.fs_ptr[j + 1]; q += LEV_WG) {
      const int b = d.fs_blk[q];
      const double* L = d.Lb + 49 * b;
      const double* y = d.g + 7 * d.blk_col[b];
      double yv[7];
#pragma unroll
      for (int u = 0; u < 7; ++u) yv[u] = y[u];
#pragma unroll
      for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int u = 0; u < 7; ++u) acc[r] += L[7 * r + u] * yv[u];
    }
    wave_totals_f64(acc);
    if (lane == 0)
#pragma unroll
      for (int r = 0; r < 7; ++r) part[wv][r] = acc[r];
    __syncthreads();
    if (s_fail) {
      if (threadIdx.x == 0) *d.status = 2;
      return;
    }
    if (threadIdx.x >= 64 && threadIdx.x < 64 + 49) d.Di[49 * col + threadIdx.x - 64] = sDi[threadIdx.x - 64];
    if (threadIdx.x == 0) {
      double v[7];
#pragma unroll
      for (int r = 0; r < 7; ++r) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < LEV_WG / 64; ++q) s += part[q][r];
        v[r] = d.g[7 * col + r] - s;
      }
#pragma unroll
      for (int r = 0; r < 7; ++r) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k <= r; ++k) t += sDi[7 * r + k] * v[k];
        d.g[7 * col + r] = t;
        if (bwc) bwc[(28 + r) * NJ] = t;
      }
    }
    const int b0 = d.col_ptr[col], nb = d.col_ptr[col + 1] - b0;
    const int pq = d.bs_ptr[j] - la.Q0, NQ = la.NQ;
    for (int x = (int)threadIdx.x; x < 7 * nb; x += LEV_WG)
      trsm_row(d.Lb + 49 * (b0 + x / 7) + 7 * (x % 7), sDi,
               d.bw ? d.bw + la.lb + 7 * (x % 7) * NQ + pq + x / 7 : nullptr, NQ);
    __syncthreads();
  }
}

// Everything the front needs from the sparse part, one wavefront per item, spread
// over the whole chip (the items are independent):
//   [0, n_dt)              a front block with the sparse columns' updates applied;
//   [n_dt, + n_fz)         a lower block outside the structure, zero;
//   [.., + K)              front node row i's right-hand side after the sparse
//                          columns' forward solve, y_i - sum over sparse k of L_ik y_k,
//                          into yF;
//   [.., + pad waves)      the padding rows' lower entries, identity (and their
//                          right-hand side, zero).
__global__ __launch_bounds__(256) void k_pgo_clique_updates(PgoDev d) {
  int ti = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int r = lane < 49 ? lane / 7 : 0, s = lane < 49 ? lane % 7 : 0;
  if (ti < d.n_dt) {
    const int t = d.dt_tgt[ti];
    const int row = t < d.m ? t : d.blk_row[t - d.m], col = t < d.m ? t : d.blk_col[t - d.m];
    double* dst = d.F + (size_t)(7 * (col - d.p0) + s) * d.nF + 7 * (row - d.p0) + r;
    update_target(d, target_elem(d, t, lane), dst, d.dt_ptr[ti], d.dt_ptr[ti + 1], d.dup_a, d.dup_b, lane);
    return;
  }
  ti -= d.n_dt;
  if (ti < d.n_fz) {
    const int row = d.fz_rc[2 * ti], col = d.fz_rc[2 * ti + 1];
    if (lane < 49) d.F[(size_t)(7 * col + s) * d.nF + 7 * row + r] = 0.0;
    return;
  }
  ti -= d.n_fz;
  if (ti < d.K) {
    const int c = d.p0 + ti;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int q = d.row_ptr[c] + lane; q < d.row_ptr[c + 1]; q += 64) {
      const int b = d.row_blk[q];
      const int k = d.blk_col[b];
      if (k >= d.p0) continue;
      const double* L = d.Lb + 49 * b;
      const double* y = d.g + 7 * k;
      double yv[7];
#pragma unroll
      for (int u = 0; u < 7; ++u) yv[u] = y[u];
#pragma unroll
      for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int u = 0; u < 7; ++u) acc[i] += L[7 * i + u] * yv[u];
    }
    wave_totals_f64(acc);
    if (lane < 7) {
      double a = acc[0];
#pragma unroll
      for (int i = 1; i < 7; ++i) a = lane == i ? acc[i] : a;
      d.yF[7 * ti + lane] = d.g[7 * c + lane] - a;
    }
    return;
  }
  ti -= d.K;
  // padding rows nK .. nF-1 (fewer than FT): zero right-hand side; their lower
  // entries, columns 0 .. row: 256 per wavefront, row by row
  const int n = d.nF, nK = 7 * d.K;
  if (ti == 0 && nK + lane < n) d.yF[nK + lane] = 0.0;
  const int64_t n_pad = (int64_t)(n - nK) * (n + nK + 1) / 2;
  for (int64_t x = (int64_t)ti * 256 + lane; x < min((int64_t)(ti + 1) * 256, n_pad); x += 64) {
    // row nK + j starts at offset j (2 nK + j + 1) / 2
    int j = (int)((sqrt(8.0 * (double)x + (2.0 * nK + 1) * (2.0 * nK + 1)) - (2.0 * nK + 1)) * 0.5);
    while (j > 0 && (int64_t)j * (2 * nK + j + 1) / 2 > x) --j;
    while ((int64_t)(j + 1) * (2 * nK + j + 2) / 2 <= x) ++j;
    const int row = nK + j, col = (int)(x - (int64_t)j * (2 * nK + j + 1) / 2);
    d.F[(size_t)col * n + row] = row == col ? 1.0 : 0.0;
  }
}

// Wavefronts of k_pgo_clique_updates.
inline int64_t clique_update_waves(const PgoDev& d) {
  const int64_t n_pad = (int64_t)(d.nF - 7 * d.K) * (d.nF + 7 * d.K + 1) / 2;
  return (int64_t)d.n_dt + d.n_fz + d.K + (n_pad + 255) / 256;
}

// Identity padding of the front (rows and columns 7 K .. nF-1), zeros elsewhere.
__global__ __launch_bounds__(256) void k_pgo_front_init(PgoDev d) {
  const size_t n = (size_t)d.nF, x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n * n) return;
  const size_t r = x % n, c = x / n;
  d.F[x] = (r == c && r >= (size_t)(7 * d.K)) ? 1.0 : 0.0;
}

__device__ inline double readlane_f64(double x, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// LDS of the diagonal-block factor: columns being broadcast (two buffers used in turn).
__shared__ double front_cb[2 * (FB + 1)];

// Right-looking blocked Cholesky of the front F (order nF, a multiple of FT;
// column-major, lower triangle) in place, panel by panel of FB columns, one
// launch per panel across the chip (the diagonal blocks stay a chain: each
// panel needs the previous one's update):
//   k_front_diag    the first diagonal block (one wavefront, front_factor);
//   k_front_update  panel k0, whose diagonal block is factored: one workgroup per
//                   FT x FT tile of the trailing lower triangle solves the panel
//                   rows it needs and updates its tile on the matrix cores; the
//                   workgroup of the leading tile then factors the next diagonal
//                   block, and one more workgroup inverts panel k0's diagonal
//                   block for the backward solve (front_inverse), off the chain.
// The last diagonal block is solved by substitution in the solves kernel, so no
// inverse is formed on the chain. Only the factor of each diagonal block is on
// the chain: pivots by reciprocal square root (hardware estimate, two Newton
// steps), no division.
constexpr int FRONT_TWG = 256;

// (1) on the chain: the FB x FB diagonal block at (kd, kd) factored by one
// wavefront (lane = row, right-looking: the pivot is read from its lane, each
// updated column goes to LDS one step before it is needed) from src (element
// (i, c) at src[c * ld + i]: the block in F, or a copy in LDS) into F; 1 / L_jj
// to rd. False (in every lane) if a pivot is not positive.
__device__ __attribute__((always_inline)) inline bool front_factor(const double* src, int ld, double* F, int n, int kd,
                                                                  int lane, double* rd) {
  double* cb = front_cb;
  const int r = lane < FB ? lane : FB - 1, e = lane < FB ? lane : FB;
  double a[FB];  // row r; entries above the diagonal carry values that are never read
#pragma unroll
  for (int c = 0; c < FB; ++c) a[c] = src[(size_t)c * ld + (c <= r ? r : c)];
  bool ok = true;
  double rv = 1.0;
  cb[e] = a[0];
  wave_sync();
#pragma unroll
  for (int k = 0; k < FB; ++k) {
    double* cur = cb + (k & 1) * (FB + 1);
    double* nxt = cb + ((k + 1) & 1) * (FB + 1);
    // the column's entries below the pivot, all read before the pivot's chain
    // (their LDS latency overlaps it instead of each read waiting in turn)
    double cv[FB];
#pragma unroll
    for (int j = k + 1; j < FB; ++j) cv[j] = cur[j];
    __builtin_amdgcn_sched_barrier(0);
    const double dkk = readlane_f64(a[k], k);
    ok = ok && dkk > 0.0;
    const double x = dkk > 0.0 ? dkk : 1.0;
    double rk = __builtin_amdgcn_rsq(x);
    rk = rk * fma(-0.5 * x * rk, rk, 1.5);
    rk = rk * fma(-0.5 * x * rk, rk, 1.5);
    const double lkk = x * rk;
    a[k] = lane == k ? lkk : a[k] * rk;
    rv = lane == k ? rk : rv;
    const double m = a[k] * rk;  // L_rk / L_kk, and L_jk = cur[j] / L_kk
    if (k + 1 < FB) {
      a[k + 1] -= m * cv[k + 1];
      nxt[e] = a[k + 1];
    }
#pragma unroll
    for (int j = k + 2; j < FB; ++j) a[j] -= m * cv[j];
    wave_sync();
  }
  if (lane < FB) {
#pragma unroll
    for (int c = 0; c < FB; ++c)
      if (c <= lane) F[(size_t)(kd + c) * n + kd + lane] = a[c];
    rd[lane] = rv;
  }
  return ok;
}

// The inverse V = L_kk^{-1} of a factored diagonal block (row-major, to Vg), by
// one wavefront: lane = column, forward substitution against e_lane.
__device__ __noinline__ void front_inverse(const double* F, int n, int kd, int lane, const double* rd, double* Vg,
                                     double* Ls) {
  for (int x = lane; x < FB * FB; x += 64) {
    const int c = x / FB, i = x % FB;  // L(i, c) by column
    Ls[c * (FB + 1) + i] = i >= c ? F[(size_t)(kd + c) * n + kd + i] : 0.0;
  }
  wave_sync();
  double t[FB];
#pragma unroll
  for (int i = 0; i < FB; ++i) t[i] = i == lane ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < FB; ++k) {
    const double v = t[k] * rd[k];
    t[k] = v;
#pragma unroll
    for (int i = k + 1; i < FB; ++i) t[i] -= Ls[k * (FB + 1) + i] * v;
  }
  if (lane < FB) {
#pragma unroll
    for (int i = 0; i < FB; ++i) Vg[i * FB + lane] = t[i];
  }
}

// Forward substitution z = L_kk^{-1} y through a factored FB x FB diagonal block
// (strictly lower part by column in Ls, 1 / L_jj in rd), by one wavefront: lane
// i < FB holds y_i on entry and z_i on return.
__device__ inline double front_subst(double v, const double* Ls, const double* rd, int lane) {
#pragma unroll
  for (int k = 0; k < FB; ++k) {
    const double zk = readlane_f64(v, k) * rd[k];
    if (lane > k && lane < FB) v -= Ls[k * (FB + 1) + lane] * zk;
    v = lane == k ? zk : v;
  }
  return v;
}


__global__ __launch_bounds__(64) void k_front_diag(PgoDev d, int kd) {
  if (!front_factor(d.F + (size_t)kd * d.nF + kd, d.nF, d.F, d.nF, kd, (int)threadIdx.x, d.Frd + kd) &&
      threadIdx.x == 0)
    *d.status = 2;
}

// Rows i < nrow of P (by column: P[k * FT + i], row i of the panel's columns
// k0..k0 + FB - 1) solved in place against the factored diagonal block:
// L_kk x = a, right-looking, one thread per row (L_kk and 1 / L_jj from LDS).
__device__ __attribute__((always_inline)) inline void front_solve_rows(double* P, int nrow, int t, const double* Ls,
                                                                    const double* rds) {
  if (t >= nrow) return;
  double x[FB], rd[FB];
#pragma unroll
  for (int c = 0; c < FB; ++c) x[c] = P[c * FT + t];
#pragma unroll
  for (int c = 0; c < FB; ++c) rd[c] = rds[c];
  // column k of L_kk below the diagonal, read one step ahead of its use
  double lk[FB];
#pragma unroll
  for (int j = 1; j < FB; ++j) lk[j] = Ls[j];
#pragma unroll
  for (int k = 0; k < FB; ++k) {
    double ln[FB];
#pragma unroll
    for (int j = k + 2; j < FB; ++j) ln[j] = Ls[(k + 1) * (FB + 1) + j];
    __builtin_amdgcn_sched_barrier(0);
    x[k] *= rd[k];
#pragma unroll
    for (int j = k + 1; j < FB; ++j) x[j] -= lk[j] * x[k];
#pragma unroll
    for (int j = k + 2; j < FB; ++j) lk[j] = ln[j];
  }
#pragma unroll
  for (int c = 0; c < FB; ++c) P[c * FT + t] = x[c];
}

// Panel k0 (its diagonal block factored by the previous launch) and the
// trailing update it makes, one launch: workgroup b < ntile takes the FT x FT
// tile (I, J) of the lower triangle from s0 = k0 + FB, solves the panel rows of
// tile rows I and J against the diagonal block itself (rows are solved by every
// tile that needs them, in parallel; tile (I, 0) stores row block I of the
// panel), then A_IJ -= L_I L_J^T on the matrix cores, a 32 x 32 quadrant per
// wavefront (16 x 16 x 4 products, computed transposed: the lane holds
// D[jb + l4 + 4 v][ib + l16], so that each lane group reads and writes 16
// consecutive rows of a column of F). The workgroup of tile (0, 0) then factors
// the next diagonal block, which its first wavefront has just updated; the last
// workgroup inverts the panel's diagonal block for the solves.
__global__ __launch_bounds__(FRONT_TWG) void k_front_update(PgoDev d, int k0) {
  __shared__ double Pa[FB * FT], Pb[FB * FT];  // panel rows of tile column J (a) and tile row I (b): [k][i]
  __shared__ double Ls[FB * (FB + 1)];         // L_kk by column, strictly lower: Ls[c * (FB + 1) + i]
  __shared__ double rds[FB];
  __shared__ double zs[FB];  // the panel's block of the forward solve
  __shared__ double Db[FB * (FB + 1)];  // tile (0, 0): the next diagonal block, updated, by column
  const int n = d.nF, s0 = k0 + FB, nr = n - s0;
  const int T = (nr + FT - 1) / FT, ntile = T * (T + 1) / 2;
  const int ti = (int)blockIdx.x, tid = (int)threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
  double* F = d.F;
  if (ti == ntile) {  // the panel's diagonal block inverse, for the solves
    if (wv == 0) front_inverse(F, n, k0, lane, d.Frd + k0, d.Finv + (size_t)(k0 / FB) * FB * FB, Ls);
    return;
  }
  int I = (int)((sqrtf(8.0f * (float)ti + 1.0f) - 1.0f) * 0.5f);
  I -= (I * (I + 1) / 2 > ti) ? 1 : 0;
  I += ((I + 1) * (I + 2) / 2 <= ti) ? 1 : 0;
  const int J = ti - I * (I + 1) / 2;
  const bool fwd = J == 0 && wv == 1;  // this wavefront carries the forward solve through the panel
  const int nb = min(FT, nr - FT * I);
  double yk = 0.0, yi = 0.0;
  if (fwd) {  // y of the panel's block and of tile row I, read early (their latency overlaps the loads below)
    if (lane < FB) yk = d.yF[k0 + lane];
    if (lane < nb) yi = d.yF[s0 + FT * I + lane];
  }
  // this wavefront's quadrant of the tile (row half qi, column half qj), read now:
  // its latency overlaps the panel's loads and solve
  const int qi = wv & 1, qj = wv >> 1;
  d4 acc[2][2];
  bool live[2][2];
#pragma unroll
  for (int cj = 0; cj < 2; ++cj)
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const int ib = FT * I + 32 * qi + 16 * ri, jb = FT * J + 32 * qj + 16 * cj;
      live[cj][ri] = ib < nr && jb < nr && (I != J || ib >= jb);
      const double* src = live[cj][ri] ? F + (size_t)(s0 + jb + l4) * n + s0 + ib + l16 : F;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cj][ri][v] = src[live[cj][ri] ? (size_t)(4 * v) * n : 0];
    }
  {  // every load issued before any is used (rows past the front's end read the next
     // column's top, in bounds since the panel is not the last, and are zeroed)
    constexpr int NL = FB * FB / FRONT_TWG, NP = FB * FT / FRONT_TWG;
    double vl[NL], va[NP], vb[NP];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int x = tid + u * FRONT_TWG, c = x / FB, i = x % FB;
      vl[u] = F[(size_t)(k0 + c) * n + k0 + i];
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int x = tid + u * FRONT_TWG, k = x / FT, i = x % FT;
      va[u] = F[(size_t)(k0 + k) * n + s0 + FT * J + i];
      vb[u] = F[(size_t)(k0 + k) * n + s0 + FT * I + i];
    }
    const double rv = tid < FB ? d.Frd[k0 + tid] : 0.0;
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int x = tid + u * FRONT_TWG, c = x / FB, i = x % FB;
      Ls[c * (FB + 1) + i] = i > c ? vl[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int x = tid + u * FRONT_TWG, i = x % FT;
      Pa[x] = FT * J + i < nr ? va[u] : 0.0;
      Pb[x] = FT * I + i < nr ? vb[u] : 0.0;
    }
    if (tid < FB) rds[tid] = rv;
  }
  static_assert(FB * FB % FRONT_TWG == 0 && FB * FT % FRONT_TWG == 0, "whole rounds of loads");
  __syncthreads();
  const int na = min(FT, nr - FT * J);
  if (tid < FT) front_solve_rows(Pa, na, tid, Ls, rds);
  else if (tid < 2 * FT && I != J) front_solve_rows(Pb, nb, tid - FT, Ls, rds);
  __syncthreads();
  if (I == J) {  // one buffer serves both sides
    for (int x = tid; x < FB * FT; x += FRONT_TWG) Pb[x] = Pa[x];
    __syncthreads();
  }
  if (J == 0) {  // row block I of the panel, final
    for (int x = tid; x < FB * FT; x += FRONT_TWG) {
      const int k = x / FT, i = x % FT;
      if (i < nb) F[(size_t)(k0 + k) * n + s0 + FT * I + i] = Pb[x];
    }
  }
#pragma unroll
  for (int k = 0; k < FB; k += 4) {
    double pa[2], pb[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      pa[q] = -Pa[(k + l4) * FT + 32 * qj + 16 * q + l16];
      pb[q] = Pb[(k + l4) * FT + 32 * qi + 16 * q + l16];
    }
#pragma unroll
    for (int cj = 0; cj < 2; ++cj)
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
        if (live[cj][ri]) acc[cj][ri] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[cj], pb[ri], acc[cj][ri], 0, 0, 0);
  }
  const bool next_diag = ti == 0 && wv == 0;  // quadrant (0, 0) of tile (0, 0): the next diagonal block
#pragma unroll
  for (int cj = 0; cj < 2; ++cj)
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      if (!live[cj][ri]) continue;
      const int ib = FT * I + 32 * qi + 16 * ri, jb = FT * J + 32 * qj + 16 * cj;
      if (next_diag) {  // to LDS for the factor, which writes the block to F
#pragma unroll
        for (int v = 0; v < 4; ++v) Db[(jb + l4 + 4 * v) * (FB + 1) + ib + l16] = acc[cj][ri][v];
        continue;
      }
      double* dst = F + (size_t)(s0 + jb + l4) * n + s0 + ib + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (ib != jb || ib + l16 >= jb + l4 + 4 * v) dst[(size_t)(4 * v) * n] = acc[cj][ri][v];
    }
  if (next_diag) {
    wave_sync();
    if (!front_factor(Db, FB + 1, F, n, s0, lane, d.Frd + s0) && lane == 0) *d.status = 2;
  }
  if (fwd) {  // forward solve through the panel: z_k, then tile row I's y_i -= L_ik z_k
    const double v = front_subst(yk, Ls, rds, lane);
    if (lane < FB) {
      zs[lane] = v;
      if (I == 0) d.zF[k0 + lane] = v;
    }
    wave_sync();
    if (lane < nb) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < FB; ++k) t += Pb[k * FT + lane] * zs[k];
      d.yF[s0 + FT * I + lane] = yi - t;
    }
  }
}

// Products of one solve level kept in LDS at a time.
constexpr int SOLVE_CHUNK = 512;
// Sparse columns whose solution is kept in LDS during the backward solve.
constexpr int XS_MAX = 1536;
// Sparse levels whose ranges are kept in LDS during the backward solve.
constexpr int LV_MAX = 512;
static_assert(SOLVE_CHUNK >= FIN_WG, "one product per thread in a level's first round");

// Barrier that orders LDS only: the global loads in flight (the next level's
// factor data) are not waited for.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// x of a row block's node for the backward solve: the front's part from ys, the
// sparse columns' from xs when it is kept there, else from g.
__device__ inline const double* bs_x(const PgoDev& d, int row, const double* xs, const double* ys) {
  if (row >= d.p0 && d.K > 0) return ys + 7 * (row - d.p0);
  return xs ? xs + 7 * row : d.g + 7 * row;
}

// One level of the backward solve L^T x = y over the sparse columns, the general
// form (any number of blocks and columns): x_c = L_cc^{-T} (y_c - sum_i L_ic^T x_i)
// over column c's blocks. Every block product of the level is formed in parallel
// (one thread per block, into LDS), then one thread per column sums its own
// products in list order. The solution goes to xs when given (else to g).
__device__ inline void solve_level_bwd(const PgoDev& d, int l, double* prod, double* xs, const double* ys) {
  const int tid = threadIdx.x;
  const int j0 = d.flev_ptr[l], j1 = d.flev_ptr[l + 1];
  for (int jb = j0; jb < j1; jb += FIN_WG) {
    const int j = jb + tid;
    const bool own = j < j1;
    const int c = own ? d.flev_col[j] : 0;
    const int p_lo = own ? d.bs_ptr[j] : 0, p_hi = own ? d.bs_ptr[j + 1] : 0;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    const int q_lo = d.bs_ptr[jb], q_hi = d.bs_ptr[min(jb + FIN_WG, j1)];
    for (int base = q_lo; base < q_hi; base += SOLVE_CHUNK) {
      const int top = min(base + SOLVE_CHUNK, q_hi);
      for (int q = base + tid; q < top; q += FIN_WG) {
        const double* L = d.Lb + 49 * d.bs_blk[q];
        const double* x = bs_x(d, d.bs_row[q], xs, ys);
        double xv[7];
#pragma unroll
        for (int u = 0; u < 7; ++u) xv[u] = x[u];
#pragma unroll
        for (int r = 0; r < 7; ++r) {
          double t = 0.0;
#pragma unroll
          for (int u = 0; u < 7; ++u) t += L[7 * u + r] * xv[u];
          prod[7 * (q - base) + r] = t;
        }
      }
      __syncthreads();
      for (int q = max(p_lo, base); q < min(p_hi, top); ++q)
#pragma unroll
        for (int r = 0; r < 7; ++r) acc[r] += prod[7 * (q - base) + r];
      __syncthreads();
    }
    if (own) {
      const double* Di = d.Di + 49 * c;
      double* y = d.g + 7 * c;
      double v[7];
#pragma unroll
      for (int r = 0; r < 7; ++r) v[r] = y[r] - acc[r];
      double* xo = xs ? xs + 7 * c : y;
#pragma unroll
      for (int r = 0; r < 7; ++r) {
        double t = 0.0;
#pragma unroll
        for (int k = r; k < 7; ++k) t += Di[7 * k + r] * v[k];
        xo[r] = t;
      }
    }
  }
  __syncthreads();
}

// What thread t reads of a level of the backward solve in its first round: the
// node of block Q0 + t's row (ok when the block exists), the column at schedule
// position j0 + t (c and its blocks' range relative to Q0; ok when it exists), and
// from the level's element-major copy of the factor the block's L, the lower
// triangle of L_cc^{-1} by rows and y_c (coalesced: lane t reads entry t of each
// element; whole wavefronts past the level's end read none). Indices past the
// level's end are clamped to its last entry. None of it depends on the solution:
// a level's share is loaded while the level before it runs, its indices one level
// earlier still.
struct BsIdx {
  int row, c, pl, ph;
  bool bok, cok;
};
struct BsData {
  double L[49], Di[28], y[7];
};

// A level with few columns takes one wavefront per column (its lanes share the
// column's sums), others one thread per column.
constexpr int BS_WIDE = FIN_WG / 64;
__device__ inline bool bs_wide(const int* lv, int l) { return lv[LVW * l + 1] - lv[LVW * l] <= BS_WIDE; }

// lv: the level table (LVW entries per level)
__device__ inline void bs_fetch_idx(const PgoDev& d, const int* lv, int l, int t, BsIdx& s) {
  const int* e = lv + LVW * l;
  const int j0 = e[0], j1 = e[1], Q0 = e[2], Q1 = e[3];
  const int q = Q0 + t, j = j0 + (bs_wide(lv, l) ? t >> 6 : t);
  const int qc = max(min(q, Q1 - 1), 0), jc = min(j, j1 - 1);
  s.row = d.bs_row[qc];
  s.c = d.flev_col[jc];
  s.pl = d.bs_ptr[jc] - Q0;
  s.ph = d.bs_ptr[jc + 1] - Q0;
  s.bok = q < Q1;
  s.cok = j < j1;
}

// the level's entries are uniform: the element addresses are formed in scalar
// registers, and each lane adds only its own offset
__device__ inline void bs_fetch_L(const PgoDev& d, const int* lv, int l, int t, BsData& x) {
  const int* e = lv + LVW * l;
  const int NQ = __builtin_amdgcn_readfirstlane(e[6]);
  const int w0 = __builtin_amdgcn_readfirstlane(t & ~63), lane = t & 63;
  if (w0 < NQ) {
    const double* L = d.bw + __builtin_amdgcn_readfirstlane(e[4]) + w0;
#pragma unroll
    for (int k = 0; k < 49; ++k) x.L[k] = L[(size_t)k * NQ + lane];
  } else {
#pragma unroll
    for (int k = 0; k < 49; ++k) x.L[k] = 0.0;
  }
}

__device__ inline void bs_fetch_col(const PgoDev& d, const int* lv, int l, int t, BsData& x) {
  const int* e = lv + LVW * l;
  const int NJ = __builtin_amdgcn_readfirstlane(e[7]);
  const bool wide = bs_wide(lv, l);
  const int w0 = __builtin_amdgcn_readfirstlane(t & ~63), lane = t & 63;
  // the column of this thread: its wavefront's (every lane the same) or its own
  const int base = wide ? w0 >> 6 : w0, off = wide ? 0 : lane;
  if ((wide ? (w0 >> 6) < e[1] - e[0] : w0 < NJ)) {
    const double* C = d.bw + __builtin_amdgcn_readfirstlane(e[5]) + base;
#pragma unroll
    for (int k = 0; k < 28; ++k) x.Di[k] = C[(size_t)k * NJ + off];
#pragma unroll
    for (int r = 0; r < 7; ++r) x.y[r] = C[(size_t)(28 + r) * NJ + off];
  } else {
#pragma unroll
    for (int k = 0; k < 28; ++k) x.Di[k] = 0.0;
#pragma unroll
    for (int r = 0; r < 7; ++r) x.y[r] = 0.0;
  }
}

// Workgroups of the solves launch besides the one that solves: those that land on
// its XCD (workgroups are handed to the XCDs in turn) read what it is about to read
// (the front's lower triangle and block inverses, the sparse part's backward copy),
// written from every XCD, into that XCD's L2 while it starts.
constexpr int FIN_HELPERS = 31;

// Reads this helper's share of [p, p + n) doubles (share h of nh), 16 B per lane,
// eight loads in flight per lane; the result depends on every load.
__device__ inline unsigned warm_range(const double* p, size_t n, int h, int nh) {
  const double2* q = reinterpret_cast<const double2*>(p);
  const size_t n2 = n / 2, lo = n2 * h / nh, hi = n2 * (h + 1) / nh;
  unsigned keep = 0;
  for (size_t i = lo + threadIdx.x; i < hi; i += 8 * FIN_WG) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = i + (size_t)u * FIN_WG < hi ? q[i + (size_t)u * FIN_WG] : double2{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 8; ++u) keep += (unsigned)__double_as_longlong(v[u].x);
  }
  return keep;
}

// The two triangular solves and the update T <- Exp(dx) T, by one workgroup:
// forward and backward through the factored front (its part of the vector in
// LDS), then backward over the sparse columns from the root. A level with at
// most one block and one column per thread runs from data loaded during the
// level before, its solution kept in LDS (the barriers between its phases then
// order LDS only); larger levels, or sparse parts too large for LDS, take the
// general form.
__global__ __launch_bounds__(FIN_WG) void k_pgo_finish(PgoDev d, s3a_sim3* T, double lambda, int lm) {
  __shared__ double sh[FIN_WG / 64 + 1];
  __shared__ double ys[FRONT_MAX];
  __shared__ double red[FB];
  __shared__ double prod[7 * SOLVE_CHUNK];
  __shared__ double xs_lds[7 * XS_MAX];
  __shared__ int lv[LVW * LV_MAX];
  const int tid = threadIdx.x;
  if (*d.status != 0) return;
  if (blockIdx.x != 0) {
    if (blockIdx.x % 8 == 0) {  // a helper on the solving workgroup's XCD
      const int h = blockIdx.x / 8 - 1;
      unsigned keep = 0;
      if (d.K > 0) {
        // the front's lower triangle, a column's part below its diagonal at a time
        const int n = d.nF;
        for (int c0 = h * 8; c0 < n; c0 += 8 * FIN_HELPERS) {
          double2 v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int c = c0 + u, r2 = c / 2 + (int)threadIdx.x;
            v[u] = c < n && r2 < n / 2 ? reinterpret_cast<const double2*>(d.F + (size_t)c * n)[r2] : double2{0.0, 0.0};
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) keep += (unsigned)__double_as_longlong(v[u].x);
        }
        keep += warm_range(d.Finv, (size_t)n * FB, h, FIN_HELPERS);
      }
      if (d.bw) keep += warm_range(d.bw, (size_t)d.bw_size, h, FIN_HELPERS);
      if (keep == 1u) sh[0] = 0.0;  // keeps the loads; this workgroup's own LDS, never read
    }
    return;
  }
  const bool lv_on = d.bw && d.nflev <= LV_MAX;
  if (lv_on)
    for (int x = tid; x < LVW * d.nflev; x += FIN_WG) lv[x] = d.lv[x];  // read after the front's barriers
  // (the forward solve over the sparse columns ran with their factorisation, k_pgo_level_factor)
  if (d.K > 0) {
    const int n = d.nF, nK = 7 * d.K;
    // ---- the front's forward solve (done panel by panel with its factorisation), into LDS
    for (int x = tid; x < n; x += FIN_WG) ys[x] = d.zF[x];
    __syncthreads();
    // ---- its last diagonal block, forward and backward by substitution (one wavefront,
    // the block by column in prod, 1 / L_jj in red): z = L^{-1} y, then x = L^{-T} z
    const int kl = n - FB;
    if (tid < 64) {
      const int lane = tid;
      double* lt = prod;
      for (int x = lane; x < FB * FB; x += 64) {
        const int c = x / FB, i = x % FB;
        lt[c * (FB + 1) + i] = i > c ? d.F[(size_t)(kl + c) * n + kl + i] : 0.0;
      }
      if (lane < FB) red[lane] = d.Frd[kl + lane];
      wave_sync();
      double v = front_subst(lane < FB ? d.yF[kl + lane] : 0.0, lt, red, lane);
#pragma unroll
      for (int k = FB - 1; k >= 0; --k) {
        const double xk = readlane_f64(v, k) * red[k];
        if (lane < k) v -= lt[lane * (FB + 1) + k] * xk;
        v = lane == k ? xk : v;
      }
      if (lane < FB) ys[kl + lane] = v;
    }
    __syncthreads();
    // ---- backward through the front: x_blk = L_blk^{-T} (y_blk - sum of L_ib^T x_i below)
    for (int k0 = kl - FB; k0 >= 0; k0 -= FB) {
      {
        constexpr int SL = FIN_WG / FB;  // row slots per column
        const int c = tid / SL, q = tid % SL;
        double t = 0.0;
        for (int i = k0 + FB + q; i < n; i += SL) t += d.F[(size_t)(k0 + c) * n + i] * ys[i];
#pragma unroll
        for (int o = SL / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (q == 0) red[c] = t;
      }
      __syncthreads();
      if (tid < FB) {
        const double* Vi = d.Finv + (size_t)(k0 / FB) * FB * FB;
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < FB; ++r) t += Vi[r * FB + tid] * (ys[k0 + r] - red[r]);
        wave_sync();  // the other lanes' reads of ys before this write
        ys[k0 + tid] = t;
      }
      __syncthreads();
    }
    for (int x = tid; x < nK; x += FIN_WG) d.g[7 * d.p0 + x] = ys[x];
    __syncthreads();
  }
  // ---- backward solve L^T x = y over the sparse columns, levels from the root
  double* xs = d.p0 <= XS_MAX ? xs_lds : nullptr;
  if (d.K == 0) __syncthreads();  // lv (the front's barriers order it otherwise)
  auto fast = [&](int l) {
    return lv_on && xs && lv[LVW * l + 1] - lv[LVW * l] <= FIN_WG && lv[LVW * l + 3] - lv[LVW * l + 2] <= FIN_WG;
  };
  for (int l = d.nflev - 1; l >= 0;) {
    if (!fast(l)) {
      solve_level_bwd(d, l, prod, xs, ys);
      --l;
      continue;
    }
    // a run of levels that each fit in one round. Two sets of indices take turns
    // (the loop runs two levels per turn), so that the next level's set is never
    // copied: a copy would wait for its loads and, the counter of loads in flight
    // being in order, for the blocks loaded after them.
    BsIdx ia, ib;
    BsData sd;
    bs_fetch_idx(d, lv, l, tid, ia);
    bs_fetch_L(d, lv, l, tid, sd);
    bs_fetch_col(d, lv, l, tid, sd);
    if (l > 0 && fast(l - 1)) bs_fetch_idx(d, lv, l - 1, tid, ib);
    // one level from cur (its indices), with nxt holding the next level's; cur takes
    // the indices of the level after next. False when the run ends with this level.
    auto level = [&](int lc, BsIdx& cur) -> bool {
      // block phase: this thread's block product L^T x_row
      if (cur.bok) {
        const double* x = bs_x(d, cur.row, xs, ys);
        double xv[7];
#pragma unroll
        for (int u = 0; u < 7; ++u) xv[u] = x[u];
#pragma unroll
        for (int r = 0; r < 7; ++r) {
          double t = 0.0;
#pragma unroll
          for (int u = 0; u < 7; ++u) t += sd.L[7 * u + r] * xv[u];
          prod[7 * tid + r] = t;
        }
      }
      const bool more = lc > 0 && fast(lc - 1);
      if (more) {  // the next level's blocks (L is free once the products are formed)
        __builtin_amdgcn_sched_barrier(0);
        bs_fetch_L(d, lv, lc - 1, tid, sd);
      }
      lds_barrier();
      // column phase: x_c = L_cc^{-T} (y_c - sum of the column's products). One thread
      // per column sums in list order, three blocks' products read at a time; with
      // few columns a wavefront per column sums lane-strided partials and reduces
      // them with the fixed DPP tree.
      const bool wide = bs_wide(lv, lc);
      if (cur.cok) {
        double acc[7] = {0, 0, 0, 0, 0, 0, 0};
        if (wide) {
          for (int q = cur.pl + (tid & 63); q < cur.ph; q += 64)
#pragma unroll
            for (int r = 0; r < 7; ++r) acc[r] += prod[7 * q + r];
          wave_totals_f64(acc);
        } else {
          int q = cur.pl;
          for (; q + 3 <= cur.ph; q += 3) {
            double pv[3][7];
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
              for (int r = 0; r < 7; ++r) pv[u][r] = prod[7 * (q + u) + r];
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
              for (int r = 0; r < 7; ++r) acc[r] += pv[u][r];
          }
          for (; q < cur.ph; ++q)
#pragma unroll
            for (int r = 0; r < 7; ++r) acc[r] += prod[7 * q + r];
        }
        double v[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) v[r] = sd.y[r] - acc[r];
        if (!wide || (tid & 63) == 0) {
          double* xo = xs + 7 * cur.c;
#pragma unroll
          for (int r = 0; r < 7; ++r) {
            double t = 0.0;
#pragma unroll
            for (int k = r; k < 7; ++k) t += sd.Di[k * (k + 1) / 2 + r] * v[k];
            xo[r] = t;
          }
        }
      }
      if (more) {  // the next level's diagonal blocks and y, then the indices of the one after it
        __builtin_amdgcn_sched_barrier(0);
        bs_fetch_col(d, lv, lc - 1, tid, sd);
        if (lc > 1 && fast(lc - 2)) bs_fetch_idx(d, lv, lc - 2, tid, cur);
      }
      lds_barrier();
      return more;
    };
    for (;;) {
      if (!level(l--, ia)) break;
      if (!level(l--, ib)) break;
    }
  }
  __syncthreads();
  if (xs) {
    for (int x = tid; x < 7 * d.p0; x += FIN_WG) d.g[x] = xs[x];
    __syncthreads();
  }
  // ---- LM: reduction the quadratic model predicts, dx^T (lambda D dx - g) / 2 (fixed order)
  if (lm) {
    double part2 = 0.0;
    for (int x = tid; x < d.m * 7; x += FIN_WG) part2 += d.g[x] * (lambda * d.dsave[x] * d.g[x] + d.gsave[x]);
    const double pr = wg_sum<FIN_WG>(part2, sh);
    if (tid == 0) d.pred[0] = 0.5 * pr;
  }
  // ---- update T <- Exp(dx) T for the free nodes
  for (int c = tid; c < d.m; c += FIN_WG) {
    const int nd = d.node[c];
    const Sim3d E = sim3_exp(d.g + 7 * c);
    store_sim3(T + nd, sim3_compose(E, ld_pose(T + nd)));
  }
}

// ------------------------------------------------------------------ host

struct PgoWorkspace {
  int32_t n_nodes = -1, n_edges = -1, gauge = -1;
  std::vector<int32_t> flev, ct;  // host copies of the sparse levels' column and target ranges (launch sizes)
  std::vector<int32_t> lvh;       // host copy of the level table
  std::vector<int32_t> ij;  // topology the symbolic analysis was made for
  void* buf = nullptr;
  PgoDev dev{};
  int32_t cap_iters = 0;
  int64_t nnz_blocks = 0;
  // Levenberg-Marquardt: a second linearisation (the trial's) and the poses before a trial
  double* M_alt = nullptr;
  double* v_alt = nullptr;
  double* r2_alt = nullptr;
  s3a_sim3* T_bak = nullptr;
};

namespace {

struct Symbolic {
  int m = 0, nblk = 0, nlev = 0, nflev = 0, K = 0, p0 = 0, nF = 0;
  bool bw_on = false;
  int64_t bw_size = 0;
  std::vector<int32_t> pos, node, col_ptr, blk_row, blk_col, dg_ptr, dg_edge, ob_ptr, ob_edge, gv_ptr, gv_edge,
      up_ptr, up_a, up_b, lev_ptr, lev_col, flev_ptr, flev_col, lt_tgt, row_ptr, row_blk,
      chain, chain_lev, dt_tgt, dt_ptr, dup_a, dup_b, fs_ptr, fs_blk, bs_ptr, bs_blk, fu_ptr, fu_a, fu_b, ct_ptr,
      fz_rc, bs_row, lv;
  std::vector<int8_t> gv_sign;
};

// Minimum degree (smallest current degree, ties by node id) on the free nodes,
// by explicit elimination of the node graph.
std::vector<int32_t> min_degree(int n, int gauge, const std::vector<std::set<int>>& adj0) {
  std::vector<std::set<int>> adj(adj0);
  std::set<std::pair<int, int>> pq;
  std::vector<char> done(n, 0);
  for (int v = 0; v < n; ++v)
    if (v != gauge) pq.insert({(int)adj[v].size(), v});
  std::vector<int32_t> order;
  while (!pq.empty()) {
    const int v = pq.begin()->second;
    pq.erase(pq.begin());
    done[v] = 1;
    order.push_back(v);
    std::vector<int> nb(adj[v].begin(), adj[v].end());
    for (int a : nb) {
      pq.erase({(int)adj[a].size(), a});
      adj[a].erase(v);
      for (int b : nb)
        if (b != a) adj[a].insert(b);
      pq.insert({(int)adj[a].size(), a});
    }
    adj[v].clear();
  }
  return order;
}

Symbolic analyse(int n, int E, const int32_t* ij, int gauge) {
  Symbolic S;
  std::vector<std::set<int>> adj(n);
  for (int k = 0; k < E; ++k) {
    const int i = ij[2 * k], j = ij[2 * k + 1];
    if (i != gauge && j != gauge) {
      adj[i].insert(j);
      adj[j].insert(i);
    }
  }
  const std::vector<int32_t> order = min_degree(n, gauge, adj);
  const int m = (int)order.size();
  S.m = m;
  S.pos.assign(n, -1);
  S.node = order;
  for (int c = 0; c < m; ++c) S.pos[order[c]] = c;
  // symbolic factorisation: struct(c) = rows > c, merged into the parent
  std::vector<std::set<int>> cs(m);
  for (int k = 0; k < E; ++k) {
    const int a = S.pos[ij[2 * k]], b = S.pos[ij[2 * k + 1]];
    if (a < 0 || b < 0) continue;
    cs[std::min(a, b)].insert(std::max(a, b));
  }
  std::vector<int> parent(m, -1);
  for (int c = 0; c < m; ++c) {
    if (cs[c].empty()) continue;
    const int p = *cs[c].begin();
    parent[c] = p;
    for (int r : cs[c])
      if (r != p) cs[p].insert(r);
  }
  S.col_ptr.assign(m + 1, 0);
  for (int c = 0; c < m; ++c) S.col_ptr[c + 1] = S.col_ptr[c] + (int)cs[c].size();
  S.nblk = S.col_ptr[m];
  S.blk_row.resize(S.nblk);
  S.blk_col.resize(S.nblk);
  std::vector<std::vector<std::pair<int, int>>> colrows(m);  // (row, block)
  for (int c = 0; c < m; ++c) {
    int b = S.col_ptr[c];
    for (int r : cs[c]) {
      S.blk_row[b] = r;
      S.blk_col[b] = c;
      colrows[c].push_back({r, b});
      ++b;
    }
  }
  auto block_of = [&](int r, int c) -> int {  // r > c
    auto& v = colrows[c];
    auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(r, -1));
    return (it != v.end() && it->first == r) ? it->second : -1;
  };
  // assembly lists
  std::vector<std::vector<int>> dg(m), ob(S.nblk), gv(m);
  std::vector<std::vector<int8_t>> gs(m);
  for (int k = 0; k < E; ++k) {
    const int a = S.pos[ij[2 * k]], b = S.pos[ij[2 * k + 1]];
    if (a >= 0) { dg[a].push_back(k); gv[a].push_back(k); gs[a].push_back(-1); }
    if (b >= 0) { dg[b].push_back(k); gv[b].push_back(k); gs[b].push_back(+1); }
    if (a >= 0 && b >= 0) ob[block_of(std::max(a, b), std::min(a, b))].push_back(k);
  }
  auto flatten = [](const std::vector<std::vector<int>>& L, std::vector<int32_t>& ptr, std::vector<int32_t>& val) {
    ptr.assign(L.size() + 1, 0);
    for (size_t i = 0; i < L.size(); ++i) ptr[i + 1] = ptr[i] + (int)L[i].size();
    val.clear();
    for (auto& v : L) val.insert(val.end(), v.begin(), v.end());
  };
  flatten(dg, S.dg_ptr, S.dg_edge);
  flatten(ob, S.ob_ptr, S.ob_edge);
  flatten(gv, S.gv_ptr, S.gv_edge);
  for (auto& v : gs) S.gv_sign.insert(S.gv_sign.end(), v.begin(), v.end());
  // update lists: column k contributes L(a,k) L(b,k)^T to target (a, b), a >= b
  std::vector<std::vector<std::pair<int, int>>> up(m + S.nblk);
  for (int k = 0; k < m; ++k) {
    const auto& rows = colrows[k];
    for (size_t x = 0; x < rows.size(); ++x)
      for (size_t y = 0; y <= x; ++y) {
        const int ra = rows[x].first, rb = rows[y].first;  // ra >= rb
        const int t = (ra == rb) ? ra : S.m + block_of(ra, rb);
        up[t].push_back({rows[x].second, rows[y].second});
      }
  }
  S.up_ptr.assign(m + S.nblk + 1, 0);
  for (size_t t = 0; t < up.size(); ++t) S.up_ptr[t + 1] = S.up_ptr[t] + (int)up[t].size();
  for (auto& v : up)
    for (auto& p : v) { S.up_a.push_back(p.first); S.up_b.push_back(p.second); }
  // levels from the leaves
  std::vector<int> lev(m, 0);
  int nlev = 0;
  for (int c = 0; c < m; ++c) {
    if (parent[c] >= 0) lev[parent[c]] = std::max(lev[parent[c]], lev[c] + 1);
    nlev = std::max(nlev, lev[c] + 1);
  }
  S.nlev = nlev;
  S.lev_ptr.assign(nlev + 1, 0);
  for (int c = 0; c < m; ++c) S.lev_ptr[lev[c] + 1]++;
  for (int l = 0; l < nlev; ++l) S.lev_ptr[l + 1] += S.lev_ptr[l];
  S.lev_col.resize(m);
  std::vector<int> fill(S.lev_ptr.begin(), S.lev_ptr.end() - 1);
  for (int c = 0; c < m; ++c) S.lev_col[fill[lev[c]]++] = c;
  // dense trailing clique: the last K columns each hold every row below them
  int K = 0;
  for (int c = m - 1; c >= 0 && (int)cs[c].size() == m - 1 - c; --c) ++K;
  if (K < 8) K = 0;
  if (K > PGO_KMAX) K = PGO_KMAX;  // the last PGO_KMAX columns of a larger clique are one too
  // The columns just before the clique join the front while they fit in its identity
  // padding: the dense factor costs the same, and each one taken off the sparse
  // schedule can shorten it by a level. Their rows all lie below them, so in the
  // front; the blocks their structure lacks are exact zeros of L too (the symbolic
  // factor is closed under elimination) and are rewritten as zeros every iteration.
  if (K > 0) {
    const int nF0 = (7 * K + FT - 1) / FT * FT;
    while (K < m && K < PGO_KMAX && 7 * (K + 1) <= nF0) ++K;
  }
  const int p0 = m - K;
  S.K = K;
  S.p0 = p0;
  S.nF = K > 0 ? (7 * K + FT - 1) / FT * FT : 0;
  for (int c = p0; c < m; ++c) {  // the front's lower blocks outside the structure
    int r = c + 1;
    for (int x : cs[c]) {
      for (; r < x; ++r) S.fz_rc.insert(S.fz_rc.end(), {r - p0, c - p0});
      r = x + 1;
    }
    for (; r < m; ++r) S.fz_rc.insert(S.fz_rc.end(), {r - p0, c - p0});
  }
  // schedule of the sparse columns (levels without one are dropped)
  S.flev_ptr.assign(1, 0);
  S.ct_ptr.assign(1, 0);
  for (int l = 0; l < nlev; ++l) {
    bool any = false;
    for (int q = S.lev_ptr[l]; q < S.lev_ptr[l + 1]; ++q) {
      const int c = S.lev_col[q];
      if (c >= p0) continue;
      any = true;
      S.flev_col.push_back(c);
      auto has_updates = [&](int t) { return S.up_ptr[t + 1] > S.up_ptr[t]; };  // others keep their assembled value
      if (has_updates(c)) S.lt_tgt.push_back(c);
      for (int b = S.col_ptr[c]; b < S.col_ptr[c + 1]; ++b) {
        if (has_updates(m + b)) S.lt_tgt.push_back(m + b);
      }
      S.ct_ptr.push_back((int32_t)S.lt_tgt.size());
    }
    if (!any) continue;
    S.flev_ptr.push_back((int32_t)S.flev_col.size());
  }
  S.nflev = (int)S.flev_ptr.size() - 1;
  // the front: block map, and each of its targets' updates from sparse columns
  S.dt_ptr.assign(1, 0);
  for (int c = p0; c < m; ++c) {
    std::vector<int> tg{c};
    for (int b = S.col_ptr[c]; b < S.col_ptr[c + 1]; ++b) tg.push_back(m + b);
    for (int t : tg) {
      S.dt_tgt.push_back(t);
      for (int q = S.up_ptr[t]; q < S.up_ptr[t + 1]; ++q)
        if (S.blk_col[S.up_a[q]] < p0) {
          S.dup_a.push_back(S.up_a[q]);
          S.dup_b.push_back(S.up_b[q]);
        }
      S.dt_ptr.push_back((int32_t)S.dup_a.size());
    }
  }
  // rows of L (blocks (c, k), k < c) for the forward solve
  std::vector<std::vector<int>> rows(m);
  for (int b = 0; b < S.nblk; ++b) rows[S.blk_row[b]].push_back(b);
  flatten(rows, S.row_ptr, S.row_blk);
  // the update pairs of the sparse columns' targets, in schedule order
  S.fu_ptr.assign(1, 0);
  for (int t : S.lt_tgt) {
    for (int q = S.up_ptr[t]; q < S.up_ptr[t + 1]; ++q) {
      S.fu_a.push_back(S.up_a[q]);
      S.fu_b.push_back(S.up_b[q]);
    }
    S.fu_ptr.push_back((int32_t)S.fu_a.size());
  }
  // the sparse columns' row and column blocks in schedule order, for the solves
  S.fs_ptr.assign(1, 0);
  S.bs_ptr.assign(1, 0);
  for (int c : S.flev_col) {
    S.fs_blk.insert(S.fs_blk.end(), rows[c].begin(), rows[c].end());
    S.fs_ptr.push_back((int32_t)S.fs_blk.size());
    for (int b = S.col_ptr[c]; b < S.col_ptr[c + 1]; ++b) {
      S.bs_blk.push_back(b);
      S.bs_row.push_back(S.blk_row[b]);
    }
    S.bs_ptr.push_back((int32_t)S.bs_blk.size());
  }
  // level table; the backward solve's element-major copy of the factor is kept when
  // the sparse part's solution and the table fit in the solve's LDS
  S.bw_on = S.p0 <= XS_MAX && S.nflev <= LV_MAX;
  int64_t off = 0;
  for (int l = 0; l < S.nflev; ++l) {
    const int j0 = S.flev_ptr[l], j1 = S.flev_ptr[l + 1];
    const int Q0 = S.bs_ptr[j0], Q1 = S.bs_ptr[j1];
    const int NQ = (Q1 - Q0 + 63) / 64 * 64, NJ = (j1 - j0 + 63) / 64 * 64;
    const int lb = (int)off, dc = (int)(off + 49 * (int64_t)NQ);
    if (S.bw_on) off += 49 * (int64_t)NQ + 35 * (int64_t)NJ;
    S.lv.insert(S.lv.end(), {j0, j1, Q0, Q1, S.bw_on ? lb : 0, S.bw_on ? dc : 0, NQ, NJ});
  }
  S.bw_size = off;
  S.bs_blk.push_back(0);  // a valid block and node past the end: the solve's clamped reads
  S.bs_row.push_back(0);
  // chaining order (breadth-first from the gauge over edges in input order)
  std::vector<std::vector<int>> inc(n);
  for (int k = 0; k < E; ++k) {
    inc[ij[2 * k]].push_back(k);
    inc[ij[2 * k + 1]].push_back(k);
  }
  std::vector<char> placed(n, 0);
  std::vector<int> depth(n, 0);
  placed[gauge] = 1;
  std::deque<int> q{gauge};
  while (!q.empty()) {
    const int a = q.front();
    q.pop_front();
    for (int k : inc[a]) {
      const int i = ij[2 * k], j = ij[2 * k + 1];
      if (i == a && !placed[j]) {
        placed[j] = 1;
        depth[j] = depth[a] + 1;
        S.chain.insert(S.chain.end(), {j, i, k, 0});
        q.push_back(j);
      } else if (j == a && !placed[i]) {
        placed[i] = 1;
        depth[i] = depth[a] + 1;
        S.chain.insert(S.chain.end(), {i, j, k, 1});
        q.push_back(i);
      }
    }
  }
  // breadth-first order is nondecreasing in depth: level boundaries of the chain
  S.chain_lev.assign(1, 0);
  for (size_t c = 0; c < S.chain.size() / 4; ++c) {
    const int dep = depth[S.chain[4 * c]];
    while ((int)S.chain_lev.size() < dep) S.chain_lev.push_back((int32_t)c);
  }
  S.chain_lev.push_back((int32_t)(S.chain.size() / 4));
  return S;
}

template <typename T>
T* carve(char*& p, size_t n) {
  T* r = reinterpret_cast<T*>(p);
  p += ((n * sizeof(T)) + 255) & ~size_t(255);
  return r;
}

template <typename T>
size_t bytes_of(size_t n) {
  return ((n * sizeof(T)) + 255) & ~size_t(255);
}

int fail(int* last_hip, hipError_t e) {
  if (last_hip) *last_hip = (int)e;
  return e == hipErrorOutOfMemory ? S3A_ENOMEM : S3A_EHIP;
}

}  // namespace

namespace {

// One damped solve and update of the poses (or, without update, only chi^2 at the
// current linearisation): assembly across the chip, the sparse factorisation and
// forward solve level by level across the chip, the front's sparse-column updates
// and right-hand side across the chip, the front and its forward solve one panel
// per launch, then the backward solves and the update in one workgroup.
hipError_t launch_iteration(const PgoDev& d, const std::vector<int32_t>& flev, const std::vector<int32_t>& ct,
                            const std::vector<int32_t>& lvh,
                            s3a_sim3* T, double lambda, int it, int update, int lm, hipStream_t st) {
  hipLaunchKernelGGL(k_pgo_chi2, dim3(1), dim3(PGO_WG), 0, st, d, it);
  if (!update || d.m == 0) return hipGetLastError();
  const int64_t work = std::max<int64_t>((int64_t)d.nblk * 49, (int64_t)d.m * 49);
  const int ga = (int)std::min<int64_t>((work + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pgo_assemble, dim3(ga), dim3(256), 0, st, d, lambda, lm);
  for (int l = 0; l + 1 < (int)flev.size(); ++l) {
    const int ntgt = ct[flev[l + 1]] - ct[flev[l]], ncol = flev[l + 1] - flev[l];
    if (ntgt > 0) {
      const int g = std::min((ntgt + LEV_WG / 64 - 1) / (LEV_WG / 64), 1024);
      hipLaunchKernelGGL(k_pgo_level_updates, dim3(g), dim3(LEV_WG), 0, st, d, ct[flev[l]], ct[flev[l + 1]]);
    }
    const int32_t* e = lvh.data() + LVW * l;
    const LevelArg la{e[0], e[1], e[2], e[4], e[5], e[6], e[7]};
    hipLaunchKernelGGL(k_pgo_level_factor, dim3(std::min(ncol, 1024)), dim3(LEV_WG), 0, st, d, l, la);
  }
  if (d.K > 0) {
    hipLaunchKernelGGL(k_pgo_clique_updates, dim3((unsigned)((clique_update_waves(d) + 3) / 4)), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_front_diag, dim3(1), dim3(64), 0, st, d, 0);
    for (int k0 = 0; k0 + FB < d.nF; k0 += FB) {
      const int nr = d.nF - k0 - FB, T = (nr + FT - 1) / FT;
      hipLaunchKernelGGL(k_front_update, dim3(T * (T + 1) / 2 + 1), dim3(FRONT_TWG), 0, st, d, k0);
    }
  }
  hipLaunchKernelGGL(k_pgo_finish, dim3(1 + 8 * FIN_HELPERS), dim3(FIN_WG), 0, st, d, T, lambda, lm);
  return hipGetLastError();
}

double huber_energy(const std::vector<double>& r2, double delta) {
  double F = 0.0;
  for (double x : r2) {
    const double r = sqrt(x > 0.0 ? x : 0.0);
    F += r <= delta ? 0.5 * r * r : delta * (r - 0.5 * delta);
  }
  return F;
}

// Levenberg-Marquardt driver: every trial is one damped solve on the device
// (launch_iteration, which also leaves the predicted reduction), a
// linearisation at the trial poses into the second buffer set, and a read of
// the trial's per-edge e^T Omega e to decide on the host.
int pgo_solve_lm(PgoWorkspace* ws, int* last_hip, int32_t n_nodes, int32_t n_edges, const s3a_sim3* T_meas,
                 const double* omega, s3a_sim3* T, const s3a_pgo_params& p, s3a_pgo_report* report, hipStream_t st) {
  PgoDev cur = ws->dev, trial = ws->dev;
  trial.M = ws->M_alt;
  trial.v = ws->v_alt;
  trial.r2 = ws->r2_alt;
  const int max_rej = p.max_rejects > 0 ? p.max_rejects : 10;
  double lam = p.lambda > 0.0 ? p.lambda : 1e-4, nu = 2.0;
  std::vector<double> r2(n_edges), r2t(n_edges), chi;
  hipError_t e = hipSuccess;
  auto linearize = [&](const PgoDev& dd, std::vector<double>& out) -> hipError_t {
    if (n_edges == 0) return hipSuccess;
    hipError_t ee = launch_linearize(dd, T_meas, omega, T, p.huber_delta, 0, st);
    if (ee == hipSuccess) ee = hipMemcpyAsync(out.data(), dd.r2, sizeof(double) * n_edges, hipMemcpyDeviceToHost, st);
    if (ee == hipSuccess) ee = hipStreamSynchronize(st);
    return ee;
  };
  auto sum = [](const std::vector<double>& x) {
    double s = 0.0;
    for (double v : x) s += v;
    return s;
  };
  if ((e = linearize(cur, r2)) != hipSuccess) return fail(last_hip, e);
  double F = huber_energy(r2, p.huber_delta);
  chi.push_back(sum(r2));
  int kept_steps = 0, rejected = 0, stalled = 0, converged = 0, status = 0;
  for (int it = 0; it < p.iters && cur.m > 0 && n_edges > 0; ++it) {
    bool kept = false;
    for (int rej = 0; rej < max_rej; ++rej) {
      e = hipMemcpyAsync(ws->T_bak, T, sizeof(s3a_sim3) * n_nodes, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = launch_fill_zero(reinterpret_cast<uint32_t*>(cur.status), 1, st);
      if (e != hipSuccess) return fail(last_hip, e);
      if ((e = launch_iteration(cur, ws->flev, ws->ct, ws->lvh, T, lam, it, 1, 1, st)) != hipSuccess) return fail(last_hip, e);
      int32_t fst = 0;
      double pred = 0.0;
      e = hipMemcpyAsync(&fst, cur.status, sizeof(int32_t), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(&pred, cur.pred, sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return fail(last_hip, e);
      status = fst;
      if (fst == 0 && pred <= 1e-15 * F) {  // below what F resolves: converged
        e = hipMemcpyAsync(T, ws->T_bak, sizeof(s3a_sim3) * n_nodes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fail(last_hip, e);
        converged = 1;
        break;
      }
      if (fst == 0) {
        if ((e = linearize(trial, r2t)) != hipSuccess) return fail(last_hip, e);
        const double Ft = huber_energy(r2t, p.huber_delta);
        if (pred > 0.0 && Ft < F) {
          const double rho = (F - Ft) / pred;
          const double f = 1.0 - (2.0 * rho - 1.0) * (2.0 * rho - 1.0) * (2.0 * rho - 1.0);
          lam *= f > 1.0 / 3.0 ? f : 1.0 / 3.0;
          nu = 2.0;
          std::swap(cur.M, trial.M);
          std::swap(cur.v, trial.v);
          std::swap(cur.r2, trial.r2);
          r2.swap(r2t);
          F = Ft;
          kept = true;
          break;
        }
      }
      // rejected: restore the poses, raise the damping
      e = hipMemcpyAsync(T, ws->T_bak, sizeof(s3a_sim3) * n_nodes, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return fail(last_hip, e);
      ++rejected;
      lam *= nu;
      nu *= 2.0;
    }
    if (converged) break;
    if (!kept) {
      stalled = 1;
      break;
    }
    status = 0;
    ++kept_steps;
    chi.push_back(sum(r2));
  }
  // the linearisation buffers the workspace names are the ones kept last
  ws->dev.M = cur.M;
  ws->dev.v = cur.v;
  ws->dev.r2 = cur.r2;
  ws->M_alt = trial.M;
  ws->v_alt = trial.v;
  ws->r2_alt = trial.r2;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(last_hip, e);
  if (report) {
    memset(report, 0, sizeof(*report));
    for (size_t i = 0; i < chi.size() && i < 64; ++i) report->chi2[i] = chi[i];
    report->final_chi2 = chi.back();
    report->iters = kept_steps;
    report->status = stalled ? status : 0;
    report->factor_nnz_blocks = ws->nnz_blocks;
    report->lambda_final = lam;
    report->rejected = rejected;
    report->stalled = stalled;
  }
  return S3A_OK;
}

}  // namespace

// ------------------------------------------------------------------ edges from alignments

// One lane per pair of an alignment batch: the registration result becomes a
// pose-graph edge (Sec. III-C.2 feeding Sec. III-E). The alignment of source
// points of submap j onto target points of submap i returns S = T_ij, and its
// last Gauss-Newton matrix H for left perturbations S -> Exp(xi) S. A relative
// pose T = Exp(xi) S has edge residual e = Log(S^-1 T) = Ad(S^-1) xi, so
// 1/2 xi^T H xi = 1/2 e^T Ad(S)^T H Ad(S) e; with kappa = info_scale * n_valid,
// Omega = kappa Ad(S)^T H Ad(S) (row-major, symmetric by construction: both
// triangles are written from one product). A failed pair gives the identity
// and Omega = 0, and its status is passed on.
__global__ __launch_bounds__(64) void k_edges_from_alignment(int n, const s3a_sim3* S,
                                                            const s3a_align_info* __restrict__ info,
                                                            double info_scale, s3a_sim3* T_out,
                                                            double* __restrict__ omega,
                                                            int32_t* __restrict__ status) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const s3a_align_info& in = info[e];
  const int st = in.status;
  s3a_sim3 T;
  for (int k = 0; k < 16; ++k) (&T.R[0])[k] = 0.0;
  double* Om = omega + 49 * (size_t)e;
  if (st != S3A_PAIR_OK) {
    T.R[0] = T.R[4] = T.R[8] = 1.0;
    T.s = 1.0;
    for (int k = 0; k < 49; ++k) Om[k] = 0.0;
  } else {
    Sim3d A;
    for (int k = 0; k < 9; ++k) A.R[k] = S[e].R[k];
    for (int k = 0; k < 3; ++k) A.t[k] = S[e].t[k];
    A.s = S[e].s;
    for (int k = 0; k < 9; ++k) T.R[k] = A.R[k];
    for (int k = 0; k < 3; ++k) T.t[k] = A.t[k];
    T.s = A.s;
    double Ad[49], H[49], HA[49];
    sim3_Ad(A, Ad);
    // unpack the upper triangle (row-major) of H
    int u = 0;
    for (int r = 0; r < 7; ++r)
      for (int c = r; c < 7; ++c) {
        const double v = in.H[u++];
        H[7 * r + c] = v;
        H[7 * c + r] = v;
      }
    for (int r = 0; r < 7; ++r)
      for (int c = 0; c < 7; ++c) {
        double a = 0.0;
        for (int k = 0; k < 7; ++k) a = fma(H[7 * r + k], Ad[7 * k + c], a);
        HA[7 * r + c] = a;
      }
    const double kappa = info_scale * (double)in.n_valid;
    for (int r = 0; r < 7; ++r)
      for (int c = r; c < 7; ++c) {
        double a = 0.0;
        for (int k = 0; k < 7; ++k) a = fma(Ad[7 * k + r], HA[7 * k + c], a);
        a *= kappa;
        Om[7 * r + c] = a;
        Om[7 * c + r] = a;
      }
  }
  T_out[e] = T;
  if (status) status[e] = st;
}

hipError_t launch_edges_from_alignment(int n, const s3a_sim3* S, const s3a_align_info* info, double info_scale,
                                       s3a_sim3* T_out, double* omega, int32_t* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_edges_from_alignment, dim3((n + 63) / 64), dim3(64), 0, st, n, S, info, info_scale, T_out,
                     omega, status);
  return hipGetLastError();
}

void pgo_free(PgoWorkspace* ws) {
  if (!ws) return;
  if (ws->buf) (void)hipFree(ws->buf);
  delete ws;
}

int pgo_solve(PgoWorkspace** wsp, int* last_hip, int32_t n_nodes, int32_t n_edges, const int32_t* ij,
              const s3a_sim3* T_meas, const double* omega, s3a_sim3* T, const s3a_pgo_params* params,
              s3a_pgo_report* report, hipStream_t st) {
  s3a_pgo_params p;
  if (params) {
    p = *params;
  } else {
    memset(&p, 0, sizeof(p));
    p.iters = 20;
    p.huber_delta = __builtin_inf();
  }
  if (n_nodes < 1 || n_edges < 0 || !T || (n_edges > 0 && (!ij || !T_meas))) return S3A_EINVAL;
  if (p.iters < 0 || p.iters > 1000 || p.gauge < 0 || p.gauge >= n_nodes) return S3A_EINVAL;
  if (!(p.huber_delta > 0.0) || !(p.lambda >= 0.0) || !(p.lambda < 1e300) ||
      (p.flags & ~(S3A_PGO_INIT_CHAIN | S3A_PGO_LM)) || p.max_rejects < 0 || p.max_rejects > 1000)
    return S3A_EINVAL;
  for (int k = 0; k < n_edges; ++k) {
    const int i = ij[2 * k], j = ij[2 * k + 1];
    if (i < 0 || j < 0 || i >= n_nodes || j >= n_nodes || i == j) return S3A_EINVAL;
  }
  if (!*wsp) *wsp = new PgoWorkspace();
  PgoWorkspace* ws = *wsp;
  const bool same = ws->buf && ws->n_nodes == n_nodes && ws->n_edges == n_edges && ws->gauge == p.gauge &&
                    ws->cap_iters >= p.iters + 1 && ws->ij.size() == 2 * (size_t)n_edges &&
                    std::equal(ws->ij.begin(), ws->ij.end(), ij);
  if (!same) {
    const Symbolic S = analyse(n_nodes, n_edges, ij, p.gauge);
    const int E = n_edges, m = S.m, nb = S.nblk;
    const int iters_cap = std::max(p.iters + 1, 64);
    size_t total = 0;
    total += bytes_of<int32_t>(E) * 2 + bytes_of<int32_t>(n_nodes) + bytes_of<int32_t>(m);
    total += bytes_of<int32_t>(m + 1) + bytes_of<int32_t>(nb) * 2;
    total += bytes_of<int32_t>(S.dg_ptr.size()) + bytes_of<int32_t>(S.dg_edge.size());
    total += bytes_of<int32_t>(S.ob_ptr.size()) + bytes_of<int32_t>(S.ob_edge.size());
    total += bytes_of<int32_t>(S.gv_ptr.size()) + bytes_of<int32_t>(S.gv_edge.size()) + bytes_of<int8_t>(S.gv_sign.size());
    total += bytes_of<int32_t>(S.up_ptr.size()) + bytes_of<int32_t>(S.up_a.size()) * 2;
    total += bytes_of<int32_t>(S.flev_ptr.size()) + bytes_of<int32_t>(S.flev_col.size() + 1);
    total += bytes_of<int32_t>(S.dt_tgt.size() + 1) + bytes_of<int32_t>(S.dt_ptr.size());
    total += bytes_of<int32_t>(S.dup_a.size() + 1) * 2 + bytes_of<int32_t>(S.fz_rc.size() + 2);
    total += bytes_of<int32_t>(S.lt_tgt.size() + 1) + bytes_of<int32_t>(S.ct_ptr.size());
    total += bytes_of<int32_t>(S.row_ptr.size()) + bytes_of<int32_t>(S.row_blk.size());
    total += bytes_of<int32_t>(S.fs_ptr.size()) + bytes_of<int32_t>(S.fs_blk.size() + 1);
    total += bytes_of<int32_t>(S.fu_ptr.size()) + bytes_of<int32_t>(S.fu_a.size() + 1) * 2;
    total += bytes_of<int32_t>(S.bs_ptr.size()) + bytes_of<int32_t>(S.bs_blk.size() + 1) * 2 +
             bytes_of<int32_t>(S.lv.size() + LVW) + bytes_of<double>((size_t)S.bw_size + 1);
    total += bytes_of<int32_t>(S.chain.size() + 4) + bytes_of<int32_t>(S.chain_lev.size());
    total += bytes_of<double>(49 * (size_t)m) * 2 + bytes_of<double>(49 * (size_t)nb + 49) + bytes_of<double>(7 * (size_t)m + 7);
    total += bytes_of<double>(49 * (size_t)E + 49) + bytes_of<double>(7 * (size_t)E + 7) + bytes_of<double>(E + 1);
    total += bytes_of<double>(iters_cap) + bytes_of<int32_t>(4);
    total += bytes_of<double>(7 * (size_t)m + 7) * 2 + bytes_of<double>(8);  // LM: gsave, dsave, pred
    total += bytes_of<double>(49 * (size_t)E + 49) + bytes_of<double>(7 * (size_t)E + 7) + bytes_of<double>(E + 1);
    total += bytes_of<s3a_sim3>(n_nodes);
    total += bytes_of<double>(56 * (size_t)E + 56);  // Aw
    total += bytes_of<double>((size_t)S.nF * S.nF + 1) + bytes_of<double>((size_t)S.nF * FB + 1) +
             bytes_of<double>((size_t)S.nF + 1) * 3;  // front, its diagonal blocks' inverses, reciprocal pivots,
                                                      // right-hand side, forward solve
    if (ws->buf) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(ws->buf);
      ws->buf = nullptr;
    }
    void* buf = nullptr;
    hipError_t e = hipMalloc(&buf, total);
    if (e != hipSuccess) return fail(last_hip, e);
    ws->buf = buf;
    char* c = static_cast<char*>(buf);
    PgoDev& d = ws->dev;
    d.n_nodes = n_nodes; d.n_edges = E; d.m = m; d.gauge = p.gauge; d.nblk = nb;
    d.nflev = S.nflev; d.K = S.K; d.p0 = S.p0; d.nF = S.nF; d.n_dt = (int32_t)S.dt_tgt.size();
    std::vector<int32_t> ei(E), ej(E);
    for (int k = 0; k < E; ++k) { ei[k] = ij[2 * k]; ej[k] = ij[2 * k + 1]; }
    std::vector<std::pair<void*, std::pair<const void*, size_t>>> up;
    auto put = [&](auto* dst, const auto& src) {
      if (!src.empty()) up.push_back({(void*)dst, {(const void*)src.data(), src.size() * sizeof(src[0])}});
    };
    int32_t* p_ei = carve<int32_t>(c, E); put(p_ei, ei); d.ei = p_ei;
    int32_t* p_ej = carve<int32_t>(c, E); put(p_ej, ej); d.ej = p_ej;
    int32_t* p_pos = carve<int32_t>(c, n_nodes); put(p_pos, S.pos); d.pos = p_pos;
    int32_t* p_node = carve<int32_t>(c, m); put(p_node, S.node); d.node = p_node;
    int32_t* p_cp = carve<int32_t>(c, m + 1); put(p_cp, S.col_ptr); d.col_ptr = p_cp;
    int32_t* p_br = carve<int32_t>(c, nb); put(p_br, S.blk_row); d.blk_row = p_br;
    int32_t* p_bc = carve<int32_t>(c, nb); put(p_bc, S.blk_col); d.blk_col = p_bc;
    int32_t* p_dgp = carve<int32_t>(c, S.dg_ptr.size()); put(p_dgp, S.dg_ptr); d.dg_ptr = p_dgp;
    int32_t* p_dge = carve<int32_t>(c, S.dg_edge.size()); put(p_dge, S.dg_edge); d.dg_edge = p_dge;
    int32_t* p_obp = carve<int32_t>(c, S.ob_ptr.size()); put(p_obp, S.ob_ptr); d.ob_ptr = p_obp;
    int32_t* p_obe = carve<int32_t>(c, S.ob_edge.size()); put(p_obe, S.ob_edge); d.ob_edge = p_obe;
    int32_t* p_gvp = carve<int32_t>(c, S.gv_ptr.size()); put(p_gvp, S.gv_ptr); d.gv_ptr = p_gvp;
    int32_t* p_gve = carve<int32_t>(c, S.gv_edge.size()); put(p_gve, S.gv_edge); d.gv_edge = p_gve;
    int8_t* p_gvs = carve<int8_t>(c, S.gv_sign.size()); put(p_gvs, S.gv_sign); d.gv_sign = p_gvs;
    int32_t* p_upp = carve<int32_t>(c, S.up_ptr.size()); put(p_upp, S.up_ptr); d.up_ptr = p_upp;
    int32_t* p_upa = carve<int32_t>(c, S.up_a.size()); put(p_upa, S.up_a); d.up_a = p_upa;
    int32_t* p_upb = carve<int32_t>(c, S.up_b.size()); put(p_upb, S.up_b); d.up_b = p_upb;
    int32_t* p_flp = carve<int32_t>(c, S.flev_ptr.size()); put(p_flp, S.flev_ptr); d.flev_ptr = p_flp;
    int32_t* p_flc = carve<int32_t>(c, S.flev_col.size() + 1); put(p_flc, S.flev_col); d.flev_col = p_flc;
    int32_t* p_dtt = carve<int32_t>(c, S.dt_tgt.size() + 1); put(p_dtt, S.dt_tgt); d.dt_tgt = p_dtt;
    int32_t* p_dtp = carve<int32_t>(c, S.dt_ptr.size()); put(p_dtp, S.dt_ptr); d.dt_ptr = p_dtp;
    int32_t* p_dua = carve<int32_t>(c, S.dup_a.size() + 1); put(p_dua, S.dup_a); d.dup_a = p_dua;
    int32_t* p_dub = carve<int32_t>(c, S.dup_b.size() + 1); put(p_dub, S.dup_b); d.dup_b = p_dub;
    int32_t* p_fz = carve<int32_t>(c, S.fz_rc.size() + 2); put(p_fz, S.fz_rc); d.fz_rc = p_fz;
    d.n_fz = (int32_t)(S.fz_rc.size() / 2);
    int32_t* p_ltt = carve<int32_t>(c, S.lt_tgt.size() + 1); put(p_ltt, S.lt_tgt); d.lt_tgt = p_ltt;
    int32_t* p_ctp = carve<int32_t>(c, S.ct_ptr.size()); put(p_ctp, S.ct_ptr); d.ct_ptr = p_ctp;
    int32_t* p_rwp = carve<int32_t>(c, S.row_ptr.size()); put(p_rwp, S.row_ptr); d.row_ptr = p_rwp;
    int32_t* p_rwb = carve<int32_t>(c, S.row_blk.size()); put(p_rwb, S.row_blk); d.row_blk = p_rwb;
    int32_t* p_fsp = carve<int32_t>(c, S.fs_ptr.size()); put(p_fsp, S.fs_ptr); d.fs_ptr = p_fsp;
    int32_t* p_fup = carve<int32_t>(c, S.fu_ptr.size()); put(p_fup, S.fu_ptr); d.fu_ptr = p_fup;
    int32_t* p_fua = carve<int32_t>(c, S.fu_a.size() + 1); put(p_fua, S.fu_a); d.fu_a = p_fua;
    int32_t* p_fub = carve<int32_t>(c, S.fu_b.size() + 1); put(p_fub, S.fu_b); d.fu_b = p_fub;
    int32_t* p_fsb = carve<int32_t>(c, S.fs_blk.size() + 1); put(p_fsb, S.fs_blk); d.fs_blk = p_fsb;
    int32_t* p_bsp = carve<int32_t>(c, S.bs_ptr.size()); put(p_bsp, S.bs_ptr); d.bs_ptr = p_bsp;
    int32_t* p_bsb = carve<int32_t>(c, S.bs_blk.size() + 1); put(p_bsb, S.bs_blk); d.bs_blk = p_bsb;
    int32_t* p_bsr = carve<int32_t>(c, S.bs_row.size() + 1); put(p_bsr, S.bs_row); d.bs_row = p_bsr;
    int32_t* p_lv = carve<int32_t>(c, S.lv.size() + LVW); put(p_lv, S.lv); d.lv = p_lv;
    d.bw = carve<double>(c, (size_t)S.bw_size + 1);
    d.bw_size = S.bw_size;
    if (!S.bw_on) d.bw = nullptr;
    int32_t* p_ch = carve<int32_t>(c, S.chain.size() + 4); put(p_ch, S.chain); d.chain = p_ch;
    d.n_chain = (int32_t)(S.chain.size() / 4);
    int32_t* p_cl = carve<int32_t>(c, S.chain_lev.size()); put(p_cl, S.chain_lev); d.chain_lev = p_cl;
    d.n_chain_lev = (int32_t)S.chain_lev.size() - 1;
    d.Ld = carve<double>(c, 49 * (size_t)m);
    d.Di = carve<double>(c, 49 * (size_t)m);
    d.Lb = carve<double>(c, 49 * (size_t)nb + 49);
    d.g = carve<double>(c, 7 * (size_t)m + 7);
    d.M = carve<double>(c, 49 * (size_t)E + 49);
    d.Aw = carve<double>(c, 56 * (size_t)E + 56);
    d.v = carve<double>(c, 7 * (size_t)E + 7);
    d.r2 = carve<double>(c, E + 1);
    d.chi2 = carve<double>(c, iters_cap);
    d.status = carve<int32_t>(c, 4);
    d.gsave = carve<double>(c, 7 * (size_t)m + 7);
    d.dsave = carve<double>(c, 7 * (size_t)m + 7);
    d.pred = carve<double>(c, 8);
    ws->M_alt = carve<double>(c, 49 * (size_t)E + 49);
    ws->v_alt = carve<double>(c, 7 * (size_t)E + 7);
    ws->r2_alt = carve<double>(c, E + 1);
    ws->T_bak = carve<s3a_sim3>(c, n_nodes);
    d.F = carve<double>(c, (size_t)S.nF * S.nF + 1);
    d.Finv = carve<double>(c, (size_t)S.nF * FB + 1);
    d.Frd = carve<double>(c, (size_t)S.nF + 1);
    d.yF = carve<double>(c, (size_t)S.nF + 1);
    d.zF = carve<double>(c, (size_t)S.nF + 1);
    for (auto& u : up) {
      e = hipMemcpyAsync(u.first, u.second.first, u.second.second, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return fail(last_hip, e);
    }
    if (d.nF > 0) {  // identity padding of the front; its lower triangle is rewritten every iteration
      const size_t nn = (size_t)d.nF * d.nF;
      hipLaunchKernelGGL(k_pgo_front_init, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, d);
      if ((e = hipGetLastError()) != hipSuccess) return fail(last_hip, e);
    }
    e = hipStreamSynchronize(st);  // the host vectors go out of scope
    if (e != hipSuccess) return fail(last_hip, e);
    ws->n_nodes = n_nodes;
    ws->n_edges = n_edges;
    ws->gauge = p.gauge;
    ws->ij.assign(ij, ij + 2 * (size_t)n_edges);
    ws->cap_iters = iters_cap;
    ws->flev = S.flev_ptr;
    ws->ct = S.ct_ptr;
    ws->lvh = S.lv;
    ws->nnz_blocks = (int64_t)nb + m;
  }
  PgoDev d = ws->dev;
  hipError_t e = launch_fill_zero(reinterpret_cast<uint32_t*>(d.status), 1, st);
  if (e != hipSuccess) return fail(last_hip, e);
  if (p.flags & S3A_PGO_INIT_CHAIN) {
    hipLaunchKernelGGL(k_pgo_chain, dim3(1), dim3(CHAIN_WG), 0, st, d, T_meas, T);
    if ((e = hipGetLastError()) != hipSuccess) return fail(last_hip, e);
  }
  if (p.flags & S3A_PGO_LM) return pgo_solve_lm(ws, last_hip, n_nodes, n_edges, T_meas, omega, T, p, report, st);
  for (int it = 0; it <= p.iters; ++it) {
    const int update = it < p.iters;
    if (n_edges > 0) {
      if ((e = launch_linearize(d, T_meas, omega, T, p.huber_delta, !update, st)) != hipSuccess) return fail(last_hip, e);
    }
    if (update && d.m == 0) continue;
    if ((e = launch_iteration(d, ws->flev, ws->ct, ws->lvh, T, p.lambda, it, update, 0, st)) != hipSuccess) return fail(last_hip, e);
  }
  if (report) {
    std::vector<double> chi(p.iters + 1, 0.0);
    int32_t status = 0;
    e = hipMemcpyAsync(chi.data(), d.chi2, sizeof(double) * (p.iters + 1), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&status, d.status, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(last_hip, e);
    memset(report, 0, sizeof(*report));
    for (int i = 0; i < std::min(p.iters, 64); ++i) report->chi2[i] = chi[i];
    report->final_chi2 = n_edges > 0 ? chi[p.iters] : 0.0;
    report->status = status;
    report->iters = p.iters;
    report->factor_nnz_blocks = ws->nnz_blocks;
  } else {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(last_hip, e);
  }
  return S3A_OK;
}

}  // namespace s3a
