// Point passes of the dense Sim(3) alignment, its cost and its adjoint.
//
// One pass streams the seven SoA planes of every pair once and reduces
// per-point terms to NSTAT values per tile (see s3a_internal.h for the
// layout). Reads are 16-byte vectors (4 FP32 or 8 BF16 elements per plane per
// load), consecutive lanes on consecutive vectors. A tile is WG * ITEMS
// vectors of one pair; its reduction goes lane -> wavefront (butterfly) ->
// workgroup (LDS, FP64) -> one FP64 partial per tile. Per-pair totals are
// summed later over the pair's tiles in a fixed order, so results are
// bitwise reproducible run to run.
#pragma once

#include <type_traits>

#include "s3a_internal.h"

namespace s3a {

// ---------------------------------------------------------------- loads

template <int DT>
struct Planes;

// The planes live in global memory: loads go through global (not flat)
// address-space pointers, and are marked non-temporal. Each stored point is
// read once per pass and a pass streams far more than the caches hold, so
// keeping the lines buys nothing; on gfx950 the streaming hint lifts a
// read-only SoA sweep from about 6.2 to about 7.0 TB/s.
#if defined(__HIP_DEVICE_COMPILE__)
#define S3A_GLOBAL __attribute__((address_space(1)))
#else
#define S3A_GLOBAL
#endif
typedef float s3a_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int s3a_u4 __attribute__((ext_vector_type(4)));

// What a tile's loads need besides the element index: the stored xyz planes,
// or for depth input the three planes and the tile's pair (start element and
// cameras, in uniform registers when the whole tile lies in one frame).
template <int DT>
struct SrcCtx {
  const void* const* pl;
};

struct DepthCtx {
  const void* pl[3];
  const DepthPair* dp;
  int64_t a;            // first element of the pair
  int width, rows, frame_pixels, n_frames;
  float inv_width, inv_frame;
  int frame;            // the tile's frame when it lies in one, else -1
  DepthCam cp, cq;      // that frame's cameras (valid when frame >= 0)
};
template <>
struct SrcCtx<DT_DEPTH_F32> : DepthCtx {};
template <>
struct SrcCtx<DT_DEPTH_BF16> : DepthCtx {};

// Stored xyz planes are read in two steps: fetch() issues one 16-byte vector
// per plane into raw registers (so a tile body can have the next vectors in
// flight while it works on the current ones), unpack() turns them into floats.
// A vector that runs past the end of the planes is gathered element by element
// (zeros past the end) into the same raw form.
typedef s3a_u4 RawVec[7];

template <>
struct Planes<S3A_F32> {
  static constexpr int VEC = 4;
  __device__ static inline void fetch(const SrcCtx<S3A_F32>& src, int64_t g0, int64_t n, RawVec& r) {
    const void* const* pl = src.pl;
    if (g0 + 4 <= n) {
#pragma unroll
      for (int j = 0; j < 7; ++j)
        r[j] = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u4*)(static_cast<const uint32_t*>(pl[j]) + g0));
    } else {
#pragma unroll
      for (int j = 0; j < 7; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          r[j][e] = (g0 + e < n) ? static_cast<const uint32_t*>(pl[j])[g0 + e] : 0u;
    }
  }
  __device__ static inline void unpack(const RawVec& r, float (&v)[7][4]) {
#pragma unroll
    for (int j = 0; j < 7; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) v[j][e] = __uint_as_float(r[j][e]);
  }
  __device__ static inline void load(const SrcCtx<S3A_F32>& src, int64_t g0, int64_t n, float (&v)[7][4]) {
    RawVec r;
    fetch(src, g0, n, r);
    unpack(r, v);
  }
  // element e of plane j of a raw vector; its finiteness; zeroing it
  __device__ static inline float elem(const RawVec& r, int j, int e) { return __uint_as_float(r[j][e]); }
  __device__ static inline bool elem_finite(const RawVec& r, int j, int e) {
    return (r[j][e] & 0x7f800000u) != 0x7f800000u;
  }
  __device__ static inline void keep_elem(RawVec& r, int e, bool keep) {
#pragma unroll
    for (int j = 0; j < 7; ++j) r[j][e] = keep ? r[j][e] : 0u;
  }
};

template <>
struct Planes<S3A_BF16> {
  static constexpr int VEC = 8;
  __device__ static inline float lo(uint32_t u) { return __uint_as_float(u << 16); }
  __device__ static inline float hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
  __device__ static inline void fetch(const SrcCtx<S3A_BF16>& src, int64_t g0, int64_t n, RawVec& r) {
    const void* const* pl = src.pl;
    if (g0 + 8 <= n) {
#pragma unroll
      for (int j = 0; j < 7; ++j)
        r[j] = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u4*)(static_cast<const uint16_t*>(pl[j]) + g0));
    } else {
#pragma unroll
      for (int j = 0; j < 7; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint16_t* h = static_cast<const uint16_t*>(pl[j]);
          const uint32_t a = (g0 + 2 * i < n) ? h[g0 + 2 * i] : 0u;
          const uint32_t b = (g0 + 2 * i + 1 < n) ? h[g0 + 2 * i + 1] : 0u;
          r[j][i] = a | (b << 16);
        }
    }
  }
  __device__ static inline void unpack(const RawVec& r, float (&v)[7][8]) {
#pragma unroll
    for (int j = 0; j < 7; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[j][2 * i] = lo(r[j][i]);
        v[j][2 * i + 1] = hi(r[j][i]);
      }
  }
  __device__ static inline void load(const SrcCtx<S3A_BF16>& src, int64_t g0, int64_t n, float (&v)[7][8]) {
    RawVec r;
    fetch(src, g0, n, r);
    unpack(r, v);
  }
  // element e (half e % 2 of word e / 2) of plane j of a raw vector; its finiteness; zeroing it
  __device__ static inline float elem(const RawVec& r, int j, int e) {
    return (e & 1) ? hi(r[j][e >> 1]) : lo(r[j][e >> 1]);
  }
  __device__ static inline bool elem_finite(const RawVec& r, int j, int e) {
    const uint32_t m = (e & 1) ? 0x7f800000u : 0x00007f80u;
    return (r[j][e >> 1] & m) != m;
  }
  __device__ static inline void keep_elem(RawVec& r, int e, bool keep) {
    const uint32_t m = (e & 1) ? 0x0000ffffu : 0xffff0000u;  // the other half
#pragma unroll
    for (int j = 0; j < 7; ++j) r[j][e >> 1] = keep ? r[j][e >> 1] : (r[j][e >> 1] & m);
  }
};

// Walk the lane's vectors of a tile: item it = 0 .. ITEMS-1 starts at element
// rel0 = (it * WG + lane) * VEC after the tile's first. Two raw buffers
// alternate: the next item's loads are issued before the current item is
// worked on, so every wavefront keeps loads in flight while it computes.
// fetch(rel, raw) issues the loads of the vector at rel; body(raw, rel0)
// consumes one. ITEMS is even. A lane runs the items with rel0 < end_rel; with
// UNIFORM, every lane runs every item that starts before end_rel for some lane
// (end_rel is the same for the whole workgroup), so that the body may use
// cross-lane operations, and masks elements at or past end_rel itself (the
// fetch bounds-checks against the planes' end).
template <int WG, int ITEMS, int VEC, typename Raw, bool UNIFORM = false, typename Fetch, typename Body>
__device__ inline void pipelined_items(int end_rel, Fetch&& fetch, Body&& body) {
  static_assert(ITEMS % 2 == 0, "items per lane must be even");
  constexpr int STRIDE = WG * VEC;
  Raw A, B;
  const int first = (int)threadIdx.x * VEC;
  if (UNIFORM ? end_rel <= 0 : first >= end_rel) return;
  fetch(first, A);
#pragma unroll 1
  for (int it = 0; it < ITEMS; it += 2) {
    const int base = it * STRIDE;
    const int r0 = first + base;
    const int r1 = r0 + STRIDE;
    const bool more1 = UNIFORM ? base + STRIDE < end_rel : r1 < end_rel;
    if (more1) fetch(r1, B);
    body(A, r0);
    if (!more1) break;
    const int r2 = r1 + STRIDE;
    const bool more2 = it + 2 < ITEMS && (UNIFORM ? base + 2 * STRIDE < end_rel : r2 < end_rel);
    if (more2) fetch(r2, A);
    body(B, r1);
    if (!more2) break;
  }
}

// Gradients are written once and not read back by the library: streaming
// (non-temporal) global stores.
__device__ inline void store_grad_vec(float* base, int64_t g0, int64_t n, const float* v, int VEC, int64_t lo,
                                 int64_t hi) {
  if (!base) return;
  if (g0 >= lo && g0 + VEC <= hi && g0 + VEC <= n) {
    for (int e = 0; e < VEC; e += 4) {
      const s3a_f4 x = {v[e], v[e + 1], v[e + 2], v[e + 3]};
      __builtin_nontemporal_store(x, (S3A_GLOBAL s3a_f4*)(base + g0 + e));
    }
  } else {
    for (int e = 0; e < VEC; ++e) {
      const int64_t g = g0 + e;
      if (g >= lo && g < hi && g < n) base[g] = v[e];
    }
  }
}

__device__ inline bool finite7(const float* x) {
  bool f = true;
#pragma unroll
  for (int j = 0; j < 7; ++j) f = f && __builtin_isfinite(x[j]);
  return f;
}

// ---------------------------------------------------------------- uniform parameters

// The per-pair parameters are the same for every lane of a tile: read them
// once and keep them in scalar registers.
__device__ inline float uniform_f32(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ inline int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline double uniform_f64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline PointParams load_params(const PointParams* p) {
  PointParams r;
#pragma unroll
  for (int i = 0; i < 9; ++i) { r.M[i] = uniform_f64(p->M[i]); r.Mf[i] = uniform_f32(p->Mf[i]); }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    r.t[i] = uniform_f64(p->t[i]);
    r.c[i] = uniform_f64(p->c[i]);
    r.tcf[i] = uniform_f32(p->tcf[i]);
    r.cf[i] = uniform_f32(p->cf[i]);
  }
  r.inv_C = uniform_f32(p->inv_C);
  r.scale = uniform_f32(p->scale);
  r.L = uniform_f32(p->L);
  r.active = uniform_i32(p->active);
  r.nonfinite = uniform_i32(p->nonfinite);
  return r;
}

__device__ inline TileDesc load_tile(const TileDesc* p) {
  TileDesc r;
  const long long b = p->begin, e = p->end, l = p->lo;
  r.begin = ((long long)(unsigned)uniform_i32((int)(b >> 32)) << 32) | (unsigned)uniform_i32((int)b);
  r.end = ((long long)(unsigned)uniform_i32((int)(e >> 32)) << 32) | (unsigned)uniform_i32((int)e);
  r.lo = ((long long)(unsigned)uniform_i32((int)(l >> 32)) << 32) | (unsigned)uniform_i32((int)l);
  r.pair = uniform_i32(p->pair);
  r.pad = 0;
  return r;
}

// Depth input: three planes (d_p, d_q, c), the pixel's frame, row and column
// from its index in the pair, and each side unprojected with its camera:
// x = R (d ((col, row) * inv_f + o, 1)) + t. Elements before the pair's start
// (the head of a boundary vector) get the pair's first pixel; the tile bodies
// zero them anyway.
__device__ inline DepthCam load_cam_uniform(const DepthCam* c) {
  DepthCam r;
  r.ifx = uniform_f32(c->ifx);
  r.ify = uniform_f32(c->ify);
  r.ox = uniform_f32(c->ox);
  r.oy = uniform_f32(c->oy);
#pragma unroll
  for (int i = 0; i < 9; ++i) r.R[i] = uniform_f32(c->R[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) r.t[i] = uniform_f32(c->t[i]);
  return r;
}

__device__ inline void unproject(const DepthCam& c, float col, float row, float d, float* x) {
  const float rx = fmaf(col, c.ifx, c.ox), ry = fmaf(row, c.ify, c.oy);
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = fmaf(d, fmaf(c.R[3 * i], rx, fmaf(c.R[3 * i + 1], ry, c.R[3 * i + 2])), c.t[i]);
}

// q = floor(x / m) for 0 <= x < 2^31, m >= 1: a float estimate, corrected.
__device__ inline int div_floor(int x, int m, float inv_m) {
  int q = (int)((float)x * inv_m);
  q -= (q * m > x) ? 1 : 0;
  q += ((q + 1) * m <= x) ? 1 : 0;
  q -= (q * m > x) ? 1 : 0;
  return q;
}

template <int DT>
struct DepthPlanes {
  static constexpr bool BF = DT == DT_DEPTH_BF16;
  static constexpr int VEC = BF ? 8 : 4;
  // d[0], d[1], d[2] = d_p, d_q, c of elements g0 .. g0 + VEC - 1 (0 past n)
  __device__ static inline void load_raw(const SrcCtx<DT>& s, int64_t g0, int64_t n, float (&d)[3][VEC]) {
    if (g0 + VEC <= n) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if constexpr (BF) {
          const s3a_u4 x = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u4*)(static_cast<const uint16_t*>(s.pl[j]) + g0));
          d[j][0] = __uint_as_float(x.x << 16); d[j][1] = __uint_as_float(x.x & 0xffff0000u);
          d[j][2] = __uint_as_float(x.y << 16); d[j][3] = __uint_as_float(x.y & 0xffff0000u);
          d[j][4] = __uint_as_float(x.z << 16); d[j][5] = __uint_as_float(x.z & 0xffff0000u);
          d[j][6] = __uint_as_float(x.w << 16); d[j][7] = __uint_as_float(x.w & 0xffff0000u);
        } else {
          const s3a_f4 x = __builtin_nontemporal_load((const S3A_GLOBAL s3a_f4*)(static_cast<const float*>(s.pl[j]) + g0));
          d[j][0] = x.x; d[j][1] = x.y; d[j][2] = x.z; d[j][3] = x.w;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          if constexpr (BF)
            d[j][e] = (g0 + e < n) ? __uint_as_float((uint32_t)static_cast<const uint16_t*>(s.pl[j])[g0 + e] << 16) : 0.0f;
          else
            d[j][e] = (g0 + e < n) ? static_cast<const float*>(s.pl[j])[g0 + e] : 0.0f;
        }
    }
  }

  // The same in two steps (raw 16-byte vectors first; see RawVec).
  typedef s3a_u4 Raw[3];
  __device__ static inline void fetch(const SrcCtx<DT>& s, int64_t g0, int64_t n, Raw& r) {
    if (g0 + VEC <= n) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if constexpr (BF)
          r[j] = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u4*)(static_cast<const uint16_t*>(s.pl[j]) + g0));
        else
          r[j] = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u4*)(static_cast<const uint32_t*>(s.pl[j]) + g0));
      }
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if constexpr (BF) {
            const uint16_t* h = static_cast<const uint16_t*>(s.pl[j]);
            const uint32_t a = (g0 + 2 * i < n) ? h[g0 + 2 * i] : 0u;
            const uint32_t b = (g0 + 2 * i + 1 < n) ? h[g0 + 2 * i + 1] : 0u;
            r[j][i] = a | (b << 16);
          } else {
            r[j][i] = (g0 + i < n) ? static_cast<const uint32_t*>(s.pl[j])[g0 + i] : 0u;
          }
        }
    }
  }
  __device__ static inline void unpack(const Raw& r, float (&d)[3][VEC]) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (BF) {
          d[j][2 * i] = __uint_as_float(r[j][i] << 16);
          d[j][2 * i + 1] = __uint_as_float(r[j][i] & 0xffff0000u);
        } else {
          d[j][i] = __uint_as_float(r[j][i]);
        }
      }
  }

  // frame, row and column of element g0 (elements before the pair count as its first pixel)
  __device__ static inline void position(const SrcCtx<DT>& s, int64_t g0, int& f, int& row, int& col) {
    int j = (int)(g0 - s.a);
    j = j < 0 ? 0 : j;
    f = div_floor(j, s.frame_pixels, s.inv_frame);
    const int pin = j - f * s.frame_pixels;
    row = div_floor(pin, s.width, s.inv_width);
    col = pin - row * s.width;
  }

  // the next pixel (row-major, frame after frame)
  __device__ static inline void advance(const SrcCtx<DT>& s, int& f, int& row, int& col) {
    if (++col == s.width) {
      col = 0;
      if (++row == s.rows) {
        row = 0;
        ++f;
      }
    }
  }

  __device__ static inline void load(const SrcCtx<DT>& s, int64_t g0, int64_t n, float (&v)[7][VEC]) {
    float d[3][VEC];
    load_raw(s, g0, n, d);
    int f, row, col;
    position(s, g0, f, row, col);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      float x[3], y[3];
      if (s.frame >= 0) {
        unproject(s.cp, (float)col, (float)row, d[0][e], x);
        unproject(s.cq, (float)col, (float)row, d[1][e], y);
      } else {
        const int fc = f < s.n_frames ? f : s.n_frames - 1;
        unproject(s.dp->p[fc], (float)col, (float)row, d[0][e], x);
        unproject(s.dp->q[fc], (float)col, (float)row, d[1][e], y);
      }
      v[0][e] = x[0]; v[1][e] = x[1]; v[2][e] = x[2];
      v[3][e] = y[0]; v[4][e] = y[1]; v[5][e] = y[2];
      v[6][e] = d[2][e];
      if (g0 + e >= s.a) advance(s, f, row, col);
    }
  }
};

template <>
struct Planes<DT_DEPTH_F32> : DepthPlanes<DT_DEPTH_F32> {};
template <>
struct Planes<DT_DEPTH_BF16> : DepthPlanes<DT_DEPTH_BF16> {};

// The load context of a tile (see SrcCtx).
template <int DT>
__device__ inline SrcCtx<DT> make_src(const void* const* pl, const Work& w, const TileDesc& td) {
  if constexpr (DT == DT_DEPTH_F32 || DT == DT_DEPTH_BF16) {
    SrcCtx<DT> s;
    s.pl[0] = pl[0];
    s.pl[1] = pl[1];
    s.pl[2] = pl[2];
    s.dp = w.dpairs + td.pair;
    s.a = td.lo;
    s.width = uniform_i32(s.dp->width);
    s.rows = uniform_i32(s.dp->rows);
    s.frame_pixels = uniform_i32(s.dp->frame_pixels);
    s.n_frames = uniform_i32(s.dp->n_frames);
    s.inv_width = uniform_f32(s.dp->inv_width);
    s.inv_frame = uniform_f32(s.dp->inv_frame);
    const int HW = s.frame_pixels, nf = s.n_frames;
    const int64_t first = td.begin > td.lo ? td.begin : td.lo;
    const int f0 = (int)((first - td.lo) / HW), f1 = (int)((td.end - 1 - td.lo) / HW);
    s.frame = (f0 == f1 && f0 < nf && td.end > first) ? f0 : -1;
    if (s.frame >= 0) {
      s.cp = load_cam_uniform(s.dp->p + s.frame);
      s.cq = load_cam_uniform(s.dp->q + s.frame);
    }
    return s;
  } else {
    (void)w;
    (void)td;
    return SrcCtx<DT>{pl};
  }
}

// ---------------------------------------------------------------- per-point terms

// Residual r = s R p + t - q and centred model point y_c = s R p + t - c,
// formed in FP64 (so that r keeps full FP32 relative precision however far
// the points are from the origin), then rounded to FP32.
__device__ inline void residual(const PointParams& P, const float* x, float (&r)[3], float (&yc)[3]) {
  const double p0 = x[0], p1 = x[1], p2 = x[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double y = fma(P.M[3 * i], p0, fma(P.M[3 * i + 1], p1, fma(P.M[3 * i + 2], p2, P.t[i])));
    r[i] = (float)(y - (double)x[3 + i]);
    yc[i] = (float)(y - P.c[i]);
  }
}

// Cost at S: 0 sum w, 1 sum w rho, 2 V (FP64 per lane).
__device__ inline void point_cost(double (&a)[3], const PointParams& P, float* x, bool in, float tau,
                                  float delta) {
  const bool valid = in && finite7(x) && x[6] >= tau;
  if (!valid) {
#pragma unroll
    for (int j = 0; j < 7; ++j) x[j] = 0.0f;
  }
  float r[3], y[3];
  residual(P, x, r, y);
  const float e2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  float rho;
  if (e2 <= delta * delta) rho = 0.5f * e2;
  else rho = delta * (e2 * rsqrtf(e2) - 0.5f * delta);
  a[0] += (double)x[6];
  a[1] = fma((double)x[6], (double)rho, a[1]);
  a[2] += valid ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- reductions

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// FP32 sums over the 64 lanes of a wavefront with DPP row operations (a fixed
// pairwise tree: neighbours within quads, half rows, rows, then across rows;
// the total ends in lane 63). All NSTAT sums advance one step at a time, so
// consecutive DPP operations never read a register written just before.
template <int N>
__device__ inline void wave_totals_f32(float (&v)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j)  // quad_perm [1,0,3,2]
    v[j] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), 0xb1, 0xf, 0xf, false));
#pragma unroll
  for (int j = 0; j < N; ++j)  // quad_perm [2,3,0,1]
    v[j] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), 0x4e, 0xf, 0xf, false));
#pragma unroll
  for (int j = 0; j < N; ++j)  // row_half_mirror
    v[j] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), 0x141, 0xf, 0xf, false));
#pragma unroll
  for (int j = 0; j < N; ++j)  // row_mirror
    v[j] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), 0x140, 0xf, 0xf, false));
#pragma unroll
  for (int j = 0; j < N; ++j)  // row_bcast:15 into rows 1 and 3
    v[j] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), 0x142, 0xa, 0xf, false));
#pragma unroll
  for (int j = 0; j < N; ++j)  // row_bcast:31 into rows 2 and 3
    v[j] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), 0x143, 0xc, 0xf, false));
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[j]), 63));
}

// Reduce NSTAT per-lane FP32 values over the workgroup (DPP within a
// wavefront, then FP64 across wavefronts through LDS) and store one FP64
// partial.
template <int WG>
__device__ inline void block_store_f32(float (&acc)[NSTAT], double (*red)[NSTAT], double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  wave_totals_f32(acc);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NSTAT; ++j) red[wv][j] = (double)acc[j];
  }
  __syncthreads();
  if ((int)threadIdx.x < NSTAT) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < WG / 64; ++q) s += red[q][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// One DPP step on a double: both 32-bit halves move with the same control.
template <int CTRL, int ROWS>
__device__ inline double dpp_f64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// FP64 sums over the 64 lanes of a wavefront: the same fixed DPP tree as the
// FP32 reduction above, advanced step-major over the N sums; every lane ends
// with the totals (read from lane 63).
template <int N>
__device__ inline void wave_totals_f64(double (&v)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] += dpp_f64<0xb1, 0xf>(v[j]);
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] += dpp_f64<0x4e, 0xf>(v[j]);
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] += dpp_f64<0x141, 0xf>(v[j]);
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] += dpp_f64<0x140, 0xf>(v[j]);
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] += dpp_f64<0x142, 0xa>(v[j]);
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] += dpp_f64<0x143, 0xc>(v[j]);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v[j]);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    v[j] = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
}

// Reduce N <= NSTAT per-lane FP64 values over the workgroup (DPP within a
// wavefront, then across wavefronts through LDS) and store N FP64 sums.
template <int WG, int N>
__device__ inline void block_store_f64(double (&acc)[N], double (*red)[NSTAT], double* out) {
  static_assert(N <= NSTAT, "too many sums");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  wave_totals_f64(acc);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) red[wv][j] = acc[j];
  }
  __syncthreads();
  if ((int)threadIdx.x < N) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < WG / 64; ++q) s += red[q][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- tile bodies

// One point of the Gauss-Newton statistics: centred model point y, residual
// r, weight w (0 for masked points); Huber weight branch-free. COST: also the
// cost and inlier count (statistics 17 and 18), which only the pass at the
// last linearisation point reports; the other passes leave them at zero.
template <bool COST = true>
__device__ inline void gn_point(float (&a)[NSTAT], float y0, float y1, float y2, float r0, float r1, float r2, float w,
                                float d2, float delta, float hd2) {
  const float e2 = fmaf(r0, r0, fmaf(r1, r1, r2 * r2));
  const float ie = __builtin_amdgcn_rsqf(e2);
  const bool inl = e2 <= d2;
  const float psi = inl ? 1.0f : delta * ie;
  const float om = w * psi;
  const float oy0 = om * y0, oy1 = om * y1, oy2 = om * y2;
  a[0] += om;
  a[1] += oy0; a[2] += oy1; a[3] += oy2;
  a[4] = fmaf(oy0, y0, a[4]); a[5] = fmaf(oy0, y1, a[5]); a[6] = fmaf(oy0, y2, a[6]);
  a[7] = fmaf(oy1, y1, a[7]); a[8] = fmaf(oy1, y2, a[8]); a[9] = fmaf(oy2, y2, a[9]);
  a[10] = fmaf(om, r0, a[10]); a[11] = fmaf(om, r1, a[11]); a[12] = fmaf(om, r2, a[12]);
  a[13] = fmaf(oy1, r2, fmaf(-oy2, r1, a[13]));
  a[14] = fmaf(oy2, r0, fmaf(-oy0, r2, a[14]));
  a[15] = fmaf(oy0, r1, fmaf(-oy1, r0, a[15]));
  a[16] = fmaf(oy0, r0, fmaf(oy1, r1, fmaf(oy2, r2, a[16])));
  if constexpr (COST) {
    const float rho = inl ? 0.5f * e2 : fmaf(delta * e2, ie, -hd2);
    a[17] = fmaf(w, rho, a[17]);
    a[18] += (inl && w > 0.0f) ? 1.0f : 0.0f;
  }
}

// Gauss-Newton pass over a depth tile that lies in one frame: the pair's
// current similarity is folded into each side's camera once per tile, so a
// pixel costs one affine map per side on its ray:
//   y_c = d_p (A ray_p) + b,  A = sR R_p, b = sR t_p + t - c;   q_c = d_q (R_q ray_q) + t_q - c.
template <int DT, int WG, int ITEMS, bool COST>
__device__ inline void tile_gn_depth_frame(const Shape& sh, const SrcCtx<DT>& src, const TileDesc& td,
                                           const PointParams& P, float (&a)[NSTAT]) {
  using L = DepthPlanes<DT>;
  constexpr int VEC = L::VEC;
  const DepthCam& cp = src.cp;
  const DepthCam& cq = src.cq;
  float A[9], b[3], bq[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
      A[3 * i + j] = fmaf(P.Mf[3 * i], cp.R[j], fmaf(P.Mf[3 * i + 1], cp.R[3 + j], P.Mf[3 * i + 2] * cp.R[6 + j]));
    b[i] = fmaf(P.Mf[3 * i], cp.t[0], fmaf(P.Mf[3 * i + 1], cp.t[1], fmaf(P.Mf[3 * i + 2], cp.t[2], P.tcf[i])));
    bq[i] = cq.t[i] - P.cf[i];
  }
  const float tau = sh.tau, delta = sh.delta_f;
  const float d2 = delta * delta, hd2 = 0.5f * delta * delta;
  const int lo_rel = (int)(td.lo - td.begin), end_rel = (int)(td.end - td.begin);
  const bool check_finite = P.nonfinite != 0;
  pipelined_items<WG, ITEMS, VEC, typename L::Raw>(
      end_rel, [&](int rel, typename L::Raw& r) { L::fetch(src, td.begin + rel, sh.n_points, r); },
      [&](const typename L::Raw& raw, int rel0) {
    float d[3][VEC];
    L::unpack(raw, d);
    int f, row, col;
    L::position(src, td.begin + rel0, f, row, col);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const bool in = rel0 + e >= lo_rel && rel0 + e < end_rel;
      const float fc = (float)col, fr = (float)row;
      const float rxp = fmaf(fc, cp.ifx, cp.ox), ryp = fmaf(fr, cp.ify, cp.oy);
      const float rxq = fmaf(fc, cq.ifx, cq.ox), ryq = fmaf(fr, cq.ify, cq.oy);
      float y[3], q[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        y[i] = fmaf(d[0][e], fmaf(A[3 * i], rxp, fmaf(A[3 * i + 1], ryp, A[3 * i + 2])), b[i]);
        q[i] = fmaf(d[1][e], fmaf(cq.R[3 * i], rxq, fmaf(cq.R[3 * i + 1], ryq, cq.R[3 * i + 2])), bq[i]);
      }
      bool ok = in;
      if (check_finite) ok = ok && __builtin_isfinite(y[0] + y[1] + y[2] + q[0] + q[1] + q[2]) && __builtin_isfinite(d[2][e]);
      const float c = d[2][e];
      const float w = (ok && c >= tau) ? c : 0.0f;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        y[i] = ok ? y[i] : 0.0f;
        q[i] = ok ? q[i] : 0.0f;
      }
      gn_point<COST>(a, y[0], y[1], y[2], y[0] - q[0], y[1] - q[1], y[2] - q[2], w, d2, delta, hd2);
      if (rel0 + e >= lo_rel) L::advance(src, f, row, col);
    }
  });
}


// Gauss-Newton pass over one tile. Every quantity is formed in FP32 in
// coordinates centred on the pair's centre c (the weighted target centroid):
//   y_c = Mf p + (t - c),  q_c = q - c,  r = y_c - q_c,
// so no product or difference involves coordinates far from the data, and the
// 17 statistics (plus cost and inlier count when COST) accumulate per lane
// over the few points the lane handles in this tile (then pairwise across
// lanes, FP64 across wavefronts and tiles). Points outside the pair's range,
// below the confidence threshold, or (in pairs that hold any) with a NaN/Inf
// value get zero weight and zeroed coordinates.
// Elements of a raw vector that lie outside the pair's range [lo_rel, end_rel),
// or (check_finite) hold a NaN/Inf in any plane, are zeroed in place: zero
// weight and zero coordinates. Both cases are rare (a pair's first and last
// vectors; pairs the moments pass found non-finite values in), so the common
// vector pays one uniform test each.
template <int DT>
__device__ inline void mask_raw(RawVec& r, int rel0, int lo_rel, int end_rel, bool check_finite) {
  constexpr int VEC = Planes<DT>::VEC;
  if (rel0 < lo_rel || rel0 + VEC > end_rel) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) Planes<DT>::keep_elem(r, e, rel0 + e >= lo_rel && rel0 + e < end_rel);
  }
  if (check_finite) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      bool fin = true;
#pragma unroll
      for (int j = 0; j < 7; ++j) fin = fin && Planes<DT>::elem_finite(r, j, e);
      Planes<DT>::keep_elem(r, e, fin);
    }
  }
}

template <int DT, bool COST>
__device__ inline void gn_vector(const Shape& sh, const PointParams& P, RawVec& r, int rel0, int lo_rel,
                                 int end_rel, bool check_finite, float (&a)[NSTAT]) {
  constexpr int VEC = Planes<DT>::VEC;
  using L = Planes<DT>;
  const float tau = sh.tau, delta = sh.delta_f;
  const float d2 = delta * delta, hd2 = 0.5f * delta * delta;
  mask_raw<DT>(r, rel0, lo_rel, end_rel, check_finite);
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const float px = L::elem(r, 0, e), py = L::elem(r, 1, e), pz = L::elem(r, 2, e);
    const float c = L::elem(r, 6, e);
    const float w = c >= tau ? c : 0.0f;
    const float y0 = fmaf(P.Mf[0], px, fmaf(P.Mf[1], py, fmaf(P.Mf[2], pz, P.tcf[0])));
    const float y1 = fmaf(P.Mf[3], px, fmaf(P.Mf[4], py, fmaf(P.Mf[5], pz, P.tcf[1])));
    const float y2 = fmaf(P.Mf[6], px, fmaf(P.Mf[7], py, fmaf(P.Mf[8], pz, P.tcf[2])));
    gn_point<COST>(a, y0, y1, y2, y0 - (L::elem(r, 3, e) - P.cf[0]), y1 - (L::elem(r, 4, e) - P.cf[1]),
                   y2 - (L::elem(r, 5, e) - P.cf[2]), w, d2, delta, hd2);
  }
}

template <int DT, int WG, int ITEMS, bool COST>
__device__ inline void tile_gn(const Shape& sh, const SrcCtx<DT>& pl, const TileDesc& td, const PointParams& P,
                               double (*red)[NSTAT], double* out) {
  constexpr int VEC = Planes<DT>::VEC;
  float a[NSTAT];
#pragma unroll
  for (int j = 0; j < NSTAT; ++j) a[j] = 0.0f;
  if constexpr (DT == DT_DEPTH_F32 || DT == DT_DEPTH_BF16) {
    if (P.active && pl.frame >= 0) {
      tile_gn_depth_frame<DT, WG, ITEMS, COST>(sh, pl, td, P, a);
      block_store_f32<WG>(a, red, out);
      return;
    }
  }
  if (P.active) {
    const int lo_rel = (int)(td.lo - td.begin), end_rel = (int)(td.end - td.begin);
    const bool check_finite = P.nonfinite != 0;
    if constexpr (DT == S3A_F32 || DT == S3A_BF16) {
      pipelined_items<WG, ITEMS, VEC, RawVec>(
          end_rel, [&](int rel, RawVec& r) { Planes<DT>::fetch(pl, td.begin + rel, sh.n_points, r); },
          [&](RawVec& r, int rel0) { gn_vector<DT, COST>(sh, P, r, rel0, lo_rel, end_rel, check_finite, a); });
    } else {
      // depth input whose tile spans frames: unprojected per element (DepthPlanes::load)
      const float tau = sh.tau, delta = sh.delta_f;
      const float d2 = delta * delta, hd2 = 0.5f * delta * delta;
#pragma unroll 1
      for (int it = 0; it < ITEMS; ++it) {
        const int rel0 = (it * WG + (int)threadIdx.x) * VEC;
        if (rel0 >= end_rel) break;
        float v[7][VEC];
        Planes<DT>::load(pl, td.begin + rel0, sh.n_points, v);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          float x[7];
#pragma unroll
          for (int j = 0; j < 7; ++j) x[j] = v[j][e];
          const bool keep = rel0 + e >= lo_rel && rel0 + e < end_rel && (!check_finite || finite7(x));
#pragma unroll
          for (int j = 0; j < 7; ++j) x[j] = keep ? x[j] : 0.0f;
          const float w = x[6] >= tau ? x[6] : 0.0f;
          const float y0 = fmaf(P.Mf[0], x[0], fmaf(P.Mf[1], x[1], fmaf(P.Mf[2], x[2], P.tcf[0])));
          const float y1 = fmaf(P.Mf[3], x[0], fmaf(P.Mf[4], x[1], fmaf(P.Mf[5], x[2], P.tcf[1])));
          const float y2 = fmaf(P.Mf[6], x[0], fmaf(P.Mf[7], x[1], fmaf(P.Mf[8], x[2], P.tcf[2])));
          gn_point<COST>(a, y0, y1, y2, y0 - (x[3] - P.cf[0]), y1 - (x[4] - P.cf[1]), y2 - (x[5] - P.cf[2]), w,
                         d2, delta, hd2);
        }
      }
    }
  }
  block_store_f32<WG>(a, red, out);
}

// Moments of a depth-input tile whose pixels all lie in one frame. Each side is
// formed in its camera's frame, x' = d (R ray) (coordinates of the size of the
// scene, so FP32 products keep their precision), the products of the VEC pixels of
// one vector are summed in FP32 and added to FP64 lane sums (the weight sum itself
// in FP64 per pixel), and the lane sums are moved to the submap frame
// (x = x' + t) once, in FP64, at the end.
template <int DT, int WG, int ITEMS>
__device__ inline void tile_moments_depth_frame(const Shape& sh, const SrcCtx<DT>& src, const TileDesc& td,
                                                double (&a)[NSTAT], int& nvalid, int& nbad) {
  using L = DepthPlanes<DT>;
  constexpr int VEC = L::VEC;
  const DepthCam& cp = src.cp;
  const DepthCam& cq = src.cq;
  const float tau = sh.tau;
  const int lo_rel = (int)(td.lo - td.begin), end_rel = (int)(td.end - td.begin);
  pipelined_items<WG, ITEMS, VEC, typename L::Raw>(
      end_rel, [&](int rel, typename L::Raw& r) { L::fetch(src, td.begin + rel, sh.n_points, r); },
      [&](const typename L::Raw& raw, int rel0) {
    float d[3][VEC];
    L::unpack(raw, d);
    int f, row, col;
    L::position(src, td.begin + rel0, f, row, col);
    float s[17];
#pragma unroll
    for (int j = 0; j < 17; ++j) s[j] = 0.0f;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const bool in = rel0 + e >= lo_rel && rel0 + e < end_rel;
      const float fc = (float)col, fr = (float)row;
      const float rxp = fmaf(fc, cp.ifx, cp.ox), ryp = fmaf(fr, cp.ify, cp.oy);
      const float rxq = fmaf(fc, cq.ifx, cq.ox), ryq = fmaf(fr, cq.ify, cq.oy);
      float x[3], y[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        x[i] = d[0][e] * fmaf(cp.R[3 * i], rxp, fmaf(cp.R[3 * i + 1], ryp, cp.R[3 * i + 2]));
        y[i] = d[1][e] * fmaf(cq.R[3 * i], rxq, fmaf(cq.R[3 * i + 1], ryq, cq.R[3 * i + 2]));
      }
      const float c = d[2][e];
      const bool fin = __builtin_isfinite(x[0] + x[1] + x[2] + y[0] + y[1] + y[2]) && __builtin_isfinite(c);
      const bool valid = in && fin && c >= tau;
      nvalid += valid ? 1 : 0;
      nbad += (in && !fin) ? 1 : 0;
      const float w = valid ? c : 0.0f;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        x[i] = valid ? x[i] : 0.0f;
        y[i] = valid ? y[i] : 0.0f;
      }
      const float wx0 = w * x[0], wx1 = w * x[1], wx2 = w * x[2];
      const float wy0 = w * y[0], wy1 = w * y[1], wy2 = w * y[2];
      a[0] += (double)w;  // the weight sum stays exact
      s[1] += wx0; s[2] += wx1; s[3] += wx2;
      s[4] += wy0; s[5] += wy1; s[6] += wy2;
      s[7] = fmaf(wx0, x[0], fmaf(wx1, x[1], fmaf(wx2, x[2], s[7])));
      s[8] = fmaf(wy0, x[0], s[8]);  s[9] = fmaf(wy0, x[1], s[9]);  s[10] = fmaf(wy0, x[2], s[10]);
      s[11] = fmaf(wy1, x[0], s[11]); s[12] = fmaf(wy1, x[1], s[12]); s[13] = fmaf(wy1, x[2], s[13]);
      s[14] = fmaf(wy2, x[0], s[14]); s[15] = fmaf(wy2, x[1], s[15]); s[16] = fmaf(wy2, x[2], s[16]);
      if (rel0 + e >= lo_rel) L::advance(src, f, row, col);
    }
#pragma unroll
    for (int j = 1; j < 17; ++j) a[j] += (double)s[j];
  });
  // to the submap frame: x = x' + tp, y = y' + tq
  const double tp[3] = {cp.t[0], cp.t[1], cp.t[2]}, tq[3] = {cq.t[0], cq.t[1], cq.t[2]};
  const double W = a[0], Sx[3] = {a[1], a[2], a[3]}, Sy[3] = {a[4], a[5], a[6]};
  a[7] += 2.0 * (tp[0] * Sx[0] + tp[1] * Sx[1] + tp[2] * Sx[2]) + (tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]) * W;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) a[8 + 3 * i + j] += tq[i] * Sx[j] + Sy[i] * tp[j] + tq[i] * tp[j] * W;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a[1 + i] += tp[i] * W;
    a[4 + i] += tq[i] * W;
  }
}

// Moments pass over one tile: FP64 products and per-lane FP64 sums (the
// coordinates are uncentred here, so the second moments must keep more than
// FP32 precision), integer counts, DPP wavefront reduction.
template <int DT, int WG, int ITEMS>
__device__ inline void tile_moments(const Shape& sh, const SrcCtx<DT>& pl, const TileDesc& td,
                                   double (*red)[NSTAT], double* out) {
  constexpr int VEC = Planes<DT>::VEC;
  double a[NSTAT];
#pragma unroll
  for (int j = 0; j < NSTAT; ++j) a[j] = 0.0;
  int nvalid = 0, nbad = 0;
  const float tau = sh.tau;
  const int lo_rel = (int)(td.lo - td.begin), end_rel = (int)(td.end - td.begin);
  if constexpr (DT == DT_DEPTH_F32 || DT == DT_DEPTH_BF16) {
    if (pl.frame >= 0) {
      tile_moments_depth_frame<DT, WG, ITEMS>(sh, pl, td, a, nvalid, nbad);
      a[17] = (double)nvalid;
      a[18] = (double)nbad;
      block_store_f64<WG, NSTAT>(a, red, out);
      return;
    }
  }
  // one point: validity (counted), then the weighted raw moments in FP64
  auto point = [&](float (&x)[7], bool in) {
    const bool fin = finite7(x);
    const bool valid = in && fin && x[6] >= tau;
    nvalid += valid ? 1 : 0;
    nbad += (in && !fin) ? 1 : 0;
#pragma unroll
    for (int j = 0; j < 7; ++j) x[j] = valid ? x[j] : 0.0f;
    const double w = x[6];
    const double p0 = x[0], p1 = x[1], p2 = x[2], q0 = x[3], q1 = x[4], q2 = x[5];
    const double wp0 = w * p0, wp1 = w * p1, wp2 = w * p2;
    const double wq0 = w * q0, wq1 = w * q1, wq2 = w * q2;
    a[0] += w;
    a[1] += wp0; a[2] += wp1; a[3] += wp2;
    a[4] += wq0; a[5] += wq1; a[6] += wq2;
    a[7] = fma(wp0, p0, fma(wp1, p1, fma(wp2, p2, a[7])));
    a[8] = fma(wq0, p0, a[8]);  a[9] = fma(wq0, p1, a[9]);  a[10] = fma(wq0, p2, a[10]);
    a[11] = fma(wq1, p0, a[11]); a[12] = fma(wq1, p1, a[12]); a[13] = fma(wq1, p2, a[13]);
    a[14] = fma(wq2, p0, a[14]); a[15] = fma(wq2, p1, a[15]); a[16] = fma(wq2, p2, a[16]);
  };
  if constexpr (DT == S3A_F32 || DT == S3A_BF16) {
    pipelined_items<WG, ITEMS, VEC, RawVec>(
        end_rel, [&](int rel, RawVec& r) { Planes<DT>::fetch(pl, td.begin + rel, sh.n_points, r); },
        [&](RawVec& r, int rel0) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            float x[7];
#pragma unroll
            for (int j = 0; j < 7; ++j) x[j] = Planes<DT>::elem(r, j, e);
            point(x, rel0 + e >= lo_rel && rel0 + e < end_rel);
          }
        });
  } else {
#pragma unroll 1
    for (int it = 0; it < ITEMS; ++it) {
      const int rel0 = (it * WG + (int)threadIdx.x) * VEC;
      if (rel0 >= end_rel) break;
      float v[7][VEC];
      Planes<DT>::load(pl, td.begin + rel0, sh.n_points, v);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        float x[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) x[j] = v[j][e];
        point(x, rel0 + e >= lo_rel && rel0 + e < end_rel);
      }
    }
  }
  a[17] = (double)nvalid;
  a[18] = (double)nbad;
  block_store_f64<WG, NSTAT>(a, red, out);
}

// Cost pass over one tile: sum w, sum w rho (FP64 residuals, FP64 sums), V.
template <int DT, int WG, int ITEMS>
__device__ inline void tile_cost(const Shape& sh, const SrcCtx<DT>& pl, const TileDesc& td, const PointParams& P,
                                 double (*red)[NSTAT], double* out) {
  constexpr int VEC = Planes<DT>::VEC;
  double acc[3] = {0.0, 0.0, 0.0};
  if (P.active) {
    const int lo_rel = (int)(td.lo - td.begin), end_rel = (int)(td.end - td.begin);
#pragma unroll 1
    for (int it = 0; it < ITEMS; ++it) {
      const int rel0 = (it * WG + (int)threadIdx.x) * VEC;
      if (rel0 >= end_rel) break;
      float v[7][VEC];
      Planes<DT>::load(pl, td.begin + rel0, sh.n_points, v);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const bool in = rel0 + e >= lo_rel && rel0 + e < end_rel;
        float x[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) x[j] = v[j][e];
        point_cost(acc, P, x, in, sh.tau, sh.delta_f);
      }
    }
  }
  block_store_f64<WG, 3>(acc, red, out);
}

template <int DT, int MODE, int WG, int ITEMS>
__device__ inline void tile_body(const Shape& sh, const SrcCtx<DT>& pl, const TileDesc& td,
                                 const PointParams& P, double (*red)[NSTAT], double* out) {
  if constexpr (MODE == MODE_GN) {
    tile_gn<DT, WG, ITEMS, true>(sh, pl, td, P, red, out);
  } else if constexpr (MODE == MODE_GN_NC) {
    tile_gn<DT, WG, ITEMS, false>(sh, pl, td, P, red, out);
  } else if constexpr (MODE == MODE_MOMENTS) {
    tile_moments<DT, WG, ITEMS>(sh, pl, td, red, out);
  } else {
    static_assert(MODE == MODE_COST, "unknown pass mode");
    tile_cost<DT, WG, ITEMS>(sh, pl, td, P, red, out);
  }
}

// Sum the pair's tile partials in a fixed order (lane-strided, then the fixed
// DPP tree): the same value on every run, in every lane.
__device__ inline void pair_sums(const Work& w, const PairSched& sc, int nstat, double (&s)[NSTAT]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < NSTAT; ++j) s[j] = 0.0;
  for (int t = sc.tile0 + lane; t < sc.tile0 + sc.ntiles; t += 64) {
    const double* p = w.partials + (int64_t)t * NSTAT;
#pragma unroll
    for (int j = 0; j < NSTAT; ++j)
      if (j < nstat) s[j] += p[j];
  }
  wave_totals_f64(s);
}

}  // namespace s3a
