// Point correction (Sec. III-C.3): submap points to the world frame by their
// submap's similarity, and replacement of sparse-map points by the world
// coordinates of their dense counterparts. Both are streaming / gather
// kernels bound by HBM traffic.
#include "points.h"

#include "align_kernels.h"

namespace s3a {

// One workgroup: flag[0] = 1 unless offsets are non-decreasing with
// offsets[0] >= 0 and offsets[n_sub] <= n_points.
__global__ __launch_bounds__(256) void k_check_offsets(int64_t n_points, int32_t n_sub, const int64_t* off,
                                                       int32_t* flag, int32_t* status) {
  int bad = 0;
  for (int k = (int)threadIdx.x; k < n_sub; k += 256) bad |= off[k] > off[k + 1];
  if (threadIdx.x == 0) bad |= off[0] < 0 || off[n_sub] > n_points;
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    flag[0] = bad ? 1 : 0;
    if (status) status[0] = bad ? 1 : 0;
  }
}

// Last submap k in [0, n_sub) with off[k] <= g (offsets known to be valid).
__device__ inline int find_segment(const int64_t* off, int32_t n_sub, int64_t g) {
  int lo = 0, hi = n_sub - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct SegXform {
  int64_t lo, hi;  // rows of the segment (empty when lo == hi)
  double M[9], t[3];
};

__device__ inline void load_segment(const int64_t* off, const s3a_sim3* T, int k, SegXform& s) {
  s.lo = off[k];
  s.hi = off[k + 1];
  const double sc = T[k].s;
#pragma unroll
  for (int i = 0; i < 9; ++i) s.M[i] = sc * T[k].R[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) s.t[i] = T[k].t[i];
}

template <int DT>
struct Xyz;

template <>
struct Xyz<S3A_F32> {
  static constexpr int VEC = 4;
  __device__ static inline void load(const void* const* pl, int64_t g0, int64_t n, float (&v)[3][4]) {
    if (g0 + 4 <= n) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const s3a_f4 x = __builtin_nontemporal_load((const S3A_GLOBAL s3a_f4*)(static_cast<const float*>(pl[j]) + g0));
        v[j][0] = x.x; v[j][1] = x.y; v[j][2] = x.z; v[j][3] = x.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[j][e] = (g0 + e < n) ? static_cast<const float*>(pl[j])[g0 + e] : 0.0f;
    }
  }
};

template <>
struct Xyz<S3A_BF16> {
  static constexpr int VEC = 8;
  __device__ static inline void load(const void* const* pl, int64_t g0, int64_t n, float (&v)[3][8]) {
    if (g0 + 8 <= n) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const s3a_u4 x = __builtin_nontemporal_load((const S3A_GLOBAL s3a_u4*)(static_cast<const uint16_t*>(pl[j]) + g0));
        v[j][0] = __uint_as_float(x.x << 16); v[j][1] = __uint_as_float(x.x & 0xffff0000u);
        v[j][2] = __uint_as_float(x.y << 16); v[j][3] = __uint_as_float(x.y & 0xffff0000u);
        v[j][4] = __uint_as_float(x.z << 16); v[j][5] = __uint_as_float(x.z & 0xffff0000u);
        v[j][6] = __uint_as_float(x.w << 16); v[j][7] = __uint_as_float(x.w & 0xffff0000u);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[j][e] = (g0 + e < n) ? __uint_as_float((uint32_t)static_cast<const uint16_t*>(pl[j])[g0 + e] << 16) : 0.0f;
    }
  }
};

// VEC consecutive rows per thread; the workgroup's first row locates its
// submap once (shared), and a thread searches again only for rows past that
// submap's end. World coordinates in FP64, rounded once to FP32.
template <int DT>
__global__ __launch_bounds__(256) void k_transform(int64_t n, int32_t n_sub, const int64_t* __restrict__ off,
                                                   const s3a_sim3* __restrict__ T, const void* x, const void* y,
                                                   const void* z, float* ox, float* oy, float* oz,
                                                   const int32_t* __restrict__ flag) {
  constexpr int VEC = Xyz<DT>::VEC;
  __shared__ int seg0;
  const int64_t first = (int64_t)blockIdx.x * 256 * VEC;
  const bool bad = __builtin_amdgcn_readfirstlane(flag[0]) != 0;
  if (threadIdx.x == 0) seg0 = (!bad && n_sub > 0) ? find_segment(off, n_sub, first) : -1;
  __syncthreads();
  const int64_t g0 = first + (int64_t)threadIdx.x * VEC;
  if (g0 >= n) return;
  const void* pl[3] = {x, y, z};
  float v[3][VEC];
  Xyz<DT>::load(pl, g0, n, v);
  float o[3][VEC];
  if (bad) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) o[0][e] = o[1][e] = o[2][e] = __builtin_nanf("");
  } else {
    SegXform s;
    int k = seg0;
    if (k >= 0) load_segment(off, T, k, s);
    else s.lo = s.hi = 0;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t g = g0 + e;
      if (k >= 0 && g >= s.hi && k + 1 < n_sub) {  // a later submap (rows only grow within a thread)
        k = find_segment(off, n_sub, g);
        load_segment(off, T, k, s);
      }
      if (k >= 0 && g >= s.lo && g < s.hi) {
        const double px = v[0][e], py = v[1][e], pz = v[2][e];
#pragma unroll
        for (int i = 0; i < 3; ++i)
          o[i][e] = (float)fma(s.M[3 * i], px, fma(s.M[3 * i + 1], py, fma(s.M[3 * i + 2], pz, s.t[i])));
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) o[i][e] = v[i][e];
      }
    }
  }
  float* out[3] = {ox, oy, oz};
  if (g0 + VEC <= n) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int e = 0; e < VEC; e += 4) {
        const s3a_f4 w = {o[i][e], o[i][e + 1], o[i][e + 2], o[i][e + 3]};
        __builtin_nontemporal_store(w, (S3A_GLOBAL s3a_f4*)(out[i] + g0 + e));
      }
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (g0 + e < n) out[i][g0 + e] = o[i][e];
  }
}

__global__ __launch_bounds__(256) void k_correct(int64_t n_corr, const int64_t* __restrict__ src,
                                                 const int64_t* __restrict__ dst, int64_t n_world,
                                                 const float* __restrict__ wx, const float* __restrict__ wy,
                                                 const float* __restrict__ wz, int64_t n_sparse, float* sx, float* sy,
                                                 float* sz, unsigned long long* skipped) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n_corr) return;
  const int64_t s = src[m], d = dst[m];
  if (s >= 0 && s < n_world && d >= 0 && d < n_sparse) {
    sx[d] = wx[s];
    sy[d] = wy[s];
    sz[d] = wz[s];
  } else if (skipped) {
    atomicAdd(skipped, 1ull);
  }
}

hipError_t launch_check_offsets(int64_t n, int32_t n_sub, const int64_t* off, int32_t* flag, int32_t* status,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_check_offsets, dim3(1), dim3(256), 0, st, n, n_sub, off, flag, status);
  return hipGetLastError();
}

hipError_t launch_transform(int dtype, int64_t n, int32_t n_sub, const int64_t* off, const s3a_sim3* T,
                            const void* x, const void* y, const void* z, float* ox, float* oy, float* oz,
                            const int32_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int vec = dtype == S3A_F32 ? 4 : 8;
  const int64_t grid = (n + 256 * vec - 1) / (256 * vec);
  if (dtype == S3A_F32)
    hipLaunchKernelGGL(k_transform<S3A_F32>, dim3((unsigned)grid), dim3(256), 0, st, n, n_sub, off, T, x, y, z, ox,
                       oy, oz, flag);
  else
    hipLaunchKernelGGL(k_transform<S3A_BF16>, dim3((unsigned)grid), dim3(256), 0, st, n, n_sub, off, T, x, y, z, ox,
                       oy, oz, flag);
  return hipGetLastError();
}

hipError_t launch_correct(int64_t n_corr, const int64_t* src, const int64_t* dst, int64_t n_world, const float* wx,
                          const float* wy, const float* wz, int64_t n_sparse, float* sx, float* sy, float* sz,
                          unsigned long long* skipped, hipStream_t st) {
  if (n_corr == 0) return hipSuccess;
  const int64_t grid = (n_corr + 255) / 256;
  hipLaunchKernelGGL(k_correct, dim3((unsigned)grid), dim3(256), 0, st, n_corr, src, dst, n_world, wx, wy, wz, n_sparse,
                     sx, sy, sz, skipped);
  return hipGetLastError();
}

}  // namespace s3a
