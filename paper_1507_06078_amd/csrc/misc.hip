// Element-wise and column-wise block kernels: column sums of squares (norms
// for the multi-power normalization of Sec. 3 and residuals of eq. resi),
// deterministic reduction of per-workgroup partials, column scaling, column
// gathers (merging converged and new Ritz vectors, Sec. 6 deflation), dtype
// conversion (mixed precision), fills and the starting Gaussian block.
#include <algorithm>

#include "common.h"

namespace arr {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

template <typename T, int NJ>
__global__ __launch_bounds__(kThreads) void k_colsumsq(int64_t n, int w, const T *__restrict__ P, int64_t ldp,
                                                        const T *__restrict__ Q, int64_t ldq,
                                                        const double *__restrict__ mu, double *__restrict__ partial,
                                                        int wtot, int c0) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double ss[NJ], m[NJ];
#pragma unroll
  for (int t = 0; t < NJ; ++t) {
    ss[t] = 0.0;
    const int c = lane + 64 * t;
    m[t] = (Q && c < w) ? mu[c0 + c] : 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * kWaves + wv; i < n; i += (int64_t)gridDim.x * kWaves) {
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
      const int c = lane + 64 * t;
      if (c < w) {
        double v = (double)P[i * ldp + c];
        if (Q) v -= m[t] * (double)Q[i * ldq + c];
        ss[t] = fma(v, v, ss[t]);
      }
    }
  }
  __shared__ double red[kWaves][64 * NJ];
#pragma unroll
  for (int t = 0; t < NJ; ++t) red[wv][lane + 64 * t] = ss[t];
  __syncthreads();
  for (int c = threadIdx.x; c < w; c += kThreads) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) s += red[q][c];
    partial[(int64_t)blockIdx.x * wtot + c0 + c] = s;
  }
}

// One workgroup per column: strided partial sums then a fixed-shape tree.
__global__ __launch_bounds__(256) void k_reduce_groups(const double *__restrict__ partial, int groups, int w,
                                                       double *__restrict__ out, int take_sqrt) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int g = threadIdx.x; g < groups; g += 256) s += partial[(int64_t)g * w + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = take_sqrt ? sqrt(red[0]) : red[0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale_columns(int64_t n, int w, T *X, int64_t ld,
                                                       const double *__restrict__ scale, int inv_sqrt) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nw) {
    for (int c = lane; c < w; c += 64) {
      const double sc = inv_sqrt ? 1.0 / sqrt(scale[c]) : scale[c];
      X[i * ld + c] = (T)((double)X[i * ld + c] * sc);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_columns(int64_t n, int w, T *__restrict__ dst, int64_t lddst,
                                                        const T *const *__restrict__ srcs,
                                                        const int64_t *__restrict__ lds,
                                                        const int32_t *__restrict__ cols) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nw)
    for (int j = lane; j < w; j += 64) dst[i * lddst + j] = srcs[j][i * lds[j] + cols[j]];
}

template <typename TD, typename TS>
__global__ __launch_bounds__(256) void k_convert(int64_t n, int w, TD *__restrict__ dst, int64_t lddst,
                                                 const TS *__restrict__ src, int64_t ldsrc) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < n; i += nw)
    for (int c = lane; c < w; c += 64) dst[i * lddst + c] = (TD)src[i * ldsrc + c];
}

template <typename T>
__global__ void k_fill(T *p, int64_t count, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): 10 rounds of
// (hi, lo) = mulhilo(M, c) on counter words 0 and 2, mixed with the key,
// the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k0 += W0;
    k1 += W1;
  }
}

__global__ __launch_bounds__(256) void k_gaussian(int64_t n, int w, double *X, int64_t ld, uint32_t k0,
                                                  uint32_t k1) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * w) return;
  const int64_t i = idx / w;
  const int j = (int)(idx % w);
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)j, 0u};
  philox4x32_10(c, k0, k1);
  // two 53-bit uniforms in (0, 1], then Box-Muller
  const double u1 = ((double)(((uint64_t)(c[0] >> 5) << 26) | (c[1] >> 6)) + 1.0) * (1.0 / 9007199254740992.0);
  const double u2 = ((double)(((uint64_t)(c[2] >> 5) << 26) | (c[3] >> 6))) * (1.0 / 9007199254740992.0);
  X[i * ld + j] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

int rows_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 3) / 4, 4096)); }

template <typename T, int NJ>
void colsumsq_nj(int64_t n, Blk<const T> P, Blk<const T> Q, const double *mu, double *partial, int wc, int c0,
                 int wtot, int groups, hipStream_t s) {
  hipLaunchKernelGGL((k_colsumsq<T, NJ>), dim3(groups), dim3(kThreads), 0, s, n, wc, P.p + c0, P.ld,
                     Q.p ? Q.p + c0 : nullptr, Q.ld, mu, partial, wtot, c0);
}

}  // namespace

Pool *&device_pool() {
  static thread_local Pool *p = nullptr;
  return p;
}

template <typename T>
int launch_colsumsq(int64_t n, Blk<const T> P, Blk<const T> Q, const double *mu, double *partial, hipStream_t s) {
  const int w = P.w;
  const int groups = spmm_groups(n);
  if (w == 0) return groups;
  for (int c0 = 0; c0 < w; c0 += 1024) {
    const int wc = std::min(1024, w - c0);
    if (wc <= 64)
      colsumsq_nj<T, 1>(n, P, Q, mu, partial, wc, c0, w, groups, s);
    else if (wc <= 128)
      colsumsq_nj<T, 2>(n, P, Q, mu, partial, wc, c0, w, groups, s);
    else if (wc <= 256)
      colsumsq_nj<T, 4>(n, P, Q, mu, partial, wc, c0, w, groups, s);
    else if (wc <= 512)
      colsumsq_nj<T, 8>(n, P, Q, mu, partial, wc, c0, w, groups, s);
    else
      colsumsq_nj<T, 16>(n, P, Q, mu, partial, wc, c0, w, groups, s);
  }
  ARR_HIP(hipGetLastError());
  return groups;
}

void launch_reduce_groups(const double *partial, int groups, int w, double *out, bool take_sqrt, hipStream_t s) {
  if (w == 0) return;
  hipLaunchKernelGGL(k_reduce_groups, dim3(w), dim3(256), 0, s, partial, groups, w, out, take_sqrt ? 1 : 0);
  ARR_HIP(hipGetLastError());
}

template <typename T>
void launch_scale_columns(int64_t n, Blk<T> X, const double *scale, bool inv_sqrt, hipStream_t s) {
  if (n == 0 || X.w == 0) return;
  hipLaunchKernelGGL((k_scale_columns<T>), dim3(rows_grid(n)), dim3(256), 0, s, n, X.w, X.p, X.ld, scale,
                     inv_sqrt ? 1 : 0);
  ARR_HIP(hipGetLastError());
}

template <typename T>
void launch_gather_columns(int64_t n, int w, T *dst, int64_t lddst, const T *const *srcs, const int64_t *lds,
                           const int32_t *cols, hipStream_t s) {
  if (n == 0 || w == 0) return;
  hipLaunchKernelGGL((k_gather_columns<T>), dim3(rows_grid(n)), dim3(256), 0, s, n, w, dst, lddst, srcs, lds, cols);
  ARR_HIP(hipGetLastError());
}

template <typename TD, typename TS>
void launch_convert(int64_t n, int w, TD *dst, int64_t lddst, const TS *src, int64_t ldsrc, hipStream_t s) {
  if (n == 0 || w == 0) return;
  hipLaunchKernelGGL((k_convert<TD, TS>), dim3(rows_grid(n)), dim3(256), 0, s, n, w, dst, lddst, src, ldsrc);
  ARR_HIP(hipGetLastError());
}

template <typename T>
void launch_copy(int64_t n, int w, T *dst, int64_t lddst, const T *src, int64_t ldsrc, hipStream_t s) {
  launch_convert<T, T>(n, w, dst, lddst, src, ldsrc, s);
}

template <typename T>
void launch_fill(T *p, int64_t count, T v, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
  ARR_HIP(hipGetLastError());
}

void launch_gaussian(int64_t n, int w, double *X, int64_t ld, uint64_t seed, hipStream_t s) {
  const int64_t tot = n * w;
  if (tot == 0) return;
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, w, X, ld,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  ARR_HIP(hipGetLastError());
}

template int launch_colsumsq<double>(int64_t, Blk<const double>, Blk<const double>, const double *, double *,
                                     hipStream_t);
template int launch_colsumsq<float>(int64_t, Blk<const float>, Blk<const float>, const double *, double *,
                                    hipStream_t);
template void launch_scale_columns<double>(int64_t, Blk<double>, const double *, bool, hipStream_t);
template void launch_scale_columns<float>(int64_t, Blk<float>, const double *, bool, hipStream_t);
template void launch_gather_columns<double>(int64_t, int, double *, int64_t, const double *const *,
                                            const int64_t *, const int32_t *, hipStream_t);
template void launch_gather_columns<float>(int64_t, int, float *, int64_t, const float *const *, const int64_t *,
                                           const int32_t *, hipStream_t);
template void launch_convert<double, float>(int64_t, int, double *, int64_t, const float *, int64_t, hipStream_t);
template void launch_convert<float, double>(int64_t, int, float *, int64_t, const double *, int64_t, hipStream_t);
template void launch_copy<double>(int64_t, int, double *, int64_t, const double *, int64_t, hipStream_t);
template void launch_copy<float>(int64_t, int, float *, int64_t, const float *, int64_t, hipStream_t);
template void launch_fill<int>(int *, int64_t, int, hipStream_t);
template void launch_fill<double>(double *, int64_t, double, hipStream_t);

}  // namespace arr
