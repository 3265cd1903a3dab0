// Fused filter SpMM for gfx950: one degree of the polynomial accelerator
// (the loop body of Algorithm 7, and the plain products A*X of the Krylov
// augmentation [X, AX, ..., A^p X] of eq. S:ARR):
//
//   Yout = alpha * A * Yin + beta * Yin + gamma * Z
//
// Design (HBM-bound, about 1.5 flop per byte):
//  * one 64-lane wavefront per CSR row; the row's (col, val) entries are
//    wave-uniform, so they come through the scalar cache; lane l owns columns
//    l, l+64, l+128, ... of the row-major blocks, so every gathered Yin row is
//    read as full, contiguous 64-element segments (coalesced for any width and
//    any leading dimension);
//  * the recurrence (beta*Yin + gamma*Z) is applied in the epilogue, so a
//    degree makes exactly one pass over Yin (gathered), Z and Yout;
//  * optional epilogue: per-workgroup column sums of squares of Yout in FP64,
//    reduced later in a fixed order (deterministic column norms for the
//    multi-power normalization);
//  * XCD-aware row order: workgroup b runs on XCD b % 8; rows are dealt to the
//    XCDs in chunks of kRowChunk so stencil neighbours (i +- 1, i +- m) are
//    mostly gathered by waves of the same XCD (its L2), while all XCDs sweep
//    the matrix together (small working set in the shared Infinity Cache).
#include <algorithm>

#include "common.h"

namespace arr {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kXcd = 8;
constexpr int64_t kRowChunk = 64;

template <typename T>
__device__ __forceinline__ T ld_masked(const T *p, int c, int w) {
  return c < w ? p[c] : T(0);
}

// Row assigned to the k-th slot of XCD x.
__device__ __forceinline__ int64_t xcd_row(int64_t k, int x) {
  return (x + kXcd * (k / kRowChunk)) * kRowChunk + (k % kRowChunk);
}

template <typename T, int NJ>
__global__ __launch_bounds__(kThreads) void k_filter_spmm(
    int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const T *__restrict__ val, int w, const T *__restrict__ Yin, int64_t ldy, const T *Z, int64_t ldz,
    T *Yout, int64_t ldo, T alpha, T beta, T gamma, double *__restrict__ partial, int wtot, int c0) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = blockIdx.x % kXcd;
  const int64_t wave_in_xcd = (int64_t)(blockIdx.x / kXcd) * kWaves + wv;
  const int64_t waves_per_xcd = (int64_t)(gridDim.x / kXcd) * kWaves;

  double ss[NJ];
#pragma unroll
  for (int t = 0; t < NJ; ++t) ss[t] = 0.0;

  for (int64_t k = wave_in_xcd;; k += waves_per_xcd) {
    const int64_t i = xcd_row(k, x);
    if (i >= n) break;
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    T acc[NJ];
#pragma unroll
    for (int t = 0; t < NJ; ++t) acc[t] = T(0);
    int64_t p = b;
    for (; p + 4 <= e; p += 4) {
      const int64_t j0 = col[p], j1 = col[p + 1], j2 = col[p + 2], j3 = col[p + 3];
      const T a0 = val[p], a1 = val[p + 1], a2 = val[p + 2], a3 = val[p + 3];
      const T *r0 = Yin + j0 * ldy, *r1 = Yin + j1 * ldy, *r2 = Yin + j2 * ldy, *r3 = Yin + j3 * ldy;
      T v0[NJ], v1[NJ], v2[NJ], v3[NJ];
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        const int c = lane + 64 * t;
        v0[t] = ld_masked(r0, c, w);
        v1[t] = ld_masked(r1, c, w);
        v2[t] = ld_masked(r2, c, w);
        v3[t] = ld_masked(r3, c, w);
      }
#pragma unroll
      for (int t = 0; t < NJ; ++t) {
        acc[t] = fma(a0, v0[t], acc[t]);
        acc[t] = fma(a1, v1[t], acc[t]);
        acc[t] = fma(a2, v2[t], acc[t]);
        acc[t] = fma(a3, v3[t], acc[t]);
      }
    }
    for (; p < e; ++p) {
      const int64_t j0 = col[p];
      const T a0 = val[p];
      const T *r0 = Yin + j0 * ldy;
#pragma unroll
      for (int t = 0; t < NJ; ++t) acc[t] = fma(a0, ld_masked(r0, lane + 64 * t, w), acc[t]);
    }
    const T *yi = Yin + i * ldy;
    const T *zi = Z ? Z + i * ldz : nullptr;
    T *oi = Yout + i * ldo;
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
      const int c = lane + 64 * t;
      if (c < w) {
        T o = alpha * acc[t];
        if (beta != T(0)) o = fma(beta, yi[c], o);
        if (zi) o = fma(gamma, zi[c], o);
        oi[c] = o;
        ss[t] = fma((double)o, (double)o, ss[t]);
      }
    }
  }

  if (partial) {
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
}

template <typename T>
__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col, const T *__restrict__ val,
                                              const T *__restrict__ x, T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = T(0);
  for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s = fma(val[p], x[col[p]], s);
  y[i] = s;
}

template <typename T, int NJ>
void launch_nj(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, int w, int c0, T alpha,
               T beta, T gamma, double *partial, int wtot, int groups, hipStream_t s) {
  hipLaunchKernelGGL((k_filter_spmm<T, NJ>), dim3(groups), dim3(kThreads), 0, s, A.n, A.rowptr, A.col,
                     A.val, w, Yin.p + c0, Yin.ld, Z.p ? Z.p + c0 : nullptr, Z.ld, Yout.p + c0, Yout.ld,
                     alpha, beta, gamma, partial, wtot, c0);
}

}  // namespace

SpmmTimer *&spmm_timer() {
  static thread_local SpmmTimer *t = nullptr;
  return t;
}

hipEvent_t SpmmTimer::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  ARR_HIP(hipEventCreate(&e));
  return e;
}

void SpmmTimer::flush() {
  for (Pending &p : pending) {
    ARR_HIP(hipEventSynchronize(p.b));
    float t = 0.f;
    ARR_HIP(hipEventElapsedTime(&t, p.a, p.b));
    launches[p.cls] += 1;
    ms[p.cls] += t;
    bytes[p.cls] += p.bytes;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void SpmmTimer::reset() {
  flush();
  for (int i = 0; i < kClasses; ++i) launches[i] = 0, ms[i] = 0, bytes[i] = 0;
}

SpmmTimer::~SpmmTimer() {
  for (Pending &p : pending) pool.push_back(p.a), pool.push_back(p.b);
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

int spmm_groups(int64_t n) {
  // 8 workgroups of 4 waves per CU on 256 CUs; a multiple of the XCD count.
  int64_t need = (n + kWaves - 1) / kWaves;
  int64_t g = std::min<int64_t>(need, 2048);
  g = std::max<int64_t>(kXcd, (g + kXcd - 1) / kXcd * kXcd);
  return (int)g;
}

template <typename T>
int launch_filter_spmm(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, double alpha,
                       double beta, double gamma, double *partial, hipStream_t s) {
  const int w = Yout.w;
  ARR_REQUIRE(Yin.w >= w && (!Z.p || Z.w >= w), "filter_spmm: block widths differ");
  ARR_REQUIRE(Yin.p != Yout.p, "filter_spmm: Yout must not alias Yin");
  const int groups = spmm_groups(A.n);
  if (A.n == 0 || w == 0) return groups;
  SpmmTimer *timer = spmm_timer();
  // Column chunks of at most 1024 (16 slots per lane).
  for (int c0 = 0; c0 < w; c0 += 1024) {
    const int wc = std::min(1024, w - c0);
    const T al = (T)alpha, be = (T)beta, ga = (T)gamma;
    const int cls = (wc <= 64 ? 0 : wc <= 128 ? 1 : wc <= 256 ? 2 : wc <= 512 ? 3 : 4) + (sizeof(T) == 8 ? 5 : 0);
    SpmmTimer::Pending pend{};
    if (timer) {
      pend.a = timer->get();
      pend.b = timer->get();
      pend.cls = cls;
      // algorithmic bytes: CSR once, gathered Yin once, Z, Yout
      pend.bytes = (double)(sizeof(T) + 4) * A.nnz + 8.0 * (A.n + 1) +
                   (double)sizeof(T) * A.n * wc * (2.0 + (Z.p ? 1.0 : 0.0));
      ARR_HIP(hipEventRecord(pend.a, s));
    }
    if (wc <= 64)
      launch_nj<T, 1>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    else if (wc <= 128)
      launch_nj<T, 2>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    else if (wc <= 256)
      launch_nj<T, 4>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    else if (wc <= 512)
      launch_nj<T, 8>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    else
      launch_nj<T, 16>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    if (timer) {
      ARR_HIP(hipEventRecord(pend.b, s));
      timer->pending.push_back(pend);
    }
  }
  ARR_HIP(hipGetLastError());
  return groups;
}

template <typename T>
void launch_spmv(const DevCSR<T> &A, const T *x, T *y, hipStream_t s) {
  if (A.n == 0) return;
  const int64_t blocks = (A.n + 255) / 256;
  hipLaunchKernelGGL((k_spmv<T>), dim3((unsigned)blocks), dim3(256), 0, s, A.n, A.rowptr, A.col, A.val, x, y);
  ARR_HIP(hipGetLastError());
}

template int launch_filter_spmm<double>(const DevCSR<double> &, Blk<const double>, Blk<const double>,
                                        Blk<double>, double, double, double, double *, hipStream_t);
template int launch_filter_spmm<float>(const DevCSR<float> &, Blk<const float>, Blk<const float>, Blk<float>,
                                       double, double, double, double *, hipStream_t);
template void launch_spmv<double>(const DevCSR<double> &, const double *, double *, hipStream_t);
template void launch_spmv<float>(const DevCSR<float> &, const float *, float *, hipStream_t);

}  // namespace arr
