// Fused filter SpMM for gfx950: one degree of the polynomial accelerator
// (the loop body of Algorithm 7, and the plain products A*X of the Krylov
// augmentation [X, AX, ..., A^p X] of eq. S:ARR):
//
//   Yout = alpha * A * Yin + beta * Yin + gamma * Z
//
// Design (about 1.5 flop per byte; bound by the memory system):
//  * matrix format: the three central diagonals (band: dl, dd, du) are split
//    off the CSR at set-up; the CSR keeps the remaining ("far") entries. A
//    wave visits a run of kRun consecutive rows and keeps Yin rows i-1, i,
//    i+1 in a register window, so the band and the beta*Yin term cost one
//    new Yin row per output row instead of four gathered ones;
//  * one 64-lane wavefront per row; the far (col, val) entries are
//    wave-uniform (scalar cache); lane l owns columns l, l+64, ... of the
//    row-major blocks (FP32 blocks with 16-byte aligned rows: 4 consecutive
//    columns per lane, one 16-byte load), so every gathered Yin row is read
//    as full, contiguous segments;
//  * the recurrence (beta*Yin + gamma*Z) is applied in the epilogue, so a
//    degree makes exactly one pass over Yin (gathered), Z and Yout;
//  * optional epilogue: per-workgroup column sums of squares of Yout in FP64,
//    reduced later in a fixed order (deterministic column norms for the
//    multi-power normalization);
//  * XCD-aware order: workgroup b runs on XCD b % 8; runs are dealt to the
//    XCDs in chunks of kRunChunk so stencil neighbours are mostly gathered by
//    waves of the same XCD (its L2), while all XCDs sweep the matrix together
//    (small working set in the shared Infinity Cache).
#include <algorithm>
#include <exception>

#include "common.h"

namespace arr {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kXcd = 8;
constexpr int64_t kRun = 8;       // consecutive rows per wave visit
constexpr int64_t kRunChunk = 8;  // runs per XCD chunk
constexpr int kMaxGroups = 1024;  // 4 waves per SIMD on 256 CUs

template <typename T, int V>
struct VecT {
  typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VecT<T, 1> {
  typedef T type;
};

template <int V, typename X>
__device__ __forceinline__ double lane_elem(const X &x, int v) {
  if constexpr (V == 1)
    return (double)x;
  else
    return (double)x[v];
}

// Run assigned to the k-th slot of XCD x.
__device__ __forceinline__ int64_t xcd_run(int64_t k, int x) {
  return (x + kXcd * (k / kRunChunk)) * kRunChunk + (k % kRunChunk);
}

template <typename T, int VEC, int NT>
__global__ __launch_bounds__(kThreads) void k_filter_spmm(
    int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const T *__restrict__ val, const T *__restrict__ band, int w, const T *__restrict__ Yin, int64_t ldy,
    const T *Z, int64_t ldz, T *Yout, int64_t ldo, T alpha, T beta, T gamma, double *__restrict__ partial,
    int wtot, int c0) {
  typedef typename VecT<T, VEC>::type vec;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = blockIdx.x % kXcd;
  const int64_t wave_in_xcd = (int64_t)(blockIdx.x / kXcd) * kWaves + wv;
  const int64_t waves_per_xcd = (int64_t)(gridDim.x / kXcd) * kWaves;
  const int64_t nruns = (n + kRun - 1) / kRun;
  const T *dl = band, *dd = band + n, *du = band + 2 * n;
  auto ld = [&](const T *row, int t) -> vec {
    const int c = VEC * lane + 64 * VEC * t;
    return c < w ? *(const vec *)(row + c) : vec(0);
  };

  double ss[NT][VEC];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < VEC; ++v) ss[t][v] = 0.0;

  for (int64_t k = wave_in_xcd;; k += waves_per_xcd) {
    const int64_t r = xcd_run(k, x);
    if (r >= nruns) break;
    const int64_t i0 = r * kRun, iend = min(n, i0 + kRun);
    vec wm[NT], w0[NT], wp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      wm[t] = i0 > 0 ? ld(Yin + (i0 - 1) * ldy, t) : vec(0);
      w0[t] = ld(Yin + i0 * ldy, t);
      wp[t] = i0 + 1 < n ? ld(Yin + (i0 + 1) * ldy, t) : vec(0);
    }
    for (int64_t i = i0; i < iend; ++i) {
      // next window row, in flight while this row is gathered
      vec nx[NT];
      const bool more = i + 1 < iend && i + 2 < n;
#pragma unroll
      for (int t = 0; t < NT; ++t) nx[t] = more ? ld(Yin + (i + 2) * ldy, t) : vec(0);
      const T al = dl[i], ad = dd[i], au = du[i];
      vec acc[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = al * wm[t] + ad * w0[t] + au * wp[t];
      const int64_t b = rowptr[i], e = rowptr[i + 1];
      int64_t p = b;
      for (; p + 4 <= e; p += 4) {
        const int64_t j0 = col[p], j1 = col[p + 1], j2 = col[p + 2], j3 = col[p + 3];
        const T a0 = val[p], a1 = val[p + 1], a2 = val[p + 2], a3 = val[p + 3];
        vec v0[NT], v1[NT], v2[NT], v3[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          v0[t] = ld(Yin + j0 * ldy, t);
          v1[t] = ld(Yin + j1 * ldy, t);
          v2[t] = ld(Yin + j2 * ldy, t);
          v3[t] = ld(Yin + j3 * ldy, t);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] += a0 * v0[t] + a1 * v1[t] + a2 * v2[t] + a3 * v3[t];
      }
      for (; p < e; ++p) {
        const int64_t j0 = col[p];
        const T a0 = val[p];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] += a0 * ld(Yin + j0 * ldy, t);
      }
      const T *zi = Z ? Z + i * ldz : nullptr;
      T *oi = Yout + i * ldo;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = VEC * lane + 64 * VEC * t;
        if (c < w) {
          vec o = alpha * acc[t];
          if (beta != T(0)) o += beta * w0[t];
          if constexpr (VEC == 1) {
            // Z and Yout are touched once per launch: streaming hints keep
            // them from displacing gathered Yin rows in L2
            if (zi) o += gamma * __builtin_nontemporal_load(zi + c);
            __builtin_nontemporal_store(o, oi + c);
          } else {
            if (zi) o += gamma * *(const vec *)(zi + c);
            *(vec *)(oi + c) = o;
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const double ov = lane_elem<VEC>(o, v);
            ss[t][v] = fma(ov, ov, ss[t][v]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        wm[t] = w0[t];
        w0[t] = wp[t];
        wp[t] = nx[t];
      }
    }
  }

  if (partial) {
    __shared__ double red[kWaves][64 * VEC * NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < VEC; ++v) red[wv][VEC * lane + 64 * VEC * t + v] = ss[t][v];
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
                                              const T *__restrict__ band, const T *__restrict__ x,
                                              T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = band[n + i] * x[i];
  if (i > 0) s = fma(band[i], x[i - 1], s);
  if (i + 1 < n) s = fma(band[2 * n + i], x[i + 1], s);
  for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s = fma(val[p], x[col[p]], s);
  y[i] = s;
}

template <typename T, int VEC, int NT>
void launch_nt(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, int w, int c0, T alpha,
               T beta, T gamma, double *partial, int wtot, int groups, hipStream_t s) {
  hipLaunchKernelGGL((k_filter_spmm<T, VEC, NT>), dim3(groups), dim3(kThreads), 0, s, A.n, A.rowptr, A.col,
                     A.val, A.band, w, Yin.p + c0, Yin.ld, Z.p ? Z.p + c0 : nullptr, Z.ld, Yout.p + c0, Yout.ld,
                     alpha, beta, gamma, partial, wtot, c0);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

SpmmTimer *&spmm_timer() {
  static thread_local SpmmTimer *t = nullptr;
  return t;
}

SpmmTimer *&gemm_timer() {
  static thread_local SpmmTimer *t = nullptr;
  return t;
}

SpmmTimer::Scope::Scope(SpmmTimer *t_, int cls, double work, hipStream_t s_) : t(t_), s(s_) {
  if (!t) return;
  p.a = t->get();
  p.b = t->get();
  p.cls = cls;
  p.bytes = work;
  ARR_HIP(hipEventRecord(p.a, s));
}

SpmmTimer::Scope::~Scope() {
  if (!t) return;
  // a launch that failed leaves the pair unrecorded: it is returned unused
  if (hipEventRecord(p.b, s) == hipSuccess && !std::uncaught_exceptions()) {
    try {
      t->pending.push_back(p);
      return;
    } catch (...) {
    }
  }
  t->pool.push_back(p.a);
  t->pool.push_back(p.b);
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
  // one wave per run, at most kMaxGroups workgroups; a multiple of the XCD count
  const int64_t runs = (n + kRun - 1) / kRun;
  int64_t g = std::min<int64_t>((runs + kWaves - 1) / kWaves, kMaxGroups);
  g = std::max<int64_t>(kXcd, (g + kXcd - 1) / kXcd * kXcd);
  return (int)g;
}

void split_band(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, std::vector<int64_t> &frp,
                std::vector<int32_t> &fcol, std::vector<double> &fval, std::vector<double> &band) {
  frp.assign(n + 1, 0);
  fcol.clear();
  fval.clear();
  band.assign(3 * n, 0.0);
  const int64_t nnz = rowptr[n];
  fcol.reserve(nnz);
  fval.reserve(nnz);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      const int64_t j = col[q];
      if (j == i - 1)
        band[i] = val[q];
      else if (j == i)
        band[n + i] = val[q];
      else if (j == i + 1)
        band[2 * n + i] = val[q];
      else {
        fcol.push_back((int32_t)j);
        fval.push_back(val[q]);
      }
    }
    frp[i + 1] = (int64_t)fcol.size();
  }
}

template <typename T>
int launch_filter_spmm(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, double alpha,
                       double beta, double gamma, double *partial, hipStream_t s) {
  const int w = Yout.w;
  ARR_REQUIRE(Yin.w >= w && (!Z.p || Z.w >= w), "filter_spmm: block widths differ");
  ARR_REQUIRE(Yin.p != Yout.p, "filter_spmm: Yout must not alias Yin");
  ARR_REQUIRE(A.n == 0 || A.band, "filter_spmm: matrix band missing");
  const int groups = spmm_groups(A.n);
  if (A.n == 0 || w == 0) return groups;
  SpmmTimer *timer = spmm_timer();
  // FP32 with 16-byte aligned rows: 4 consecutive columns per lane
  const bool vec4 = sizeof(T) == 4 && Yin.ld % 4 == 0 && Yout.ld % 4 == 0 && (!Z.p || Z.ld % 4 == 0) &&
                    aligned16(Yin.p) && aligned16(Yout.p) && (!Z.p || aligned16(Z.p)) && w % 4 == 0;
  // Column chunks of at most 1024 (16 slots per lane).
  for (int c0 = 0; c0 < w; c0 += 1024) {
    const int wc = std::min(1024, w - c0);
    const T al = (T)alpha, be = (T)beta, ga = (T)gamma;
    const int slots = vec4 ? 4 * ((wc + 255) / 256) : (wc + 63) / 64;  // columns per lane
    const int cls = (slots <= 1 ? 0 : slots <= 2 ? 1 : slots <= 4 ? 2 : slots <= 8 ? 3 : 4) + (vec4 ? 5 : 0) +
                    (sizeof(T) == 8 ? 10 : 0);
    SpmmTimer::Pending pend{};
    if (timer) {
      pend.a = timer->get();
      pend.b = timer->get();
      pend.cls = cls;
      // algorithmic bytes: the matrix once (CSR of all its entries), gathered
      // Yin once, Z, Yout
      pend.bytes = (double)(sizeof(T) + 4) * A.nnz + 8.0 * (A.n + 1) +
                   (double)sizeof(T) * A.n * wc * (2.0 + (Z.p ? 1.0 : 0.0));
      ARR_HIP(hipEventRecord(pend.a, s));
    }
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (vec4) {
        if (wc <= 256)
          launch_nt<T, 4, 1>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
        else if (wc <= 512)
          launch_nt<T, 4, 2>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
        else
          launch_nt<T, 4, 4>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
        done = true;
      }
    }
    if (done) {
    } else if (wc <= 64) {
      launch_nt<T, 1, 1>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    } else if (wc <= 128) {
      launch_nt<T, 1, 2>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    } else if (wc <= 256) {
      launch_nt<T, 1, 4>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    } else if (wc <= 512) {
      launch_nt<T, 1, 8>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    } else {
      launch_nt<T, 1, 16>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, s);
    }
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
  hipLaunchKernelGGL((k_spmv<T>), dim3((unsigned)blocks), dim3(256), 0, s, A.n, A.rowptr, A.col, A.val, A.band, x,
                     y);
  ARR_HIP(hipGetLastError());
}

template int launch_filter_spmm<double>(const DevCSR<double> &, Blk<const double>, Blk<const double>,
                                        Blk<double>, double, double, double, double *, hipStream_t);
template int launch_filter_spmm<float>(const DevCSR<float> &, Blk<const float>, Blk<const float>, Blk<float>,
                                       double, double, double, double *, hipStream_t);
template void launch_spmv<double>(const DevCSR<double> &, const double *, double *, hipStream_t);
template void launch_spmv<float>(const DevCSR<float> &, const float *, float *, hipStream_t);

}  // namespace arr
