// Tall-skinny dense products on the FP64 matrix cores of gfx950
// (v_mfma_f64_16x16x4f64):
//
//  * Gram  G = X^T Y   (n x mx)^T (n x my), n >> mx, my: the inner-stop Gram
//    X^T X of eq. inn-stop, the Gram of the Cholesky-QR orthonormalization
//    and the projection U^T (A U) of Algorithm 1. Split over n: each
//    workgroup reduces a chunk of rows into a 64 x 64 tile, partial tiles are
//    summed in a fixed order (deterministic, no atomics).
//  * Update Y = beta Y + alpha X W   (n x m)(m x c): Ritz vectors U V
//    (Algorithm 1), the Cholesky-QR basis Z R^-1, and the deflation
//    projection X - Qc (Qc^T X) (Sec. 6). 64 x 64 output tiles; the X tile
//    and the W tile are staged through LDS; tiles of one row band run on the
//    same XCD one after another so the band is read from HBM once.
//
// FP32 blocks are widened exactly and use the FP64 matrix cores too, unless the
// caller asks for the FP32 matrix cores for a well-conditioned product.
//
// MFMA 16x16x4 operand layout (lane l of 64): A[i][k] with i = l % 16,
// k = l / 16; B[k][j] with k = l / 16, j = l % 16. Result D[i][j] in element
// r of lane l with j = l % 16 and i = l / 16 + 4 r for FP64 but
// i = 4 (l / 16) + r for FP32 (both checked on gfx950).
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace arr {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16f(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int64_t kGramWorkCap = int64_t(1) << 24;  // doubles of split partials (128 MiB)

struct GramPlan {
  int tile, ntx, nty, ntiles, nsplit;
  int64_t chunk;
};

GramPlan gram_plan(int64_t n, int mx, int my, bool sym, int64_t work_cap = kGramWorkCap) {
  GramPlan p;
  // 128 tiles (4x the work per row of a 64 tile) once both sides reach 128
  p.tile = (mx >= 128 && my >= 128) ? 128 : 64;
  p.ntx = (mx + p.tile - 1) / p.tile;
  p.nty = (my + p.tile - 1) / p.tile;
  p.ntiles = sym ? p.ntx * (p.ntx + 1) / 2 : p.ntx * p.nty;
  // Both tile kernels fit two workgroups per CU: 512 slots. Aim at four full
  // rounds and round the split count down to whole rounds, so the last round
  // is not a nearly empty tail.
  const int64_t target = 4 * 512;
  int64_t want = std::max<int64_t>(1, target / p.ntiles);
  // the partial tiles stay within kGramWorkCap doubles (or one product)
  want = std::min<int64_t>(want, std::max<int64_t>(1, work_cap / ((int64_t)mx * my)));
  // at least 256 rows per split so each wave streams a useful amount
  want = std::min<int64_t>(want, std::max<int64_t>(1, n / 256));
  // whole rounds of the 512 slots once there is more than one
  const int64_t rounds = (int64_t)p.ntiles * want / 512;
  if (rounds >= 1) want = std::max<int64_t>(1, rounds * 512 / p.ntiles);
  p.nsplit = (int)want;
  p.chunk = round_up((n + p.nsplit - 1) / p.nsplit, 16);
  if (p.chunk == 0) p.chunk = 16;
  p.nsplit = (int)std::max<int64_t>(1, (n + p.chunk - 1) / p.chunk);
  return p;
}

// Gram tile kernel. A workgroup owns a TILE x TILE output tile (64 or 128)
// and a chunk of rows; the rows stream through double-buffered LDS, KS at a
// time (each thread moves 8 consecutive elements of X and of Y per stage), and
// wave q accumulates the (TILE/2)-square quadrant (q & 1, q >> 1) on the
// matrix cores as (TILE/32)^2 blocks of 16 x 16, so no reduction across waves
// is needed. The 128 tiles halve the loads per flop; they serve products whose
// sides are both at least 128. Products run on the FP64 matrix cores (FP32
// data are widened exactly), except in the kMma32 variant: FP32 matrix cores
// over each stage's KS rows, added into the FP64 accumulator after every
// stage. That variant is for well-conditioned products only (a Rayleigh
// quotient of an orthonormal basis), where an FP32 rounding of each slice's
// sum is harmless.
template <typename T, bool kMma32, int TILE>
__global__ __launch_bounds__(256) void k_gram(int64_t n, const T *__restrict__ X, int64_t ldx, int mx,
                                              const T *__restrict__ Y, int64_t ldy, int my, int ntx, int nty,
                                              int ntiles, int sym, int64_t chunk, double *__restrict__ part) {
  static_assert(!kMma32 || std::is_same<T, float>::value, "FP32 matrix cores need FP32 data");
  static_assert(TILE == 64 || TILE == 128, "tile is 64 or 128");
  constexpr int KS = TILE == 64 ? 32 : 16;  // rows per stage
  constexpr int FB = TILE / 32;             // 16 x 16 blocks per wave and dimension
  constexpr int HALF = TILE / 2;
  constexpr int PER = KS * TILE / 256;      // elements per thread and matrix per stage
  static_assert(PER == 8, "8 elements per thread");
  const int tile = blockIdx.x % ntiles;
  const int split = blockIdx.x / ntiles;
  int tx, ty;
  if (sym) {  // upper-triangular tile list, row-major
    int t = tile, r = 0;
    while (t >= ntx - r) { t -= ntx - r; ++r; }
    tx = r;
    ty = r + t;
  } else {
    tx = tile / nty;
    ty = tile % nty;
  }
  const int cx = tx * TILE, cy = ty * TILE;
  const int64_t r0 = (int64_t)split * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int qx = (wv & 1) * HALF, qy = (wv >> 1) * HALF;
  // thread t stages column
  // t % TILE of rows t / TILE + q * (256 / TILE): coalesced loads, and
  // consecutive lanes write consecutive LDS words
  constexpr int PAD = 1;
  __shared__ T Xs[2][KS][TILE + PAD], Ys[2][KS][TILE + PAD];
  constexpr int RSTEP = 256 / TILE;
  const int lc = tid % TILE, lr0 = tid / TILE;
  T xv[PER], yv[PER];
  auto gload = [&](int64_t rb) {
    const bool cxok = cx + lc < mx, cyok = cy + lc < my;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int64_t row = rb + lr0 + q * RSTEP;
      const bool rok = row < r1;
      xv[q] = (rok && cxok) ? X[row * ldx + cx + lc] : T(0);
      yv[q] = (rok && cyok) ? Y[row * ldy + cy + lc] : T(0);
    }
  };
  auto lstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      Xs[b][lr0 + q * RSTEP][lc] = xv[q];
      Ys[b][lr0 + q * RSTEP][lc] = yv[q];
    }
  };
  v4d acc[FB][FB];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int g = 0; g < FB; ++g) acc[f][g] = v4d{0.0, 0.0, 0.0, 0.0};
  int buf = 0;
  if (r0 < r1) {
    gload(r0);
    lstore(0);
  }
  __syncthreads();
  for (int64_t rb = r0; rb < r1; rb += KS) {
    const bool more = rb + KS < r1;
    if (more) gload(rb + KS);
    if constexpr (!kMma32) {
#pragma unroll
      for (int ks = 0; ks < KS / 4; ++ks) {
        double a[FB], b[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          a[f] = (double)Xs[buf][4 * ks + lk][qx + 16 * f + li];
          b[f] = (double)Ys[buf][4 * ks + lk][qy + 16 * f + li];
        }
#pragma unroll
        for (int f = 0; f < FB; ++f)
#pragma unroll
          for (int g = 0; g < FB; ++g) acc[f][g] = mfma16(a[f], b[g], acc[f][g]);
      }
    } else {
      v4f sl[FB][FB];
#pragma unroll
      for (int f = 0; f < FB; ++f)
#pragma unroll
        for (int g = 0; g < FB; ++g) sl[f][g] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS / 4; ++ks) {
        float a[FB], b[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
          a[f] = Xs[buf][4 * ks + lk][qx + 16 * f + li];
          b[f] = Ys[buf][4 * ks + lk][qy + 16 * f + li];
        }
#pragma unroll
        for (int f = 0; f < FB; ++f)
#pragma unroll
          for (int g = 0; g < FB; ++g) sl[f][g] = mfma16f(a[f], b[g], sl[f][g]);
      }
#pragma unroll
      for (int f = 0; f < FB; ++f)
#pragma unroll
        for (int g = 0; g < FB; ++g)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[f][g][e] += (double)sl[f][g][e];
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double *out = part + (int64_t)split * mx * my;
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int g = 0; g < FB; ++g)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // result layouts: FP64 MFMA row lk + 4e, FP32 MFMA row 4 lk + e
        const int rr = kMma32 ? 4 * lk + e : lk + 4 * e;
        const int i = cx + qx + 16 * f + rr, j = cy + qy + 16 * g + li;
        if (i < mx && j < my) out[(int64_t)i * my + j] = acc[f][g][e];
      }
}

// G[i][j] = sum_s part[s][i][j] in order; for sym, the upper element is used
// for both (i, j) and (j, i).
__global__ void k_gram_reduce(const double *__restrict__ part, int nsplit, int mx, int my, int sym,
                              double *__restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)mx * my) return;
  int i = (int)(idx / my), j = (int)(idx % my);
  if (sym && i > j) { const int t = i; i = j; j = t; }  // mirror the upper triangle exactly
  const int64_t src = (int64_t)i * my + j;
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * mx * my + src];
  G[idx] = s;
}

// Block update tile kernel: a workgroup owns a TILE x TILE tile of Y (64, or
// 128 for the FP32 matrix cores once Y has 128 columns: half the loads per
// flop) and walks k in steps of 16 through two LDS buffers: the next step is
// loaded into registers while the current one is multiplied, then stored into
// the other buffer (one barrier per step); wave q accumulates the
// (TILE/2)-square quadrant (q & 1, q >> 1).
template <typename T, bool kMma32, int TILE>
__global__ __launch_bounds__(256) void k_update(int64_t n, const T *__restrict__ X, int64_t ldx, int m,
                                                const double *__restrict__ W, int64_t ldw, int c, double alpha,
                                                double beta, T *Y, int64_t ldy, int nct, int64_t nrt, int w_upper,
                                                const double *__restrict__ colss) {
  static_assert(TILE == 64 || TILE == 128, "tile is 64 or 128");
  constexpr int FB = TILE / 32, HALF = TILE / 2;
  // tile order: XCD x gets workgroups b = x + 8 t; t walks the column tiles of
  // one row band before moving to the next band of that XCD.
  const int xcd = blockIdx.x % kXcd;
  const int64_t t = blockIdx.x / kXcd;
  const int ct = (int)(t % nct);
  const int64_t rt = (t / nct) * kXcd + xcd;
  if (rt >= nrt) return;
  const int64_t r0 = rt * TILE;
  const int c0 = ct * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int qx = (wv & 1) * HALF, qy = (wv >> 1) * HALF;
  // W upper triangular: rows k >= c0 + TILE of this column tile are zero
  const int kend = w_upper ? min(m, c0 + TILE) : m;

  // FP64 matrix cores (FP32 data widened exactly, W kept in FP64), except in
  // the kMma32 variant for FP32 data times a well-conditioned W (an
  // orthogonal Ritz rotation): W rounded to FP32, FP32 matrix cores.
  static_assert(!kMma32 || std::is_same<T, float>::value, "FP32 matrix cores need FP32 data");
  typedef typename std::conditional<kMma32, float, double>::type S;
  typedef typename std::conditional<kMma32, v4f, v4d>::type acc_t;
  constexpr int KS = 16;                 // k per stage
  constexpr int PX = TILE * KS / 256;      // X elements per thread and stage
  constexpr int PW = KS * TILE / 256;      // W elements per thread and stage
  __shared__ S Xs[2][TILE][KS + 1];
  __shared__ S Ws[2][KS][TILE + 1];

  acc_t acc[FB][FB];
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int g = 0; g < FB; ++g) acc[f][g] = acc_t{0, 0, 0, 0};

  const int xr_ = tid / (KS / PX), xk = (tid % (KS / PX)) * PX;      // X tile: TILE rows x KS k
  const int wk_ = tid / (TILE / PW), wc = (tid % (TILE / PW)) * PW;  // W tile: KS k x TILE cols
  const int64_t xrow = r0 + xr_;
  S xv[PX], wvv[PW];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int kk = k0 + xk + q;
      xv[q] = (xrow < n && kk < kend) ? (S)X[xrow * ldx + kk] : S(0);
    }
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int kw = k0 + wk_, cc = c0 + wc + q;
      wvv[q] = (kw < kend && cc < c) ? (S)W[(int64_t)kw * ldw + cc] : S(0);
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int q = 0; q < PX; ++q) Xs[b][xr_][xk + q] = xv[q];
#pragma unroll
    for (int q = 0; q < PW; ++q) Ws[b][wk_][wc + q] = wvv[q];
  };
  int buf = 0;
  if (kend > 0) {
    load(0);
    stash(0);
  }
  __syncthreads();
  for (int k0 = 0; k0 < kend; k0 += KS) {
    const bool more = k0 + KS < kend;
    if (more) load(k0 + KS);
#pragma unroll
    for (int ks = 0; ks < KS / 4; ++ks) {
      S a[FB], b[FB];
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        a[f] = Xs[buf][qx + 16 * f + li][4 * ks + lk];
        b[f] = Ws[buf][4 * ks + lk][qy + 16 * f + li];
      }
#pragma unroll
      for (int f = 0; f < FB; ++f)
#pragma unroll
        for (int g = 0; g < FB; ++g) {
          if constexpr (kMma32)
            acc[f][g] = mfma16f(a[f], b[g], acc[f][g]);
          else
            acc[f][g] = mfma16(a[f], b[g], acc[f][g]);
        }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int f = 0; f < FB; ++f)
#pragma unroll
    for (int g = 0; g < FB; ++g) {
      const int col = c0 + qy + 16 * g + li;
      if (col >= c) continue;
      const double sc = colss ? 1.0 / sqrt(colss[col]) : 1.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = r0 + qx + 16 * f + (kMma32 ? 4 * lk + e : lk + 4 * e);
        if (row >= n) continue;
        T *yp = Y + row * ldy + col;
        double v = alpha * (double)acc[f][g][e];
        if (beta != 0.0) v += beta * (double)(*yp);
        if (colss) v *= sc;
        *yp = (T)v;
      }
    }
}

}  // namespace

size_t gram_work_bound(int64_t n, int m_max) {
  // nsplit * mx * my <= max(kGramWorkCap, mx * my) by the cap in gram_plan,
  // and nsplit <= max(1, n / 256).
  const size_t mm = (size_t)m_max * (size_t)m_max;
  const size_t by_cap = std::max<size_t>((size_t)kGramWorkCap, mm);
  const size_t by_rows = (size_t)std::max<int64_t>(1, n / 256) * mm;
  return std::min(by_cap, by_rows);
}

size_t gram_work_doubles(int64_t n, int mx, int my) {
  // the symmetric plan applies to square products only (launch_gram requires it)
  const GramPlan p = gram_plan(n, mx, my, false);
  int nsplit = p.nsplit;
  if (mx == my) nsplit = std::max(nsplit, gram_plan(n, mx, my, true).nsplit);
  return (size_t)nsplit * (size_t)mx * (size_t)my;
}

template <typename T>
void launch_gram(int64_t n, Blk<const T> X, Blk<const T> Y, double *G, double *work, bool sym, hipStream_t s,
                 bool fp32_cores, int64_t work_cap) {
  const int mx = X.w, my = Y.w;
  if (mx == 0 || my == 0) return;
  if (sym) ARR_REQUIRE(mx == my, "gram: symmetric product needs equal widths");
  if (n == 0) {
    launch_fill<double>(G, (int64_t)mx * my, 0.0, s);
    return;
  }
  const GramPlan p = gram_plan(n, mx, my, sym, work_cap > 0 ? work_cap : kGramWorkCap);
  if (work_cap > 0)
    ARR_REQUIRE((int64_t)p.nsplit * mx * my <= work_cap, "gram: split partials exceed the work buffer");
  const dim3 grid(p.ntiles * p.nsplit);
  const bool big = p.tile == 128;
  // algorithmic flops: 2 n mx my, or n m (m + 1) for the upper triangle
  const double flops = sym ? (double)n * mx * (mx + 1) : 2.0 * n * mx * my;
  SpmmTimer::Scope scope(gemm_timer(),
                         std::is_same<T, double>::value ? kGramF64 : (fp32_cores ? kGramF32Cores : kGramF32),
                         flops, s);
  const int sy = sym ? 1 : 0;
  if (std::is_same<T, float>::value && fp32_cores) {
    const float *xf = (const float *)X.p, *yf = (const float *)Y.p;
    if (big)
      hipLaunchKernelGGL((k_gram<float, true, 128>), grid, dim3(256), 0, s, n, xf, X.ld, mx, yf, Y.ld, my, p.ntx,
                         p.nty, p.ntiles, sy, p.chunk, work);
    else
      hipLaunchKernelGGL((k_gram<float, true, 64>), grid, dim3(256), 0, s, n, xf, X.ld, mx, yf, Y.ld, my, p.ntx,
                         p.nty, p.ntiles, sy, p.chunk, work);
  } else if (big) {
    hipLaunchKernelGGL((k_gram<T, false, 128>), grid, dim3(256), 0, s, n, X.p, X.ld, mx, Y.p, Y.ld, my, p.ntx,
                       p.nty, p.ntiles, sy, p.chunk, work);
  } else {
    hipLaunchKernelGGL((k_gram<T, false, 64>), grid, dim3(256), 0, s, n, X.p, X.ld, mx, Y.p, Y.ld, my, p.ntx,
                       p.nty, p.ntiles, sy, p.chunk, work);
  }
  ARR_HIP(hipGetLastError());
  const int64_t tot = (int64_t)mx * my;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, p.nsplit, mx,
                     my, sym ? 1 : 0, G);
  ARR_HIP(hipGetLastError());
}

template <typename T>
void launch_update(int64_t n, Blk<const T> X, const double *W, int64_t ldw, int c, double alpha, double beta,
                   Blk<T> Y, hipStream_t s, bool w_upper, bool fp32_cores, const double *colss) {
  const int m = X.w;
  if (n == 0 || c == 0) return;
  // algorithmic flops: 2 n m c, or with W upper triangular 2 n sum_j min(m, j + 1)
  double terms = (double)m * c;
  if (w_upper) {
    const double t = std::min(c, m);
    terms = t * (t + 1) / 2 + (double)std::max(0, c - m) * m;
  }
  SpmmTimer::Scope scope(gemm_timer(),
                         std::is_same<T, double>::value ? kUpdF64 : (fp32_cores ? kUpdF32Cores : kUpdF32),
                         2.0 * n * terms, s);
  // 128 tiles only for the FP32 matrix cores: with FP64 accumulators the
  // 128 tile needs a whole SIMD per wave and ran at half the 64 tile's rate
  const bool cores32 = std::is_same<T, float>::value && fp32_cores;
  const int tile = (cores32 && c >= 128) ? 128 : 64;
  const int nct = (c + tile - 1) / tile;
  const int64_t nrt = (n + tile - 1) / tile;
  const int64_t bands_per_xcd = (nrt + kXcd - 1) / kXcd;
  const dim3 grid((unsigned)(bands_per_xcd * nct * kXcd));
  const int wu = w_upper ? 1 : 0;
  if (cores32) {
    const float *xf = (const float *)X.p;
    float *yf = (float *)Y.p;
    if (tile == 128)
      hipLaunchKernelGGL((k_update<float, true, 128>), grid, dim3(256), 0, s, n, xf, X.ld, m, W, ldw, c, alpha,
                         beta, yf, Y.ld, nct, nrt, wu, colss);
    else
      hipLaunchKernelGGL((k_update<float, true, 64>), grid, dim3(256), 0, s, n, xf, X.ld, m, W, ldw, c, alpha,
                         beta, yf, Y.ld, nct, nrt, wu, colss);
  } else {
    hipLaunchKernelGGL((k_update<T, false, 64>), grid, dim3(256), 0, s, n, X.p, X.ld, m, W, ldw, c, alpha, beta,
                       Y.p, Y.ld, nct, nrt, wu, colss);
  }
  ARR_HIP(hipGetLastError());
}

template void launch_gram<double>(int64_t, Blk<const double>, Blk<const double>, double *, double *, bool,
                                  hipStream_t, bool, int64_t);
template void launch_gram<float>(int64_t, Blk<const float>, Blk<const float>, double *, double *, bool,
                                 hipStream_t, bool, int64_t);
template void launch_update<double>(int64_t, Blk<const double>, const double *, int64_t, int, double, double,
                                    Blk<double>, hipStream_t, bool, bool, const double *);
template void launch_update<float>(int64_t, Blk<const float>, const double *, int64_t, int, double, double,
                                   Blk<float>, hipStream_t, bool, bool, const double *);

}  // namespace arr
