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
// FP32 blocks (mixed precision) are widened to FP64 on load, so both products
// accumulate in FP64.
//
// MFMA 16x16x4 FP64 operand layout (lane l of 64): A[i][k] with i = l % 16,
// k = l / 16; B[k][j] with k = l / 16, j = l % 16; result D[i][j] in element
// r of lane l for i = l / 16 + 4 r, j = l % 16 (checked on gfx950).
#include <algorithm>

#include "common.h"

namespace arr {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct GramPlan {
  int ntx, nty, ntiles, nsplit;
  int64_t chunk;
};

GramPlan gram_plan(int64_t n, int mx, int my, bool sym) {
  GramPlan p;
  p.ntx = (mx + 63) / 64;
  p.nty = (my + 63) / 64;
  p.ntiles = sym ? p.ntx * (p.ntx + 1) / 2 : p.ntx * p.nty;
  int64_t want = std::max<int64_t>(1, (2048 + p.ntiles - 1) / p.ntiles);
  // at least 256 rows per split so each wave streams a useful amount
  want = std::min<int64_t>(want, std::max<int64_t>(1, n / 256));
  p.nsplit = (int)want;
  p.chunk = round_up((n + p.nsplit - 1) / p.nsplit, 16);
  if (p.chunk == 0) p.chunk = 16;
  p.nsplit = (int)std::max<int64_t>(1, (n + p.chunk - 1) / p.chunk);
  return p;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gram(int64_t n, const T *__restrict__ X, int64_t ldx, int mx,
                                              const T *__restrict__ Y, int64_t ldy, int my, int ntx, int nty,
                                              int ntiles, int sym, int64_t chunk, double *__restrict__ part) {
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
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int cx = tx * 64, cy = ty * 64;
  const int64_t r0 = (int64_t)split * chunk;
  const int64_t r1 = min(n, r0 + chunk);

  v4d acc[4][4];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[f][g] = v4d{0.0, 0.0, 0.0, 0.0};

  bool okx[4], oky[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    okx[f] = cx + 16 * f + li < mx;
    oky[f] = cy + 16 * f + li < my;
  }
  // software pipeline: the loads of the next 32-row step are in flight while
  // the matrix cores consume the current one
  double a[2][4], b[2][4];
  auto load = [&](int64_t r, double (&la)[2][4], double (&lb)[2][4]) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t row = r + 16 * u + lk;
      const bool rok = row < r1;
      const T *xr = X + row * ldx + cx + li;
      const T *yr = Y + row * ldy + cy + li;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        la[u][f] = (rok && okx[f]) ? (double)xr[16 * f] : 0.0;
        lb[u][f] = (rok && oky[f]) ? (double)yr[16 * f] : 0.0;
      }
    }
  };
  int64_t r = r0 + 4 * wv;
  if (r < r1) load(r, a, b);
  for (; r < r1; r += 32) {
    double na[2][4], nb[2][4];
    if (r + 32 < r1) load(r + 32, na, nb);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[f][g] = mfma16(a[u][f], b[u][g], acc[f][g]);
    if (r + 32 < r1) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          a[u][f] = na[u][f];
          b[u][f] = nb[u][f];
        }
    }
  }

  __shared__ double red[64 * 64];
  for (int q = 0; q < 4; ++q) {
    if (wv == q) {
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = 16 * f + lk + 4 * e, j = 16 * g + li;
            if (q == 0)
              red[i * 64 + j] = acc[f][g][e];
            else
              red[i * 64 + j] += acc[f][g][e];
          }
    }
    __syncthreads();
  }
  double *out = part + (int64_t)split * mx * my;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int i = idx / 64, j = idx % 64;
    if (cx + i < mx && cy + j < my) out[(int64_t)(cx + i) * my + cy + j] = red[idx];
  }
}

// G[i][j] = sum_s part[s][i][j] in order; for sym, the upper element is used
// for both (i, j) and (j, i).
__global__ void k_gram_reduce(const double *__restrict__ part, int nsplit, int mx, int my, int sym,
                              double *__restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)mx * my) return;
  int i = (int)(idx / my), j = (int)(idx % my);
  if (sym && (i / 64) > (j / 64)) { const int t = i; i = j; j = t; }
  const int64_t src = (int64_t)i * my + j;
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * mx * my + src];
  G[idx] = s;
}

__global__ void k_mirror_upper(int m, double *G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx / m), j = (int)(idx % m);
  if (i > j) G[idx] = G[(int64_t)j * m + i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_update(int64_t n, const T *__restrict__ X, int64_t ldx, int m,
                                                const double *__restrict__ W, int64_t ldw, int c, double alpha,
                                                double beta, T *Y, int64_t ldy, int nct, int64_t nrt, int w_upper) {
  // tile order: XCD x gets workgroups b = x + 8 t; t walks the column tiles of
  // one row band before moving to the next band of that XCD.
  const int xcd = blockIdx.x % kXcd;
  const int64_t t = blockIdx.x / kXcd;
  const int ct = (int)(t % nct);
  const int64_t rt = (t / nct) * kXcd + xcd;
  if (rt >= nrt) return;
  const int64_t r0 = rt * 64;
  const int c0 = ct * 64;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // W upper triangular: rows k > c0 + 63 of this column tile are zero
  const int kend = w_upper ? min(m, c0 + 64) : m;

  __shared__ double Xs[64][17];
  __shared__ double Ws[16][65];

  v4d acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = v4d{0.0, 0.0, 0.0, 0.0};

  const int xr_ = threadIdx.x >> 2, xk = (threadIdx.x & 3) * 4;   // X tile: 64 rows x 16 k
  const int wk_ = threadIdx.x >> 4, wc = (threadIdx.x & 15) * 4;  // W tile: 16 k x 64 cols
  const int64_t xrow = r0 + xr_;
  double xv[4], wvv[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = k0 + xk + q;
      xv[q] = (xrow < n && kk < kend) ? (double)X[xrow * ldx + kk] : 0.0;
      const int kw = k0 + wk_, cc = c0 + wc + q;
      wvv[q] = (kw < kend && cc < c) ? W[(int64_t)kw * ldw + cc] : 0.0;
    }
  };
  if (kend > 0) load(0);
  for (int k0 = 0; k0 < kend; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Xs[xr_][xk + q] = xv[q];
      Ws[wk_][wc + q] = wvv[q];
    }
    __syncthreads();
    if (k0 + 16 < kend) load(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = Xs[16 * wv + li][4 * ks + lk];
#pragma unroll
      for (int g = 0; g < 4; ++g) acc[g] = mfma16(a, Ws[4 * ks + lk][16 * g + li], acc[g]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int col = c0 + 16 * g + li;
    if (col >= c) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = r0 + 16 * wv + lk + 4 * e;
      if (row >= n) continue;
      T *yp = Y + row * ldy + col;
      double v = alpha * acc[g][e];
      if (beta != 0.0) v += beta * (double)(*yp);
      *yp = (T)v;
    }
  }
}

}  // namespace

size_t gram_work_bound(int64_t n, int m_max) {
  // nsplit <= ceil(2048 / ntiles) and mx * my <= 4096 * tx * ty, so the partial
  // tiles of any product with mx, my <= m_max fit in (4096 + t^2) 64 x 64
  // tiles; nsplit is also at most max(1, n / 256).
  const size_t t = (size_t)(m_max + 63) / 64;
  const size_t by_tiles = (4096 + t * t) * 4096;
  const size_t by_rows = (size_t)std::max<int64_t>(1, n / 256) * t * t * 4096;
  return std::min(by_tiles, by_rows);
}

size_t gram_work_doubles(int64_t n, int mx, int my) {
  // the symmetric plan applies to square products only (launch_gram requires it)
  const GramPlan p = gram_plan(n, mx, my, false);
  int nsplit = p.nsplit;
  if (mx == my) nsplit = std::max(nsplit, gram_plan(n, mx, my, true).nsplit);
  return (size_t)nsplit * (size_t)mx * (size_t)my;
}

template <typename T>
void launch_gram(int64_t n, Blk<const T> X, Blk<const T> Y, double *G, double *work, bool sym, hipStream_t s) {
  const int mx = X.w, my = Y.w;
  if (mx == 0 || my == 0) return;
  if (sym) ARR_REQUIRE(mx == my, "gram: symmetric product needs equal widths");
  if (n == 0) {
    launch_fill<double>(G, (int64_t)mx * my, 0.0, s);
    return;
  }
  const GramPlan p = gram_plan(n, mx, my, sym);
  hipLaunchKernelGGL((k_gram<T>), dim3(p.ntiles * p.nsplit), dim3(256), 0, s, n, X.p, X.ld, mx, Y.p, Y.ld, my,
                     p.ntx, p.nty, p.ntiles, sym ? 1 : 0, p.chunk, work);
  ARR_HIP(hipGetLastError());
  const int64_t tot = (int64_t)mx * my;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, p.nsplit, mx,
                     my, sym ? 1 : 0, G);
  ARR_HIP(hipGetLastError());
}

template <typename T>
void launch_update(int64_t n, Blk<const T> X, const double *W, int64_t ldw, int c, double alpha, double beta,
                   Blk<T> Y, hipStream_t s, bool w_upper) {
  const int m = X.w;
  if (n == 0 || c == 0) return;
  const int nct = (c + 63) / 64;
  const int64_t nrt = (n + 63) / 64;
  const int64_t bands_per_xcd = (nrt + kXcd - 1) / kXcd;
  const int64_t grid = bands_per_xcd * nct * kXcd;
  hipLaunchKernelGGL((k_update<T>), dim3((unsigned)grid), dim3(256), 0, s, n, X.p, X.ld, m, W, ldw, c, alpha,
                     beta, Y.p, Y.ld, nct, nrt, w_upper ? 1 : 0);
  ARR_HIP(hipGetLastError());
}

template void launch_gram<double>(int64_t, Blk<const double>, Blk<const double>, double *, double *, bool,
                                  hipStream_t);
template void launch_gram<float>(int64_t, Blk<const float>, Blk<const float>, double *, double *, bool,
                                 hipStream_t);
template void launch_update<double>(int64_t, Blk<const double>, const double *, int64_t, int, double, double,
                                    Blk<double>, hipStream_t, bool);
template void launch_update<float>(int64_t, Blk<const float>, const double *, int64_t, int, double, double,
                                   Blk<float>, hipStream_t, bool);

}  // namespace arr
