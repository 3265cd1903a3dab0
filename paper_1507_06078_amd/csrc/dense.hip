// Small FP64 dense linear algebra on the device (matrices of order up to a
// few thousand, row-major, resident in L2 / Infinity Cache):
//
//  * blocked right-looking Cholesky (panel of 32: every workgroup factors the
//    diagonal block in LDS, then solves its share of the rows below; the
//    trailing update is a small MFMA GEMM on the lower tiles);
//  * inverse of a lower-triangular factor (diagonal blocks in LDS, then
//    recursive doubling with batched MFMA GEMMs), used for the Cholesky-QR
//    basis Z R^-1 and for rcond;
//  * rcond(G) = 1/(|G|_1 |G^-1|_1) with G^-1 = L^-T L^-1 (eq. inn-stop);
//  * the symmetric eigensolver of the Rayleigh-Ritz step (Algorithm 1): a
//    two-sided block Jacobi method. Indices are grouped in blocks of 16; each
//    step pairs the blocks by the round-robin (circle) ordering, diagonalizes
//    every 32 x 32 pair subproblem completely in LDS (scalar cyclic Jacobi, 16
//    rotations at a time), then applies the 32 x 32 rotations to the whole
//    matrix (A' = R_t^T A R_u blockwise, double-buffered) and to the
//    eigenvectors (kept as rows of V^T so updates are coalesced). Sweeps stop
//    when no subproblem needed a rotation.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.h"

namespace arr {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C[i][j] = beta C[i][j] + alpha sum_k A(i,k) B(k,j), 0 <= i < m1, 0 <= j < m2,
// A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj]. lower: tiles strictly
// above the diagonal (in tile units, with row offset) are skipped.
__global__ __launch_bounds__(256) void k_small_gemm(int m1, int m2, int kk, double alpha, const double *A,
                                                    int64_t sai, int64_t sak, const double *B, int64_t sbk,
                                                    int64_t sbj, double beta, double *C, int64_t ldc, int lower) {
  const int nct = (m2 + 63) / 64;
  const int rt = blockIdx.x / nct, ct = blockIdx.x % nct;
  if (lower && ct > rt) return;
  const int r0 = rt * 64, c0 = ct * 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double As[64][17];
  __shared__ double Bs[16][65];
  v4d acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kk; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int r = e / 16, k = e % 16;
      As[r][k] = (r0 + r < m1 && k0 + k < kk) ? A[(int64_t)(r0 + r) * sai + (int64_t)(k0 + k) * sak] : 0.0;
      const int kb = e / 64, c = e % 64;
      Bs[kb][c] = (k0 + kb < kk && c0 + c < m2) ? B[(int64_t)(k0 + kb) * sbk + (int64_t)(c0 + c) * sbj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = As[16 * wv + li][4 * ks + lk];
#pragma unroll
      for (int g = 0; g < 4; ++g) acc[g] = mfma16(a, Bs[4 * ks + lk][16 * g + li], acc[g]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int col = c0 + 16 * g + li;
    if (col >= m2) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + 16 * wv + lk + 4 * e;
      if (row >= m1) continue;
      double *cp = C + (int64_t)row * ldc + col;
      double v = alpha * acc[g][e];
      if (beta != 0.0) v += beta * (*cp);
      *cp = v;
    }
  }
}

}  // namespace

void small_gemm(int m1, int m2, int kk, double alpha, const double *A, int64_t sai, int64_t sak, const double *B,
                int64_t sbk, int64_t sbj, double beta, double *C, int64_t ldc, bool lower, hipStream_t s) {
  if (m1 <= 0 || m2 <= 0) return;
  const int grid = ((m1 + 63) / 64) * ((m2 + 63) / 64);
  hipLaunchKernelGGL(k_small_gemm, dim3(grid), dim3(256), 0, s, m1, m2, kk, alpha, A, sai, sak, B, sbk, sbj, beta,
                     C, ldc, lower ? 1 : 0);
  ARR_HIP(hipGetLastError());
}

namespace {

constexpr int kNB = 32;       // Cholesky panel width

// Diagonal block J0..J0+nb of the Cholesky factorization, factored in place
// in LDS by one workgroup. A non-positive pivot records its (1-based) column
// in *info (first failure kept) and is replaced by 1 so the rest stays finite.
__global__ __launch_bounds__(256) void k_chol_diag(double *A, int64_t lda, int J0, int nb, int *info) {
  __shared__ double D[kNB][kNB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    D[r][c] = A[(int64_t)(J0 + r) * lda + J0 + c];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double d = D[j][j];
      if (!(d > 0.0) || !isfinite(d)) {
        if (!bad) bad = J0 + j + 1;
        D[j][j] = 1.0;
      } else {
        D[j][j] = sqrt(d);
      }
    }
    __syncthreads();
    const double djj = D[j][j];
    for (int i = j + 1 + tid; i < nb; i += 256) D[i][j] /= djj;
    __syncthreads();
    for (int e = tid; e < (nb - j - 1) * (nb - j - 1); e += 256) {
      const int i = j + 1 + e / (nb - j - 1), k = j + 1 + e % (nb - j - 1);
      if (k <= i) D[i][k] -= D[i][j] * D[k][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    if (c <= r) A[(int64_t)(J0 + r) * lda + J0 + c] = D[r][c];
  }
  if (tid == 0 && bad && *info == 0) *info = bad;
}

// Rows below the factored diagonal block: L[i][J] = A[i][J] L_JJ^-T by forward
// substitution, one row per thread.
__global__ __launch_bounds__(256) void k_chol_rows(int m, double *A, int64_t lda, int J0, int nb) {
  __shared__ double D[kNB][kNB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    D[r][c] = (c <= r) ? A[(int64_t)(J0 + r) * lda + J0 + c] : 0.0;
  }
  __syncthreads();
  const int i = J0 + nb + blockIdx.x * 256 + tid;
  if (i >= m) return;
  double *row = A + (int64_t)i * lda + J0;
  double l[kNB];
  for (int t = 0; t < nb; ++t) {
    double v = row[t];
    for (int q = 0; q < t; ++q) v -= l[q] * D[t][q];
    l[t] = v / D[t][t];
  }
  for (int t = 0; t < nb; ++t) row[t] = l[t];
}

__global__ void k_add_diag(int m, double *A, int64_t lda, double shift) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) A[(int64_t)i * lda + i] += shift;
}

// Inverse of the lower-triangular L (m x m), built in two phases:
//  1. every 32 x 32 diagonal block is inverted in LDS by one workgroup
//     (one column per thread, forward substitution);
//  2. recursive doubling: for blocks A = [lo, lo+s) and C = [lo+s, lo+2s)
//     with both inverses known, the off-diagonal block of the inverse of
//     [A 0; B C] is -C^-1 B A^-1; all pairs of one level are merged by two
//     batched GEMM launches (T = B A^-1, X = -C^-1 T).
// The result Li (lower, zeros above) is finally transposed into W = L^-T.
constexpr int kTB = 32;

__global__ __launch_bounds__(64) void k_trinv_diag(int m, const double *__restrict__ L, int64_t ldl,
                                                   double *__restrict__ Li, int64_t ldi) {
  __shared__ double D[kTB][kTB + 1];
  __shared__ double X[kTB][kTB + 1];
  const int b0 = blockIdx.x * kTB;
  const int nb = min(kTB, m - b0);
  for (int e = threadIdx.x; e < kTB * kTB; e += 64) {
    const int r = e / kTB, c = e % kTB;
    D[r][c] = (r < nb && c <= r) ? L[(int64_t)(b0 + r) * ldl + b0 + c] : 0.0;
  }
  __syncthreads();
  const int j = threadIdx.x;
  if (j < nb) {
    for (int i = 0; i < nb; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
      if (i >= j) {
        for (int q = j; q < i; ++q) v -= D[i][q] * X[q][j];
        v /= D[i][i];
      } else {
        v = 0.0;
      }
      X[i][j] = v;
    }
  }
  __syncthreads();
  // write the diagonal block and clear the row segment to its right
  for (int e = threadIdx.x; e < nb * kTB; e += 64) {
    const int r = e / kTB, c = e % kTB;
    if (c < nb) Li[(int64_t)(b0 + r) * ldi + b0 + c] = X[r][c];
  }
}

// One merge level (block size s): pair p covers A = [2ps, 2ps+s), C = [2ps+s,
// min(2ps+2s, m)). mode 0: T = B A^-1 (T stored at Ti with the same row/col
// offsets as B); mode 1: Li[C rows][A cols] = -C^-1 T.
__global__ __launch_bounds__(256) void k_trinv_merge(int m, int s, int mode, const double *__restrict__ L,
                                                     int64_t ldl, double *Li, int64_t ldi, double *T) {
  const int p = blockIdx.y;
  const int lo = 2 * p * s, mid = lo + s, hi = min(lo + 2 * s, m);
  if (mid >= m) return;
  const int rows = hi - mid, cols = s;
  const int ntc = (cols + 63) / 64;
  const int rt = blockIdx.x / ntc, ct = blockIdx.x % ntc;
  const int r0 = rt * 64, c0 = ct * 64;
  if (r0 >= rows) return;
  const int kk = mode == 0 ? s : rows;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double As[64][17];
  __shared__ double Bs[16][65];
  v4d acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kk; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int r = e / 16, k = e % 16;
      const int gr = r0 + r, gk = k0 + k;
      double av = 0.0;
      if (gr < rows && gk < kk) {
        if (mode == 0)
          av = L[(int64_t)(mid + gr) * ldl + lo + gk];   // B = L[C rows][A cols]
        else
          av = (gk <= gr) ? Li[(int64_t)(mid + gr) * ldi + mid + gk] : 0.0;  // C^-1 (lower)
      }
      As[r][k] = av;
      const int kb = e / 64, c = e % 64;
      const int gkb = k0 + kb, gc = c0 + c;
      double bv = 0.0;
      if (gkb < kk && gc < cols) {
        if (mode == 0)
          bv = (gc <= gkb) ? Li[(int64_t)(lo + gkb) * ldi + lo + gc] : 0.0;  // A^-1 (lower)
        else
          bv = T[(int64_t)(mid + gkb) * ldi + lo + gc];
      }
      Bs[kb][c] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = As[16 * wv + li][4 * ks + lk];
#pragma unroll
      for (int g = 0; g < 4; ++g) acc[g] = mfma16(a, Bs[4 * ks + lk][16 * g + li], acc[g]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int col = c0 + 16 * g + li;
    if (col >= cols) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + 16 * wv + lk + 4 * e;
      if (row >= rows) continue;
      if (mode == 0)
        T[(int64_t)(mid + row) * ldi + lo + col] = acc[g][e];
      else
        Li[(int64_t)(mid + row) * ldi + lo + col] = -acc[g][e];
    }
  }
}

// W[j][i] = Li[i][j] for i >= j, 0 for i < j.
__global__ void k_lower_to_upper_t(int m, const double *__restrict__ Li, int64_t ldi, double *__restrict__ W,
                                   int64_t ldw) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int j = (int)(idx / m), i = (int)(idx % m);
  W[(int64_t)j * ldw + i] = (i >= j) ? Li[(int64_t)i * ldi + j] : 0.0;
}

// out = max_j sum_i |M[i][j]| (1-norm) of a square matrix, one block.
__device__ double block_norm1(int m, const double *M, int64_t ld, double *scratch) {
  double best = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += fabs(M[(int64_t)i * ld + j]);
    best = fmax(best, s);
  }
  scratch[threadIdx.x] = best;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) scratch[threadIdx.x] = fmax(scratch[threadIdx.x], scratch[threadIdx.x + off]);
    __syncthreads();
  }
  const double r = scratch[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_rcond_final(int m, const double *G, const double *Ginv, const int *info,
                                                     double *rc) {
  __shared__ double scratch[256];
  const double a = block_norm1(m, G, m, scratch);
  const double b = block_norm1(m, Ginv, m, scratch);
  if (threadIdx.x == 0) {
    double r = (a > 0.0 && b > 0.0 && isfinite(a * b)) ? 1.0 / (a * b) : 0.0;
    if (*info != 0) r = 0.0;
    *rc = r;
  }
}

// C <- (C - I) / 2 for the m x m matrix C (ld m): the GN correction factor.
__global__ __launch_bounds__(256) void k_half_minus_identity(int m, double *C) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx / m), j = (int)(idx % m);
  C[idx] = 0.5 * (C[idx] - (i == j ? 1.0 : 0.0));
}

__global__ __launch_bounds__(256) void k_diag_max(int m, const double *A, int64_t lda, double *out) {
  __shared__ double s1[256], s2[256];
  double mx = 0.0, fro = 0.0;
  for (int64_t idx = threadIdx.x; idx < (int64_t)m * m; idx += 256) {
    const int i = (int)(idx / m), j = (int)(idx % m);
    const double v = A[(int64_t)i * lda + j];
    if (i == j) mx = fmax(mx, fabs(v));
    fro += v * v;
  }
  s1[threadIdx.x] = mx;
  s2[threadIdx.x] = fro;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + off]);
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s1[0];
    out[1] = sqrt(s2[0]);
  }
}

// ---- Jacobi ------------------------------------------------------------------

__device__ __forceinline__ int rr_player(int pos, int step, int me) {
  // circle method: position 0 fixed, the others rotate by `step`
  return pos == 0 ? 0 : 1 + (pos - 1 + step) % (me - 1);
}

__device__ __forceinline__ void rr_pair(int t, int step, int me, int &p, int &q) {
  int a = rr_player(t, step, me), b = rr_player(me - 1 - t, step, me);
  p = min(a, b);
  q = max(a, b);
}

// Rotation annihilating a_pq (symmetric Schur decomposition of the 2 x 2
// block, Golub & Van Loan): returns false when a_pq is negligible.
__device__ __forceinline__ bool jac_rot(double app, double aqq, double apq, double tiny, double &c, double &s,
                                        double &t) {
  if (apq == 0.0 || fabs(apq) <= tiny || fabs(apq) <= 2.2e-16 * sqrt(fabs(app) * fabs(aqq))) {
    c = 1.0;
    s = 0.0;
    t = 0.0;
    return false;
  }
  const double tau = (aqq - app) / (2.0 * apq);
  if (fabs(tau) > 1e150)
    t = 0.5 / tau;
  else
    t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
  return true;
}

// ---- block Jacobi --------------------------------------------------------------
// Index blocks of kBJ = 16; a subproblem is the 32 x 32 principal submatrix of
// a pair of blocks (P, Q); the pairs of one step come from the round-robin
// ordering of the me / 16 blocks.
constexpr int kBJ = 16;
constexpr int kBJ2 = 2 * kBJ;
constexpr int kInnerSweeps = 1;  // inner sweeps per subproblem and outer step (one measured faster than two or three)

__device__ __forceinline__ int bj_index(int r, int P, int Q) { return r < kBJ ? P * kBJ + r : Q * kBJ + (r - kBJ); }

// Diagonalize the subproblem of pair t in LDS by cyclic Jacobi (circle
// ordering, 16 rotations at a time); write the accumulated rotation R
// (S_final = R^T S R) to Rbuf + t * 32 * 32. Sets *rotated if the first inner
// sweep needed any rotation.
__global__ __launch_bounds__(256) void k_bj_solve(int me, int nb, int step, const double *__restrict__ A,
                                                  double *__restrict__ Rbuf, double tiny, int *rotated) {
  __shared__ double S[2][kBJ2][kBJ2 + 1];
  __shared__ double R[kBJ2][kBJ2 + 1];
  __shared__ double cs[kBJ2 / 2][3];
  __shared__ int act[kBJ2 / 2];
  __shared__ int any;
  const int t = blockIdx.x, tid = threadIdx.x;
  int P, Q;
  rr_pair(t, step, nb, P, Q);
  for (int e = tid; e < kBJ2 * kBJ2; e += 256) {
    const int r = e / kBJ2, c = e % kBJ2;
    S[0][r][c] = A[(int64_t)bj_index(r, P, Q) * me + bj_index(c, P, Q)];
    R[r][c] = (r == c) ? 1.0 : 0.0;
  }
  int cur = 0, first_any = 0;
  for (int sw = 0; sw < kInnerSweeps; ++sw) {
    if (tid == 0) any = 0;
    __syncthreads();
    for (int st = 0; st < kBJ2 - 1; ++st) {
      if (tid < kBJ2 / 2) {
        int p, q;
        rr_pair(tid, st, kBJ2, p, q);
        double c, sn, tv;
        const bool r = jac_rot(S[cur][p][p], S[cur][q][q], S[cur][p][q], tiny, c, sn, tv);
        cs[tid][0] = c;
        cs[tid][1] = sn;
        cs[tid][2] = tv;
        act[tid] = r ? 1 : 0;
        if (r) any = 1;
      }
      __syncthreads();
      {
        const int I = tid / (kBJ2 / 2), J = tid % (kBJ2 / 2);
        int p, q, p2, q2;
        rr_pair(I, st, kBJ2, p, q);
        rr_pair(J, st, kBJ2, p2, q2);
        double(*Si)[kBJ2 + 1] = S[cur];
        double(*So)[kBJ2 + 1] = S[cur ^ 1];
        if (I == J) {
          if (act[I]) {
            const double apq = Si[p][q], tv = cs[I][2];
            So[p][p] = Si[p][p] - tv * apq;
            So[q][q] = Si[q][q] + tv * apq;
            So[p][q] = 0.0;
            So[q][p] = 0.0;
          } else {
            So[p][p] = Si[p][p];
            So[q][q] = Si[q][q];
            So[p][q] = Si[p][q];
            So[q][p] = Si[q][p];
          }
        } else {
          const double cI = cs[I][0], sI = cs[I][1], cJ = cs[J][0], sJ = cs[J][1];
          const double b00 = Si[p][p2], b01 = Si[p][q2], b10 = Si[q][p2], b11 = Si[q][q2];
          const double x00 = cI * b00 - sI * b10, x01 = cI * b01 - sI * b11;
          const double x10 = sI * b00 + cI * b10, x11 = sI * b01 + cI * b11;
          So[p][p2] = cJ * x00 - sJ * x01;
          So[p][q2] = sJ * x00 + cJ * x01;
          So[q][p2] = cJ * x10 - sJ * x11;
          So[q][q2] = sJ * x10 + cJ * x11;
        }
      }
      for (int e = tid; e < (kBJ2 / 2) * kBJ2; e += 256) {
        const int I = e / kBJ2, r = e % kBJ2;
        if (act[I]) {
          int p, q;
          rr_pair(I, st, kBJ2, p, q);
          const double c = cs[I][0], sn = cs[I][1];
          const double rp = R[r][p], rq = R[r][q];
          R[r][p] = c * rp - sn * rq;
          R[r][q] = sn * rp + c * rq;
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    const int a = any;
    if (sw == 0) first_any = a;
    __syncthreads();
    if (!a) break;
  }
  double *out = Rbuf + (int64_t)t * kBJ2 * kBJ2;
  for (int e = tid; e < kBJ2 * kBJ2; e += 256) out[e] = R[e / kBJ2][e % kBJ2];
  if (tid == 0 && first_any) *rotated = 1;
}

// A_out[g_t, g_u] = R_t^T A_in[g_t, g_u] R_u for every pair of pairs (t, u).
__device__ void bj_update(int blk, int me, int nb, int step, const double *__restrict__ Ain,
                          double *__restrict__ Aout, const double *__restrict__ Rbuf) {
  __shared__ double X[kBJ2][kBJ2 + 1], Rt[kBJ2][kBJ2 + 1], Ru[kBJ2][kBJ2 + 1], Y[kBJ2][kBJ2 + 1];
  const int np = nb / 2;
  const int t = blk / np, u = blk % np, tid = threadIdx.x;
  int Pt, Qt, Pu, Qu;
  rr_pair(t, step, nb, Pt, Qt);
  rr_pair(u, step, nb, Pu, Qu);
  const double *rt = Rbuf + (int64_t)t * kBJ2 * kBJ2, *ru = Rbuf + (int64_t)u * kBJ2 * kBJ2;
  for (int e = tid; e < kBJ2 * kBJ2; e += 256) {
    const int r = e / kBJ2, c = e % kBJ2;
    X[r][c] = Ain[(int64_t)bj_index(r, Pt, Qt) * me + bj_index(c, Pu, Qu)];
    Rt[r][c] = rt[e];
    Ru[r][c] = ru[e];
  }
  __syncthreads();
  for (int e = tid; e < kBJ2 * kBJ2; e += 256) {
    const int r = e / kBJ2, c = e % kBJ2;
    double v = 0.0;
#pragma unroll 8
    for (int k = 0; k < kBJ2; ++k) v = fma(Rt[k][r], X[k][c], v);
    Y[r][c] = v;
  }
  __syncthreads();
  for (int e = tid; e < kBJ2 * kBJ2; e += 256) {
    const int r = e / kBJ2, c = e % kBJ2;
    double v = 0.0;
#pragma unroll 8
    for (int k = 0; k < kBJ2; ++k) v = fma(Y[r][k], Ru[k][c], v);
    Aout[(int64_t)bj_index(r, Pt, Qt) * me + bj_index(c, Pu, Qu)] = v;
  }
}

// VT[g_t, c0:c0+64] = R_t^T VT[g_t, c0:c0+64] (eigenvectors kept as rows).
__device__ void bj_vupdate(int blk, int me, int nb, int step, double *__restrict__ VT,
                           const double *__restrict__ Rbuf) {
  __shared__ double W[kBJ2][65], Rt[kBJ2][kBJ2 + 1];
  const int nchunk = (me + 63) / 64;
  const int t = blk / nchunk, c0 = (blk % nchunk) * 64, tid = threadIdx.x;
  int P, Q;
  rr_pair(t, step, nb, P, Q);
  const double *rt = Rbuf + (int64_t)t * kBJ2 * kBJ2;
  for (int e = tid; e < kBJ2 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    W[r][c] = (c0 + c < me) ? VT[(int64_t)bj_index(r, P, Q) * me + c0 + c] : 0.0;
  }
  for (int e = tid; e < kBJ2 * kBJ2; e += 256) Rt[e / kBJ2][e % kBJ2] = rt[e];
  __syncthreads();
  for (int e = tid; e < kBJ2 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    if (c0 + c >= me) continue;
    double v = 0.0;
#pragma unroll 8
    for (int k = 0; k < kBJ2; ++k) v = fma(Rt[k][r], W[k][c], v);
    VT[(int64_t)bj_index(r, P, Q) * me + c0 + c] = v;
  }
}

// One launch applies the rotations of a step to the matrix (first np^2
// workgroups) and to the eigenvectors (the rest).
__global__ __launch_bounds__(256) void k_bj_apply(int me, int nb, int step, const double *__restrict__ Ain,
                                                  double *__restrict__ Aout, double *__restrict__ VT,
                                                  const double *__restrict__ Rbuf) {
  const int np = nb / 2;
  if ((int)blockIdx.x < np * np)
    bj_update(blockIdx.x, me, nb, step, Ain, Aout, Rbuf);
  else
    bj_vupdate(blockIdx.x - np * np, me, nb, step, VT, Rbuf);
}

__global__ void k_jacobi_init(int m, int me, const double *__restrict__ H, double *__restrict__ A,
                              double *__restrict__ VT) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)me * me) return;
  const int i = (int)(idx / me), j = (int)(idx % me);
  A[idx] = (i < m && j < m) ? 0.5 * (H[(int64_t)i * m + j] + H[(int64_t)j * m + i]) : 0.0;
  VT[idx] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_jacobi_diag(int me, const double *A, double *d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < me) d[i] = A[(int64_t)i * me + i];
}

__global__ void k_gather_rows(int m, int me, const double *__restrict__ VT, const int *__restrict__ perm,
                              double *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int r = (int)(idx / m), c = (int)(idx % m);
  out[idx] = VT[(int64_t)perm[c] * me + r];
}

}  // namespace

void launch_cholesky(int m, double *A, int64_t lda, double shift, int *info, hipStream_t s) {
  launch_fill<int>(info, 1, 0, s);
  if (m == 0) return;
  if (shift != 0.0) {
    hipLaunchKernelGGL(k_add_diag, dim3((m + 255) / 256), dim3(256), 0, s, m, A, lda, shift);
    ARR_HIP(hipGetLastError());
  }
  for (int J0 = 0; J0 < m; J0 += kNB) {
    const int nb = std::min(kNB, m - J0);
    const int below = m - J0 - nb;
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, A, lda, J0, nb, info);
    ARR_HIP(hipGetLastError());
    if (below > 0) {
      hipLaunchKernelGGL(k_chol_rows, dim3((below + 255) / 256), dim3(256), 0, s, m, A, lda, J0, nb);
      ARR_HIP(hipGetLastError());
      // A22 -= L21 L21^T (lower tiles)
      const double *L21 = A + (int64_t)(J0 + nb) * lda + J0;
      small_gemm(below, below, nb, -1.0, L21, lda, 1, L21, 1, lda, 1.0, A + (int64_t)(J0 + nb) * lda + J0 + nb, lda,
                 true, s);
    }
  }
}

void launch_tri_inv_t(int m, const double *L, int64_t ldl, double *Winv, int64_t ldw, double *scratch,
                      hipStream_t s) {
  if (m == 0) return;
  double *Li = scratch, *T = Li + (size_t)m * m;
  const int nblk = (m + kTB - 1) / kTB;
  hipLaunchKernelGGL(k_trinv_diag, dim3(nblk), dim3(64), 0, s, m, L, ldl, Li, (int64_t)m);
  ARR_HIP(hipGetLastError());
  for (int bs = kTB; bs < m; bs *= 2) {
    const int pairs = (m + 2 * bs - 1) / (2 * bs);
    const int tiles = ((bs + 63) / 64) * ((bs + 63) / 64);
    hipLaunchKernelGGL(k_trinv_merge, dim3(tiles, pairs), dim3(256), 0, s, m, bs, 0, L, ldl, Li, (int64_t)m, T);
    hipLaunchKernelGGL(k_trinv_merge, dim3(tiles, pairs), dim3(256), 0, s, m, bs, 1, L, ldl, Li, (int64_t)m, T);
    ARR_HIP(hipGetLastError());
  }
  const int64_t tot = (int64_t)m * m;
  hipLaunchKernelGGL(k_lower_to_upper_t, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, Li, (int64_t)m,
                     Winv, ldw);
  ARR_HIP(hipGetLastError());
}

void launch_half_minus_identity(int m, double *C, hipStream_t s) {
  if (m == 0) return;
  const int64_t tot = (int64_t)m * m;
  hipLaunchKernelGGL(k_half_minus_identity, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, C);
  ARR_HIP(hipGetLastError());
}

void launch_diag_max(int m, const double *A, int64_t lda, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(256), 0, s, m, A, lda, out);
  ARR_HIP(hipGetLastError());
}

// rcond(G) for an m x m SPD candidate G (device, ld m). work: 5 m^2 doubles.
// Result written to rc (device).
void rcond_device(int m, const double *G, double *work, int *info, double *rc, hipStream_t s) {
  double *L = work, *Wt = work + (int64_t)m * m, *Gi = work + 2 * (int64_t)m * m;
  double *scratch = work + 3 * (int64_t)m * m;
  ARR_HIP(hipMemcpyAsync(L, G, sizeof(double) * m * m, hipMemcpyDeviceToDevice, s));
  launch_cholesky(m, L, m, 0.0, info, s);
  launch_tri_inv_t(m, L, m, Wt, m, scratch, s);
  // G^-1 = L^-T L^-1 = Wt Wt^T
  small_gemm(m, m, m, 1.0, Wt, m, 1, Wt, 1, m, 0.0, Gi, m, false, s);
  hipLaunchKernelGGL(k_rcond_final, dim3(1), dim3(256), 0, s, m, G, Gi, info, rc);
  ARR_HIP(hipGetLastError());
}

static size_t jac_pad(size_t b) { return (b + 255) / 256 * 256; }

size_t Jacobi::reserve_bytes(int m) {
  const size_t me = (size_t)(std::max(m, 1) + kBJ2 - 1) / kBJ2 * kBJ2;
  const size_t np = me / kBJ / 2;
  return 3 * jac_pad(sizeof(double) * me * me) + jac_pad(sizeof(double) * 4 + sizeof(int) * 4 + sizeof(int) * me) +
         jac_pad(sizeof(double) * (me + np * kBJ2 * kBJ2));
}

void Jacobi::reserve(int m) {
  const int me = (std::max(m, 1) + kBJ2 - 1) / kBJ2 * kBJ2;
  if (me <= mcap) return;
  const int np = me / kBJ / 2;
  bufA.alloc(sizeof(double) * me * me);
  bufB.alloc(sizeof(double) * me * me);
  bufV.alloc(sizeof(double) * me * me);
  bufOff.alloc(sizeof(double) * 4 + sizeof(int) * 4 + sizeof(int) * me);
  bufEval.alloc(sizeof(double) * (me + (size_t)np * kBJ2 * kBJ2));
  mcap = me;
}

void Jacobi::solve(int m, const double *H, double *V, std::vector<double> &evals_host, hipStream_t s,
                   int *sweeps_out) {
  evals_host.assign(m, 0.0);
  if (m == 0) return;
  const int me = (m + kBJ2 - 1) / kBJ2 * kBJ2;  // padded with decoupled zero rows/columns
  const int nb = me / kBJ, np = nb / 2;
  reserve(m);
  double *A = bufA.as<double>(), *B = bufB.as<double>(), *VT = bufV.as<double>();
  double *Rbuf = bufEval.as<double>() + me;
  double *nrm = bufOff.as<double>();
  int *flag = reinterpret_cast<int *>(nrm + 4);
  int *perm = flag + 4;
  const int64_t tot = (int64_t)me * me;
  hipLaunchKernelGGL(k_jacobi_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, me, H, A, VT);
  ARR_HIP(hipGetLastError());
  launch_diag_max(me, A, me, nrm, s);
  double hn[2];
  ARR_HIP(hipMemcpyAsync(hn, nrm, sizeof(hn), hipMemcpyDeviceToHost, s));
  ARR_HIP(hipStreamSynchronize(s));
  // A rotation is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|) or below an
  // absolute floor of 1e-18 |H|_F. Clusters of zero eigenvalues never meet
  // the relative bound and keep rotating on rounding-level entries; after
  // kLooseSweeps sweeps the floor is raised to eps |H|_F (a perturbation
  // within the rounding of H itself), which ends them.
  double tiny = std::max(1e-300, 1e-18 * hn[1]);
  const int nchunk = (me + 63) / 64;
  constexpr int kMaxSweeps = 40, kLooseSweeps = 20;
  int sweeps = 0;
  for (; sweeps < kMaxSweeps; ++sweeps) {
    if (sweeps == kLooseSweeps) tiny = std::max(tiny, 2.2e-16 * hn[1]);
    launch_fill<int>(flag, 1, 0, s);
    const int steps = nb > 1 ? nb - 1 : 1;
    for (int st = 0; st < steps; ++st) {
      hipLaunchKernelGGL(k_bj_solve, dim3(np), dim3(256), 0, s, me, nb, st, A, Rbuf, tiny, flag);
      hipLaunchKernelGGL(k_bj_apply, dim3(np * np + np * nchunk), dim3(256), 0, s, me, nb, st, A, B, VT, Rbuf);
      std::swap(A, B);
    }
    ARR_HIP(hipGetLastError());
    int hf = 0;
    ARR_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ARR_HIP(hipStreamSynchronize(s));
    if (!hf) break;
  }
  if (sweeps_out) *sweeps_out = sweeps;
  // every sweep so far still rotated some pair: the off-diagonal part has not
  // fallen below the threshold (cyclic Jacobi converges quadratically, so this
  // points at non-finite or badly scaled input)
  if (sweeps == kMaxSweeps)
    throw Error(-5, "small eigensolve: Jacobi did not converge in " + std::to_string(kMaxSweeps) +
                        " sweeps (order " + std::to_string(m) + ")");
  hipLaunchKernelGGL(k_jacobi_diag, dim3((me + 255) / 256), dim3(256), 0, s, me, A, bufEval.as<double>());
  ARR_HIP(hipGetLastError());
  std::vector<double> d(me);
  ARR_HIP(hipMemcpyAsync(d.data(), bufEval.as<double>(), sizeof(double) * me, hipMemcpyDeviceToHost, s));
  ARR_HIP(hipStreamSynchronize(s));
  std::vector<int> idx(m);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] > d[b]; });
  for (int i = 0; i < m; ++i) evals_host[i] = d[idx[i]];
  ARR_HIP(hipMemcpyAsync(perm, idx.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
  const int64_t mm = (int64_t)m * m;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, m, me, VT, perm, V);
  ARR_HIP(hipGetLastError());
  ARR_HIP(hipStreamSynchronize(s));
}

}  // namespace arr
