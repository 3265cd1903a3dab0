// Device building blocks of the ARRABIT iteration (see steps.hip).
#pragma once

#include <vector>

#include "common.h"

namespace arr {

// Scratch shared by the building blocks; grows on demand.
struct Work {
  DevBuf partial;  // per-workgroup column partial sums
  DevBuf colv;     // per-column results
  DevBuf gramw;    // split-K partial tiles of the Gram products
  DevBuf small;    // small dense matrices (several m x m)
  DevBuf proj;     // Qc^T X coefficients of the deflation projection
  DevBuf info;     // device ints / scalars
  Jacobi jac;
  int groups = 0;
  int last_sweeps = 0;
  // Size every buffer for products of width <= m_max, blocks of width <= w
  // (deflation projections) and small matrices of order <= m_small, so that a
  // solve never allocates afterwards. Returns the bytes allocated (or, with
  // count_only, the bytes it would allocate).
  size_t reserve(int64_t n, int w, int m_max, int m_small, bool count_only);
  void ensure_cols(int64_t n, int w);
  void ensure_gram(int64_t n, int mx, int my);
  void ensure_small(int m);
};

// Algorithm 7 with the caller's monomial coefficients g (leading first).
template <typename T>
void poly_apply_horner(const DevCSR<T> &A, Blk<T> X, Blk<T> Ya, Blk<T> Yb, double shift, double lo, double hi,
                       const std::vector<double> &g, Work &wk, bool want_norms, hipStream_t s,
                       const double *in_colss = nullptr);
// psi_d in the chosen PolyForm. With in_colss (device, X.w values; needs
// want_norms) the result's column j is divided by sqrt(in_colss[j]) in the
// last launch: the polynomial is linear in X, so this equals filtering X
// with its columns normalized first (a deferred normalization).
template <typename T>
void poly_apply(const DevCSR<T> &A, Blk<T> X, Blk<T> Ya, Blk<T> Yb, double shift, double lo, double hi,
                const FilterPoly &fp, int form, Work &wk, bool want_norms, hipStream_t s,
                const double *in_colss = nullptr);
template <typename T>
void normalize_from_partial(int64_t n, Blk<T> X, Work &wk, hipStream_t s);
template <typename T>
void normalize(int64_t n, Blk<T> X, Work &wk, hipStream_t s);
// X <- X - Q (Q^T X); with colss (device, X.w values) the result's column j
// is also divided by sqrt(colss[j]) (the projection commutes with it).
template <typename T>
void project_out(int64_t n, Blk<const T> Q, Blk<T> X, Work &wk, hipStream_t s, const double *colss = nullptr);
// The multi-power normalization of the filter's output (column sums of
// squares left in wk.partial by its last SpMM) fused with the projection out
// of Q (deflation): one block pass instead of two when Q is not empty.
template <typename T>
void normalize_and_project(int64_t n, Blk<const T> Q, Blk<T> X, Work &wk, hipStream_t s);
// One GN inner iteration (Sec. 2.6, GN branch of Algorithm 8); Y, Z, Ya, Yb are
// n x X.w scratch blocks.
template <typename T>
void gn_step(const DevCSR<T> &A, Blk<T> X, Blk<T> Y, Blk<T> Z, Blk<T> Ya, Blk<T> Yb, double shift, double lo,
             double hi, const FilterPoly &fp, int form, Work &wk, hipStream_t s);
template <typename T>
double rcond_gram(int64_t n, Blk<const T> X, Work &wk, hipStream_t s);
// Orthonormal basis of R(Z) (and orthogonal to Q when Q.w > 0); Z and Zalt
// are n x m buffers used alternately; returns the one holding the result.
// With rinv != nullptr the factor of the closing Cholesky QR pass may be left
// unapplied: the returned block is then Q1 with basis Q1 R^{-1}, *rinv points
// to R^{-1} (upper triangular, m x m, ld m, inside wk.small, kept until the
// next Cholesky QR or small solve); otherwise *rinv = nullptr.
template <typename T>
Blk<T> orthonormalize(int64_t n, Blk<T> Z, Blk<T> Zalt, Blk<const T> Q, Work &wk, hipStream_t s, int *passes,
                      const double **rinv = nullptr);
// W = A U, H = U^T W, eigendecomposition of H: evals (descending, host) and the
// eigenvectors as columns of the m x m matrix at wk.small + m*m. With rinv
// (from orthonormalize) the basis is U R^{-1}: H = R^{-T} (U^T W) R^{-1}, and
// the matrix at wk.small + m*m is R^{-1} V, so that U (R^{-1} V) and
// W (R^{-1} V) are the Ritz vectors and their images.
template <typename T>
void rayleigh_ritz(const DevCSR<T> &A, int64_t n, Blk<const T> U, Blk<T> W, Work &wk, std::vector<double> &evals,
                   hipStream_t s, const double *rinv = nullptr);
// The same with A U formed in column chunks of Tbuf.w columns (Tbuf: n x
// Tbuf.w scratch) instead of a whole n x m block: H's columns c are
// U^T (A U[:, c]); H is then symmetrized. For the lean-memory mode.
template <typename T>
void rayleigh_ritz_chunked(const DevCSR<T> &A, int64_t n, Blk<const T> U, Blk<T> Tbuf, Work &wk,
                           std::vector<double> &evals, hipStream_t s, const double *rinv = nullptr);
template <typename T>
std::vector<double> residual_norms(int64_t n, Blk<const T> AX, Blk<const T> X, const double *mu_dev, Work &wk,
                                   hipStream_t s);

}  // namespace arr
