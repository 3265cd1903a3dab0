// Building blocks of the ARRABIT iteration on the device, shared by the
// solver driver and the step-level C entry points:
//  * poly_apply   -- Algorithm 7's polynomial on the shifted operator, one
//                    fused SpMM launch per degree (Horner recurrence, or the
//                    product of linear factors over psi_d's real roots), the
//                    column norms of the last degree accumulated in its
//                    epilogue;
//  * normalize    -- x_i = x_i / ||x_i|| (multi-power method, Sec. 3);
//  * project_out  -- X - Qc (Qc^T X) (Sec. 6, deflation);
//  * rcond_gram   -- rcond(X^T X) (eq. inn-stop);
//  * orthonormalize -- Cholesky QR, repeated, with a diagonal shift when the
//                    Gram is not numerically positive definite (the orth(Z)
//                    step of Algorithm 1);
//  * rayleigh_ritz -- H = U^T (A U), eigendecomposition, leading Ritz pairs.
#include <algorithm>
#include <cmath>

#include "steps.h"

namespace arr {

static size_t pad256(size_t b) { return (b + 255) / 256 * 256; }

size_t Work::reserve(int64_t n, int w, int m_max, int m_small, bool count_only) {
  const size_t b_partial = sizeof(double) * (size_t)spmm_groups(n) * (size_t)std::max(m_max, 1);
  const size_t b_colv = sizeof(double) * (size_t)std::max(m_max, 1);
  const size_t b_gram = sizeof(double) * gram_work_bound(n, m_max);
  const size_t b_small = sizeof(double) * (6 * (size_t)m_small * m_small + 128);
  const size_t b_proj = sizeof(double) * (size_t)std::max(w, 1) * (size_t)std::max(m_max, 1);
  const size_t b_info = 256;
  const size_t b_jac = jac.reserve_bytes(m_small);
  if (count_only)
    return pad256(b_partial) + pad256(b_colv) + pad256(b_gram) + pad256(b_small) + pad256(b_proj) + pad256(b_info) +
           b_jac;
  partial.ensure(b_partial);
  colv.ensure(b_colv);
  gramw.ensure(b_gram);
  small.ensure(b_small);
  proj.ensure(b_proj);
  info.ensure(b_info);
  this->jac.reserve(m_small);
  return 0;
}

void Work::ensure_cols(int64_t n, int w) {
  const size_t need = (size_t)spmm_groups(n) * (size_t)std::max(w, 1);
  partial.ensure(sizeof(double) * need);
  colv.ensure(sizeof(double) * std::max(w, 1));
  if (!info.p) info.alloc(256);
}

void Work::ensure_gram(int64_t n, int mx, int my) {
  gramw.ensure(sizeof(double) * std::max<size_t>(1, gram_work_doubles(n, mx, my)));
  if (!info.p) info.alloc(256);
}

void Work::ensure_small(int m) {
  const size_t per = (size_t)m * m;
  small.ensure(sizeof(double) * std::max<size_t>(1, 6 * per + 128));
  if (!info.p) info.alloc(256);
}

template <typename T>
void poly_apply_horner(const DevCSR<T> &A, Blk<T> X, Blk<T> Ya, Blk<T> Yb, double shift, double lo, double hi,
                const std::vector<double> &g, Work &wk, bool want_norms, hipStream_t s, const double *in_colss) {
  const int d = (int)g.size() - 1;
  ARR_REQUIRE(d >= 1, "poly: degree must be >= 1");
  ARR_REQUIRE(hi != lo, "poly: empty interval");
  const int w = X.w;
  double *partial = want_norms ? wk.partial.as<double>() : nullptr;
  ARR_REQUIRE(!in_colss || want_norms, "poly: deferred normalization needs the column norms");
  const double c0 = (lo + hi) / (lo - hi), c1 = 2.0 / (hi - lo);
  const Blk<const T> Xc{X.p, X.ld, w};
  const Blk<const T> none{nullptr, 0, 0};
  // Y_1 = c0 Y_0 + c1 (A - shift I) Y_0 + g1 X with Y_0 = g0 X
  const double al1 = c1 * g[0], be1 = g[0] * (c0 - c1 * shift) + g[1];
  const double al = c1, be = c0 - c1 * shift;
  SpmmChain chain(s);
  if (d == 1) {
    wk.groups = launch_filter_spmm<T>(A, Xc, none, Ya, al1, be1, 0.0, partial, s, in_colss);
    chain.close();
    launch_copy<T>(A.n, w, X.p, X.ld, Ya.p, Ya.ld, s);
    return;
  }
  launch_filter_spmm<T>(A, Xc, none, Ya, al1, be1, 0.0, nullptr, s);
  Blk<T> cur = Ya, nxt = Yb;
  for (int j = 2; j < d; ++j) {
    launch_filter_spmm<T>(A, Blk<const T>{cur.p, cur.ld, w}, Xc, nxt, al, be, g[j], nullptr, s);
    std::swap(cur, nxt);
  }
  // last degree writes X in place (Z = X is read row-locally before the store)
  wk.groups = launch_filter_spmm<T>(A, Blk<const T>{cur.p, cur.ld, w}, Xc, X, al, be, g[d], partial, s, in_colss);
  chain.close();
}

// The same polynomial as a product of linear factors over its real roots
// (Leja order): Y <- (c1 A + (c0 - c1 shift - r_i) I) Y, the leading
// coefficient folded into the first factor. One gathered read and one write
// per degree; the last degree writes X and (optionally) its column norms.
template <typename T>
void poly_apply_product(const DevCSR<T> &A, Blk<T> X, Blk<T> Ya, Blk<T> Yb, double shift, double lo, double hi,
                        const std::vector<double> &roots, double lead, Work &wk, bool want_norms, hipStream_t s,
                        const double *in_colss) {
  const int d = (int)roots.size();
  ARR_REQUIRE(d >= 1, "poly: degree must be >= 1");
  ARR_REQUIRE(hi != lo, "poly: empty interval");
  const int w = X.w;
  double *partial = want_norms ? wk.partial.as<double>() : nullptr;
  ARR_REQUIRE(!in_colss || want_norms, "poly: deferred normalization needs the column norms");
  const double c0 = (lo + hi) / (lo - hi), c1 = 2.0 / (hi - lo);
  const Blk<const T> none{nullptr, 0, 0};
  auto beta = [&](int i) { return c0 - c1 * shift - roots[i]; };
  SpmmChain chain(s);
  if (d == 1) {
    wk.groups = launch_filter_spmm<T>(A, Blk<const T>{X.p, X.ld, w}, none, Ya, lead * c1, lead * beta(0), 0.0,
                                      partial, s, in_colss);
    chain.close();
    launch_copy<T>(A.n, w, X.p, X.ld, Ya.p, Ya.ld, s);
    return;
  }
  launch_filter_spmm<T>(A, Blk<const T>{X.p, X.ld, w}, none, Ya, lead * c1, lead * beta(0), 0.0, nullptr, s);
  Blk<T> cur = Ya, nxt = Yb;
  for (int i = 1; i < d - 1; ++i) {
    launch_filter_spmm<T>(A, Blk<const T>{cur.p, cur.ld, w}, none, nxt, c1, beta(i), 0.0, nullptr, s);
    std::swap(cur, nxt);
  }
  wk.groups =
      launch_filter_spmm<T>(A, Blk<const T>{cur.p, cur.ld, w}, none, X, c1, beta(d - 1), 0.0, partial, s, in_colss);
  chain.close();
}

// The classic Chebyshev filter (eq. cheby-poly) in place of psi_d:
// X <- T_d(t) X with t = c0 I + c1 (A - shift I), by Y_1 = t X and
// Y_{j+1} = 2 t Y_j - Y_{j-1}: one fused SpMM per degree whose recurrence
// operand is Y_{j-1}. Y_j lives in buffer j mod 3 of (X, Ya, Yb); when d is
// not a multiple of 3 the result is copied into X.
template <typename T>
void poly_apply_chebyshev(const DevCSR<T> &A, Blk<T> X, Blk<T> Ya, Blk<T> Yb, double shift, double lo, double hi,
                          int d, Work &wk, bool want_norms, hipStream_t s, const double *in_colss) {
  ARR_REQUIRE(d >= 1, "poly: degree must be >= 1");
  ARR_REQUIRE(hi != lo, "poly: empty interval");
  const int w = X.w;
  double *partial = want_norms ? wk.partial.as<double>() : nullptr;
  ARR_REQUIRE(!in_colss || want_norms, "poly: deferred normalization needs the column norms");
  const double c0 = (lo + hi) / (lo - hi), c1 = 2.0 / (hi - lo);
  const double b1 = c0 - c1 * shift;  // t = c1 A + b1 I
  const Blk<T> buf[3] = {Blk<T>{X.p, X.ld, w}, Blk<T>{Ya.p, Ya.ld, w}, Blk<T>{Yb.p, Yb.ld, w}};
  auto in = [&](int j) { return Blk<const T>{buf[j % 3].p, buf[j % 3].ld, w}; };
  const Blk<const T> none{nullptr, 0, 0};
  SpmmChain chain(s);
  int groups = launch_filter_spmm<T>(A, in(0), none, buf[1], c1, b1, 0.0, d == 1 ? partial : nullptr, s,
                                     d == 1 ? in_colss : nullptr);
  for (int j = 1; j < d; ++j)
    groups = launch_filter_spmm<T>(A, in(j), in(j - 1), buf[(j + 1) % 3], 2.0 * c1, 2.0 * b1, -1.0,
                                   j == d - 1 ? partial : nullptr, s, j == d - 1 ? in_colss : nullptr);
  chain.close();
  if (d % 3 != 0) launch_copy<T>(A.n, w, X.p, X.ld, buf[d % 3].p, buf[d % 3].ld, s);
  if (want_norms) wk.groups = groups;
}

template <typename T>
void poly_apply(const DevCSR<T> &A, Blk<T> X, Blk<T> Ya, Blk<T> Yb, double shift, double lo, double hi,
                const FilterPoly &fp, int form, Work &wk, bool want_norms, hipStream_t s, const double *in_colss) {
  if (form == kPolyHorner)
    poly_apply_horner<T>(A, X, Ya, Yb, shift, lo, hi, fp.gamma, wk, want_norms, s, in_colss);
  else if (form == kPolyChebyshev)
    poly_apply_chebyshev<T>(A, X, Ya, Yb, shift, lo, hi, (int)fp.gamma.size() - 1, wk, want_norms, s, in_colss);
  else
    poly_apply_product<T>(A, X, Ya, Yb, shift, lo, hi, fp.roots, fp.lead, wk, want_norms, s, in_colss);
}

template <typename T>
void normalize_from_partial(int64_t n, Blk<T> X, Work &wk, hipStream_t s) {
  launch_reduce_groups(wk.partial.as<double>(), wk.groups, X.w, wk.colv.as<double>(), false, s);
  launch_scale_columns<T>(n, X, wk.colv.as<double>(), true, s);
}

template <typename T>
void normalize(int64_t n, Blk<T> X, Work &wk, hipStream_t s) {
  const Blk<const T> none{nullptr, 0, 0};
  wk.groups = launch_colsumsq<T>(n, Blk<const T>{X.p, X.ld, X.w}, none, nullptr, wk.partial.as<double>(), s);
  normalize_from_partial<T>(n, X, wk, s);
}

template <typename T>
void project_out(int64_t n, Blk<const T> Q, Blk<T> X, Work &wk, hipStream_t s, const double *colss) {
  if (X.w == 0) return;
  if (Q.w == 0) {
    if (colss) launch_scale_columns<T>(n, X, colss, true, s);
    return;
  }
  wk.ensure_gram(n, Q.w, X.w);
  wk.proj.ensure(sizeof(double) * (size_t)Q.w * X.w);
  double *C = wk.proj.as<double>();
  launch_gram<T>(n, Q, Blk<const T>{X.p, X.ld, X.w}, C, wk.gramw.as<double>(), false, s);
  launch_update<T>(n, Q, C, X.w, X.w, -1.0, 1.0, X, s, false, false, colss);
}

template <typename T>
void normalize_and_project(int64_t n, Blk<const T> Q, Blk<T> X, Work &wk, hipStream_t s) {
  launch_reduce_groups(wk.partial.as<double>(), wk.groups, X.w, wk.colv.as<double>(), false, s);
  project_out<T>(n, Q, X, wk, s, wk.colv.as<double>());
}

template <typename T>
double rcond_gram(int64_t n, Blk<const T> X, Work &wk, hipStream_t s) {
  const int w = X.w;
  wk.ensure_gram(n, w, w);
  wk.ensure_small(w);
  double *G = wk.small.as<double>();
  double *work = G + (size_t)w * w;
  double *rc = work + 5 * (size_t)w * w;
  launch_gram<T>(n, X, X, G, wk.gramw.as<double>(), true, s);
  rcond_device(w, G, work, wk.info.as<int>(), rc, s);
  double h = 0.0;
  ARR_HIP(hipMemcpyAsync(&h, rc, sizeof(double), hipMemcpyDeviceToHost, s));
  ARR_HIP(hipStreamSynchronize(s));
  return h;
}

// One GN inner iteration of Algorithm 8 (Sec. 2.6, unit step) with rho =
// Algorithm 7's poly on A - shift I over [lo, hi]:
//   Y = X (X^T X)^{-1},  Z = rho(A) Y,  X <- Z - X (Y^T Z - I) / 2.
// (X^T X)^{-1} = L^{-T} L^{-1} from the FP64 Cholesky factor of the Gram.
// Y, Z, Ya, Yb are n x w scratch blocks (Ya, Yb: the poly's ping-pong pair).
template <typename T>
void gn_step(const DevCSR<T> &A, Blk<T> X, Blk<T> Y, Blk<T> Z, Blk<T> Ya, Blk<T> Yb, double shift, double lo,
             double hi, const FilterPoly &fp, int form, Work &wk, hipStream_t s) {
  const int64_t n = A.n;
  const int w = X.w;
  if (w == 0) return;
  wk.ensure_gram(n, w, w);
  wk.ensure_small(w);
  const size_t ww = (size_t)w * w;
  double *G = wk.small.as<double>();
  double *Wt = G + ww;         // L^{-T}
  double *Gi = Wt + ww;        // (X^T X)^{-1}, later (Y^T Z - I) / 2
  double *scratch = Gi + ww;   // 2 w^2 for the triangular inverse
  const Blk<const T> Xc{X.p, X.ld, w};
  launch_gram<T>(n, Xc, Xc, G, wk.gramw.as<double>(), true, s);
  launch_cholesky(w, G, w, 0.0, wk.info.as<int>(), s);
  int info = 0;
  ARR_HIP(hipMemcpyAsync(&info, wk.info.as<int>(), sizeof(int), hipMemcpyDeviceToHost, s));
  ARR_HIP(hipStreamSynchronize(s));
  if (info) throw Error(-5, "GN step: X^T X is not numerically positive definite");
  launch_tri_inv_t(w, G, w, Wt, w, scratch, s);
  small_gemm(w, w, w, 1.0, Wt, w, 1, Wt, 1, w, 0.0, Gi, w, false, s);  // L^{-T} L^{-1}
  launch_update<T>(n, Xc, Gi, w, w, 1.0, 0.0, Y, s);                    // Y = X G^{-1}
  launch_copy<T>(n, w, Z.p, Z.ld, Y.p, Y.ld, s);
  poly_apply<T>(A, Z, Ya, Yb, shift, lo, hi, fp, form, wk, false, s);   // Z = rho(A) Y
  launch_gram<T>(n, Blk<const T>{Y.p, Y.ld, w}, Blk<const T>{Z.p, Z.ld, w}, Gi, wk.gramw.as<double>(), false, s);
  launch_half_minus_identity(w, Gi, s);                                 // (Y^T Z - I) / 2
  launch_update<T>(n, Xc, Gi, w, w, -1.0, 1.0, Z, s);                   // Z - X (Y^T Z - I) / 2
  launch_copy<T>(n, w, X.p, X.ld, Z.p, Z.ld, s);
}

// One Cholesky-QR pass: G = Z^T Z, G = L L^T, Zout = Z L^-T. If G is not
// numerically positive definite and allow_shift is set, the same Gram (kept
// aside, not recomputed) is factored again with the diagonal shift
// shift_rel * |G|_F of shifted Cholesky QR, and *shifted is set. Returns the
// (1-based) failing pivot column or 0.
template <typename T>
static int cholqr_pass(int64_t n, Blk<const T> Z, Blk<T> Zout, double shift_rel, bool allow_shift, Work &wk,
                       hipStream_t s, int *shifted, double **factor = nullptr) {
  const int m = Z.w;
  const size_t mm = (size_t)m * m;
  double *G = wk.small.as<double>();
  double *nrm = G + 2 * mm;        // 2 doubles
  double *scratch = nrm + 64;      // 2 m^2 doubles
  double *Gsave = scratch + 2 * mm;
  // R^{-1}: after G when applied here, else in the last m^2 of wk.small
  // (kept through the Rayleigh-Ritz step that applies it)
  double *Wt = factor ? Gsave + mm : G + mm;
  *shifted = 0;
  launch_gram<T>(n, Z, Z, G, wk.gramw.as<double>(), true, s);
  if (allow_shift) launch_copy<double>(m, m, Gsave, m, G, m, s);
  launch_cholesky(m, G, m, 0.0, wk.info.as<int>(), s);
  int info = 0;
  ARR_HIP(hipMemcpyAsync(&info, wk.info.as<int>(), sizeof(int), hipMemcpyDeviceToHost, s));
  ARR_HIP(hipStreamSynchronize(s));
  if (info && allow_shift) {
    launch_copy<double>(m, m, G, m, Gsave, m, s);
    launch_diag_max(m, G, m, nrm, s);
    double hn[2];
    ARR_HIP(hipMemcpyAsync(hn, nrm, sizeof(hn), hipMemcpyDeviceToHost, s));
    ARR_HIP(hipStreamSynchronize(s));
    launch_cholesky(m, G, m, shift_rel * hn[1], wk.info.as<int>(), s);
    ARR_HIP(hipMemcpyAsync(&info, wk.info.as<int>(), sizeof(int), hipMemcpyDeviceToHost, s));
    ARR_HIP(hipStreamSynchronize(s));
    *shifted = 1;
  }
  if (info) return info;
  launch_tri_inv_t(m, G, m, Wt, m, scratch, s);
  if (factor)
    *factor = Wt;
  else
    launch_update<T>(n, Z, Wt, m, m, 1.0, 0.0, Zout, s, true);
  return 0;
}

template <typename T>
Blk<T> orthonormalize(int64_t n, Blk<T> Z, Blk<T> Zalt, Blk<const T> Q, Work &wk, hipStream_t s, int *passes,
                      const double **rinv) {
  const int m = Z.w;
  wk.ensure_gram(n, m, m);
  wk.ensure_small(m);
  if (Q.w) wk.ensure_gram(n, Q.w, m);
  // shifted pass constant (shifted Cholesky QR): 11 (m n + m (m+1)) u |Z|^2
  const double u = std::is_same<T, float>::value ? 5.96e-8 : 1.11e-16;
  const double shift_rel = 11.0 * ((double)m * (double)n + (double)m * (m + 1)) * u;
  Blk<T> cur = Z, nxt = Zalt;
  int done_plain = 0, total = 0;
  if (rinv) *rinv = nullptr;
  // up to 2 plain passes after any shifted ones; at most 6 in all
  while (done_plain < 2 && total < 6) {
    if (Q.w) project_out<T>(n, Q, cur, wk, s);
    int shifted = 0;
    // the pass that closes the loop if it needs no shift may leave its factor
    // to the caller; a shifted one is applied here after all
    double *factor = nullptr;
    const bool closing = rinv && done_plain == 1 && total < 5;
    const int info = cholqr_pass<T>(n, Blk<const T>{cur.p, cur.ld, m}, nxt, shift_rel, true, wk, s, &shifted,
                                    closing ? &factor : nullptr);
    if (info) throw Error(-5, "Cholesky QR broke down even with a diagonal shift");
    ++total;
    if (closing && !shifted) {
      *rinv = factor;
      break;
    }
    if (closing) launch_update<T>(n, Blk<const T>{cur.p, cur.ld, m}, factor, m, m, 1.0, 0.0, nxt, s, true);
    done_plain = shifted ? 0 : done_plain + 1;
    std::swap(cur, nxt);
  }
  if (passes) *passes = total;
  return cur;
}

// Eigendecomposition of the m x m Rayleigh quotient H (wk.small) with the
// closing Cholesky-QR factor folded in (see rayleigh_ritz).
static void ritz_from_h(int m, Work &wk, std::vector<double> &evals, hipStream_t s, const double *rinv) {
  const size_t mm = (size_t)m * m;
  double *H = wk.small.as<double>();
  double *V = H + mm;
  double *T1 = V + mm + 64;  // below the factor rinv (last m^2 of wk.small)
  // the m x m products below run on the FP64 matrix cores as products with m
  // rows (R^{-1} is upper triangular)
  const Blk<const double> R{rinv, m, m};
  if (rinv) {
    // H <- R^{-T} (H R^{-1})
    launch_update<double>(m, Blk<const double>{H, m, m}, rinv, m, m, 1.0, 0.0, Blk<double>{T1, m, m}, s, true);
    wk.ensure_gram(m, m, m);
    launch_gram<double>(m, R, Blk<const double>{T1, m, m}, H, wk.gramw.as<double>(), false, s);
  }
  wk.jac.solve(m, H, V, evals, s, &wk.last_sweeps);
  if (rinv) {
    // V <- R^{-1} V
    launch_update<double>(m, R, V, m, m, 1.0, 0.0, Blk<double>{T1, m, m}, s, false);
    launch_copy<double>(m, m, V, m, T1, m, s);
  }
}

template <typename T>
void rayleigh_ritz(const DevCSR<T> &A, int64_t n, Blk<const T> U, Blk<T> W, Work &wk, std::vector<double> &evals,
                   hipStream_t s, const double *rinv) {
  const int m = U.w;
  const Blk<const T> none{nullptr, 0, 0};
  launch_filter_spmm<T>(A, U, none, W, 1.0, 0.0, 0.0, nullptr, s);
  wk.ensure_gram(n, m, m);
  wk.ensure_small(m);
  // H = U^T (A U) is symmetric: form its upper tiles and mirror them
  launch_gram<T>(n, U, Blk<const T>{W.p, W.ld, m}, wk.small.as<double>(), wk.gramw.as<double>(), true, s,
                 /*fp32_cores=*/true);
  ritz_from_h(m, wk, evals, s, rinv);
}

__global__ __launch_bounds__(256) void k_symmetrize(int m, double *__restrict__ H) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx / m), j = (int)(idx % m);
  if (i < j) {
    const double v = 0.5 * (H[(int64_t)i * m + j] + H[(int64_t)j * m + i]);
    H[(int64_t)i * m + j] = v;
    H[(int64_t)j * m + i] = v;
  }
}

template <typename T>
void rayleigh_ritz_chunked(const DevCSR<T> &A, int64_t n, Blk<const T> U, Blk<T> Tbuf, Work &wk,
                           std::vector<double> &evals, hipStream_t s, const double *rinv) {
  const int m = U.w, cw = Tbuf.w;
  ARR_REQUIRE(cw > 0, "chunked Rayleigh-Ritz: empty chunk buffer");
  const Blk<const T> none{nullptr, 0, 0};
  wk.ensure_small(m);
  const size_t mm = (size_t)m * m;
  double *H = wk.small.as<double>();
  // the column block U^T (A U[:, c0:c0+c]) is formed in V's place (free until
  // the eigensolve) and copied into H's columns
  double *Gc = H + mm;
  for (int c0 = 0; c0 < m; c0 += cw) {
    const int c = std::min(cw, m - c0);
    Blk<T> Tc{Tbuf.p, Tbuf.ld, c};
    launch_filter_spmm<T>(A, U.cols(c0, c), none, Tc, 1.0, 0.0, 0.0, nullptr, s);
    wk.ensure_gram(n, m, c);
    launch_gram<T>(n, U, Blk<const T>{Tc.p, Tc.ld, c}, Gc, wk.gramw.as<double>(), false, s, /*fp32_cores=*/true);
    launch_copy<double>(m, c, H + c0, m, Gc, c, s);
  }
  hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, m, H);
  ARR_HIP(hipGetLastError());
  ritz_from_h(m, wk, evals, s, rinv);
}

template <typename T>
std::vector<double> residual_norms(int64_t n, Blk<const T> AX, Blk<const T> X, const double *mu_dev, Work &wk,
                                   hipStream_t s) {
  const int w = X.w;
  std::vector<double> r(w);
  if (w == 0) return r;
  wk.ensure_cols(n, w);
  const int groups = launch_colsumsq<T>(n, AX, X, mu_dev, wk.partial.as<double>(), s);
  launch_reduce_groups(wk.partial.as<double>(), groups, w, wk.colv.as<double>(), true, s);
  ARR_HIP(hipMemcpyAsync(r.data(), wk.colv.as<double>(), sizeof(double) * w, hipMemcpyDeviceToHost, s));
  ARR_HIP(hipStreamSynchronize(s));
  return r;
}

#define ARR_INST(T)                                                                                              \
  template void poly_apply_horner<T>(const DevCSR<T> &, Blk<T>, Blk<T>, Blk<T>, double, double, double,          \
                                     const std::vector<double> &, Work &, bool, hipStream_t, const double *);    \
  template void poly_apply<T>(const DevCSR<T> &, Blk<T>, Blk<T>, Blk<T>, double, double, double,                 \
                              const FilterPoly &, int, Work &, bool, hipStream_t, const double *);               \
  template void normalize_from_partial<T>(int64_t, Blk<T>, Work &, hipStream_t);                                 \
  template void normalize<T>(int64_t, Blk<T>, Work &, hipStream_t);                                              \
  template void project_out<T>(int64_t, Blk<const T>, Blk<T>, Work &, hipStream_t, const double *);             \
  template void normalize_and_project<T>(int64_t, Blk<const T>, Blk<T>, Work &, hipStream_t);                   \
  template void gn_step<T>(const DevCSR<T> &, Blk<T>, Blk<T>, Blk<T>, Blk<T>, Blk<T>, double, double, double,    \
                           const FilterPoly &, int, Work &, hipStream_t);                                        \
  template double rcond_gram<T>(int64_t, Blk<const T>, Work &, hipStream_t);                                     \
  template Blk<T> orthonormalize<T>(int64_t, Blk<T>, Blk<T>, Blk<const T>, Work &, hipStream_t, int *,          \
                                    const double **);                                                           \
  template void rayleigh_ritz<T>(const DevCSR<T> &, int64_t, Blk<const T>, Blk<T>, Work &, std::vector<double> &, \
                                 hipStream_t, const double *);                                                   \
  template void rayleigh_ritz_chunked<T>(const DevCSR<T> &, int64_t, Blk<const T>, Blk<T>, Work &,              \
                                         std::vector<double> &, hipStream_t, const double *);                   \
  template std::vector<double> residual_norms<T>(int64_t, Blk<const T>, Blk<const T>, const double *, Work &,    \
                                                 hipStream_t);
ARR_INST(double)
ARR_INST(float)
#undef ARR_INST

}  // namespace arr
