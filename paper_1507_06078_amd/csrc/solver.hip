// ARRABIT-MPM driver (Algorithm 8 with the heuristics of Sec. 6).
//
// The host keeps only scalars -- the interval [a, b], the continuation
// tolerance tol_t, the degree d, the augmentation count p, the Ritz values and
// residual norms -- and makes the decisions of Sec. 6 from them. Every block
// operation runs on the device: the filter SpMMs, normalization, deflation
// projections, Gram products, Cholesky/rcond, Cholesky-QR, the Jacobi
// eigensolve and the Ritz updates.
//
// Readings of the paper followed here (identical to the oracle's):
//  * the k smallest pairs are the k largest of -A;
//  * tol_1 = 1e-6 when tol <= 1e-8 (continuation), else tol;
//  * a = Lanczos theta_min - max(residual bound, 1e-3 spread) (in place of eigs);
//  * the ratio tests of eq. block and eq. hat-d use shifted values mu - a and
//    absolute values; no p update in the first outer iteration;
//  * deflated pairs are re-collected from the merged set every iteration;
//  * rcond is exact (1/(|G|_1 |G^-1|_1)), 0 if G is not positive definite.
#include "solver.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <cstdio>

namespace arr {

namespace {

// Partial dot products of the Lanczos reorthogonalization:
// part[r * nvec + c] = sum over rows of chunk r of V[c][i] w[i] (V: nvec
// contiguous vectors of length n). Summed per c in a fixed order afterwards.
constexpr int kDotChunks = 128;
__global__ __launch_bounds__(256) void k_dots_partial(int64_t n, const double *__restrict__ V, int nvec,
                                                      const double *__restrict__ w, int64_t chunk,
                                                      double *__restrict__ part) {
  __shared__ double red[256];
  const int c = blockIdx.y, r = blockIdx.x;
  const double *v = V + (int64_t)c * n;
  const int64_t i0 = (int64_t)r * chunk, i1 = min(n, i0 + chunk);
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s = fma(v[i], w[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)r * nvec + c] = red[0];
}

// w[i] -= sum_{c<j} V[c][i] h[c]
__global__ __launch_bounds__(256) void k_sub_combination(int64_t n, int j, const double *__restrict__ V,
                                                         const double *__restrict__ h, double *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int c = 0; c < j; ++c) s -= V[(int64_t)c * n + i] * h[c];
  w[i] = s;
}

__global__ __launch_bounds__(256) void k_scale_vec(int64_t n, const double *__restrict__ x, const double *nrm2,
                                                   double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] / sqrt(*nrm2);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

// h[c] = V[c] . w for c < nvec, deterministic; part >= kDotChunks * nvec doubles.
void multi_dot(int64_t n, const double *V, int nvec, const double *w, double *part, double *h, hipStream_t s) {
  const int64_t chunk = (n + kDotChunks - 1) / kDotChunks;
  hipLaunchKernelGGL(k_dots_partial, dim3(kDotChunks, nvec), dim3(256), 0, s, n, V, nvec, w, chunk, part);
  ARR_HIP(hipGetLastError());
  launch_reduce_groups(part, kDotChunks, nvec, h, false, s);
}

}  // namespace

Solver::Solver(const arr_csr_t *csr, int64_t n, int k, int which, double tol, const arr_options_t &o)
    : n_(n), k_(k), which_(which), tol_(tol), o_(o) {
  ARR_REQUIRE(csr != nullptr, "csr is NULL");
  ARR_REQUIRE(csr->n == n && n > 0, "csr->n must equal n > 0");
  ARR_REQUIRE(csr->rowptr && (csr->nnz == 0 || (csr->colind && csr->val)), "csr arrays are NULL");
  ARR_REQUIRE(which == ARR_LARGEST_ALGEBRAIC || which == ARR_SMALLEST_ALGEBRAIC, "which must be LARGEST or SMALLEST");
  ARR_REQUIRE(tol > 0.0 && std::isfinite(tol), "tol must be positive");
  ARR_REQUIRE(k > 0 && k < n, "k must satisfy 0 < k < n");
  w_ = o.w > 0 ? o.w : k + (int)std::lround(0.1 * k);
  ARR_REQUIRE(w_ >= k, "block width w must be >= k");
  ARR_REQUIRE(o.p0 >= 0 && o.p_max >= o.p0, "need 0 <= p0 <= p_max");
  ARR_REQUIRE((int64_t)(o.p_max + 1) * w_ < n, "need (p_max + 1) * w < n (Algorithm 8)");
  ARR_REQUIRE(o.d0 >= 1 && o.d_max >= o.d0 && o.d_max <= 64, "need 1 <= d0 <= d_max <= 64");
  ARR_REQUIRE(o.maxit >= 1 && o.maxit1 >= 1 && o.maxit2 >= 1, "iteration limits must be >= 1");
  ARR_REQUIRE(o.mixed_contin >= 0.0, "mixed_contin must be >= 0");
  ARR_REQUIRE(o.early_contin >= 0.0, "early_contin must be >= 0");
  ARR_REQUIRE(o.precision == ARR_FP64 || o.precision == ARR_MIXED, "unknown precision");
  ARR_REQUIRE(o.inner_solver == ARR_INNER_MPM || o.inner_solver == ARR_INNER_GN, "unknown inner solver");
  ARR_REQUIRE(o.poly_form == ARR_POLY_PRODUCT || o.poly_form == ARR_POLY_HORNER || o.poly_form == ARR_POLY_CHEBYSHEV,
              "unknown polynomial form");
  ARR_REQUIRE(o.row_form >= ARR_ROW_AUTO && o.row_form <= ARR_ROW_GRID,
              "unknown row form");
  ARR_REQUIRE(o.lean_memory == 0 || o.lean_memory == 1, "lean_memory must be 0 or 1");
  ARR_REQUIRE(o.lean_memory == 0 || o.inner_solver == ARR_INNER_MPM, "the lean-memory mode needs the MPM inner solver");
  lean_ = o.lean_memory != 0;
  // validate CSR on the host
  const int64_t *rp = csr->rowptr;
  ARR_REQUIRE(rp[0] == 0 && rp[n] == csr->nnz, "rowptr[0] must be 0 and rowptr[n] must equal nnz");
  for (int64_t i = 0; i < n; ++i) {
    ARR_REQUIRE(rp[i + 1] >= rp[i], "rowptr must be non-decreasing");
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
      const int32_t c = csr->colind[q];
      ARR_REQUIRE(c >= 0 && c < n, "column index out of range");
      ARR_REQUIRE(q == rp[i] || csr->colind[q - 1] < c, "column indices must be strictly increasing within a row");
      ARR_REQUIRE(std::isfinite(csr->val[q]), "matrix values must be finite");
    }
  }
  // symmetry: every (i, c, v) has its mirror (c, i, v)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
      const int32_t c = csr->colind[q];
      const int32_t *b = csr->colind + rp[c], *e = csr->colind + rp[c + 1];
      const int32_t *f = std::lower_bound(b, e, (int32_t)i);
      ARR_REQUIRE(f != e && *f == i && csr->val[rp[c] + (f - b)] == csr->val[q], "matrix is not symmetric");
    }
  }
  // working operator (A, or -A for the smallest end) in the split form
  split_rows(n, rp, csr->colind, csr->val, h_split_, o.row_form);
  nnz_ = csr->nnz;
  if (which == ARR_SMALLEST_ALGEBRAIC) {
    for (double &x : h_split_.coef) x = -x;
    for (double &x : h_split_.oval) x = -x;
  }
  ldz_ = round_up((int64_t)std::max(o.p_max + 1, 2) * w_, 8);
  ldq_ = round_up(w_, 8);
  lanczos_L_ = (int)std::max<int64_t>(1, std::min<int64_t>(o.lanczos_steps, n));
}

// Every device buffer of a solve, in one place: with allocate = false the
// padded byte count is returned (the footprint a server reserves).
size_t Solver::device_plan(bool allocate) {
  const int64_t n = n_, no = (int64_t)h_split_.ocol.size();  // overflow entries
  const bool mixed = o_.precision == ARR_MIXED;
  size_t total = 0;
  auto take = [&](DevBuf &b, size_t bytes) {
    total += (bytes + 255) / 256 * 256;
    if (allocate) b.alloc(bytes);
  };
  take(coef64_, sizeof(double) * 8 * n);
  if (!h_split_.gx) take(fcol_, sizeof(int32_t) * 4 * n);
  if (no) {
    take(orp_, sizeof(int64_t) * (n + 1));
    take(ocol_, sizeof(int32_t) * no);
    take(oval64_, sizeof(double) * no);
  }
  if (mixed) {
    take(coef32_, sizeof(float) * 8 * n);
    if (no) take(oval32_, sizeof(float) * no);
  }
  // lean: no A U block (chunks of ldt columns instead) and no output block
  const int64_t ldt64 = std::min<int64_t>(ldz_, 256), ldt32 = std::min<int64_t>(ldz_, 512);
  // The FP32 stage's blocks live inside FP64 blocks that the FP32 stage does
  // not use: its Z and U in the two halves of the FP64 U block (256 bytes of
  // slack keep the second half 256-byte aligned), its W (or chunk buffer) in
  // the FP64 W (chunk) block. It locks nothing, so it has no Q blocks. The
  // handover converts its Z into the FP64 Z block, which it never touched.
  const size_t half32 = (sizeof(float) * n * ldz_ + 255) / 256 * 256;
  take(B64_.Zb, sizeof(double) * n * ldz_);
  take(B64_.Ub, sizeof(double) * n * ldz_ + (mixed ? 256 : 0));
  if (lean_)
    take(B64_.Tb, sizeof(double) * n * ldt64);
  else
    take(B64_.Wb, sizeof(double) * n * ldz_);
  for (DevBuf *b : {&B64_.Qb, &B64_.Q2b}) take(*b, sizeof(double) * n * ldq_);
  if (mixed && allocate) {
    B32_.Zb.view(B64_.Ub.p, sizeof(float) * n * ldz_);
    B32_.Ub.view(B64_.Ub.as<char>() + half32, sizeof(float) * n * ldz_);
    if (lean_)
      B32_.Tb.view(B64_.Tb.p, sizeof(float) * n * ldt32);
    else
      B32_.Wb.view(B64_.Wb.p, sizeof(float) * n * ldz_);
    B32_.Qb.release();
    B32_.Q2b.release();
  }
  take(mu_, sizeof(double) * ldz_);
  take(desc_, (sizeof(void *) + sizeof(int64_t) + sizeof(int32_t)) * (size_t)ldz_ + 64);
  if (!lean_) take(outv_, sizeof(double) * n * k_);
  if (have_x0_) take(x0_, sizeof(double) * n * w_);
  const int L = lanczos_L_;
  take(lz_V_, sizeof(double) * n * L);
  take(lz_w_, sizeof(double) * n);
  take(lz_h_, sizeof(double) * (L + 4));
  take(lz_part_, sizeof(double) * 128 * (L + 1));
  const int m_small = (int)std::max<int64_t>(ldz_, L);
  total += wk_.reserve(n, w_, (int)ldz_, m_small, !allocate);
  return total;
}

void Solver::ensure_device() {
  if (device_ready_) return;
  ARR_HIP(hipSetDevice(o_.device));
  if (!s_) ARR_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
  device_plan(true);
  const int64_t n = n_, no = (int64_t)h_split_.ocol.size();
  const bool mixed = o_.precision == ARR_MIXED;
  ARR_HIP(hipMemcpyAsync(coef64_.p, h_split_.coef.data(), sizeof(double) * 8 * n, hipMemcpyHostToDevice, s_));
  if (!h_split_.gx)
    ARR_HIP(hipMemcpyAsync(fcol_.p, h_split_.fcol.data(), sizeof(int32_t) * 4 * n, hipMemcpyHostToDevice, s_));
  if (mixed) launch_convert<float, double>(8 * n, 1, coef32_.as<float>(), 1, coef64_.as<double>(), 1, s_);
  if (no) {
    ARR_HIP(hipMemcpyAsync(orp_.p, h_split_.orp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s_));
    ARR_HIP(hipMemcpyAsync(ocol_.p, h_split_.ocol.data(), sizeof(int32_t) * no, hipMemcpyHostToDevice, s_));
    ARR_HIP(hipMemcpyAsync(oval64_.p, h_split_.oval.data(), sizeof(double) * no, hipMemcpyHostToDevice, s_));
    if (mixed) launch_convert<float, double>(no, 1, oval32_.as<float>(), 1, oval64_.as<double>(), 1, s_);
  }
  if (have_x0_)
    ARR_HIP(hipMemcpyAsync(x0_.p, h_x0_.data(), sizeof(double) * n * w_, hipMemcpyHostToDevice, s_));
  const int64_t *orp = no ? orp_.as<int64_t>() : nullptr;
  const int32_t *ocol = no ? ocol_.as<int32_t>() : nullptr;
  A64_ = DevCSR<double>{n, nnz_, coef64_.as<double>(), fcol_.as<int32_t>(), orp, ocol,
                        no ? oval64_.as<double>() : nullptr, h_split_.pair, h_split_.kf,
                        h_split_.gx, h_split_.gy, h_split_.gz};
  if (mixed)
    A32_ = DevCSR<float>{n, nnz_, coef32_.as<float>(), fcol_.as<int32_t>(), orp, ocol,
                         no ? oval32_.as<float>() : nullptr, h_split_.pair, h_split_.kf,
                         h_split_.gx, h_split_.gy, h_split_.gz};
  B64_.ldz = ldz_;
  B64_.ldq = ldq_;
  B32_.ldz = ldz_;
  B32_.ldq = ldq_;
  B64_.ldt = lean_ ? std::min<int64_t>(ldz_, 256) : 0;
  B32_.ldt = lean_ ? std::min<int64_t>(ldz_, 512) : 0;
  ARR_HIP(hipStreamSynchronize(s_));
  device_ready_ = true;
}

void Solver::release_device() {
  if (s_) ARR_HIP(hipStreamSynchronize(s_));
  for (DevBuf *b : {&coef64_, &coef32_, &fcol_, &orp_, &ocol_, &oval64_, &oval32_, &B64_.Zb, &B64_.Ub, &B64_.Wb, &B64_.Qb, &B64_.Q2b,
                    &B64_.Tb, &B32_.Zb, &B32_.Ub, &B32_.Wb, &B32_.Qb, &B32_.Q2b, &B32_.Tb, &mu_, &desc_, &outv_, &x0_, &lz_V_, &lz_w_, &lz_h_,
                    &lz_part_, &wk_.partial, &wk_.colv, &wk_.gramw, &wk_.small, &wk_.proj, &wk_.info, &wk_.jac.bufA,
                    &wk_.jac.bufB, &wk_.jac.bufV, &wk_.jac.bufOff, &wk_.jac.bufEval})
    b->release();
  wk_.jac.mcap = 0;
  device_ready_ = false;
}

void Solver::stash_results(bool keep_vectors) {
  if (!solved) return;
  if (keep_vectors) {
    h_vecs_.resize((size_t)n_ * k_);
    ARR_HIP(hipMemcpy2D(h_vecs_.data(), sizeof(double) * k_, outv_p_, sizeof(double) * outv_ld_, sizeof(double) * k_,
                        n_, hipMemcpyDeviceToHost));
  } else {
    h_vecs_.clear();
  }
  host_results_ = true;
}

Solver::~Solver() {
  if (s_) (void)hipStreamDestroy(s_);
}

double Solver::now() const {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
}

const FilterPoly &Solver::coeffs(int d) {
  auto it = coef_.find(d);
  if (it == coef_.end()) it = coef_.emplace(d, filter_poly(d)).first;
  return it->second;
}

void Solver::set_initial_block(const double *X0, int64_t ld) {
  ARR_REQUIRE(X0 != nullptr && ld >= w_, "initial block: NULL or ld < w");
  ARR_REQUIRE(!device_ready_, "arr_set_initial_block must precede the first arr_solve");
  h_x0_.resize((size_t)n_ * w_);
  for (int64_t i = 0; i < n_; ++i) std::copy(X0 + i * ld, X0 + i * ld + w_, h_x0_.begin() + i * w_);
  have_x0_ = true;
}

// Interval [a, b] of Sec. 6 'Estimation of lambda_n and lambda_{k+q}':
// a from Lanczos with full reorthogonalization started at X0[:, 0] (in place of
// eigs), b = smallest Ritz value of the starting block.
void Solver::setup_interval() {
  const int64_t n = n_;
  const int L = lanczos_L_;
  double *Vp = lz_V_.as<double>(), *w = lz_w_.as<double>(), *hp = lz_h_.as<double>(), *pp = lz_part_.as<double>();
  // v_0 = X0[:, 0] / |X0[:, 0]|
  launch_copy<double>(n, 1, w, 1, B64_.Zb.as<double>(), B64_.ldz, s_);
  multi_dot(n, w, 1, w, pp, hp, s_);
  hipLaunchKernelGGL(k_scale_vec, dim3(blocks_for(n)), dim3(256), 0, s_, n, w, hp, Vp);
  ARR_HIP(hipGetLastError());
  std::vector<double> alpha, beta;
  for (int j = 0; j < L; ++j) {
    double *vj = Vp + (int64_t)j * n;
    launch_spmv<double>(A64_, vj, w, s_);
    // full reorthogonalization, twice; the first pass also yields alpha_j
    double aj = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      multi_dot(n, Vp, j + 1, w, pp, hp, s_);
      if (pass == 0) ARR_HIP(hipMemcpyAsync(&aj, hp + j, sizeof(double), hipMemcpyDeviceToHost, s_));
      hipLaunchKernelGGL(k_sub_combination, dim3(blocks_for(n)), dim3(256), 0, s_, n, j + 1, Vp, hp, w);
    }
    multi_dot(n, w, 1, w, pp, hp + L, s_);
    ARR_HIP(hipGetLastError());
    double b2 = 0.0;
    ARR_HIP(hipMemcpyAsync(&b2, hp + L, sizeof(double), hipMemcpyDeviceToHost, s_));
    ARR_HIP(hipStreamSynchronize(s_));
    alpha.push_back(aj);
    beta.push_back(std::sqrt(std::max(0.0, b2)));
    if (beta.back() <= 1e-14 * std::max(1.0, std::fabs(aj)) || j == L - 1) break;
    hipLaunchKernelGGL(k_scale_vec, dim3(blocks_for(n)), dim3(256), 0, s_, n, w, hp + L, Vp + (int64_t)(j + 1) * n);
    ARR_HIP(hipGetLastError());
  }
  const int m = (int)alpha.size();
  std::vector<double> T((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) {
    T[(size_t)i * m + i] = alpha[i];
    if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = beta[i];
  }
  wk_.ensure_small(std::max(m, w_));
  double *Td = wk_.small.as<double>(), *Vt = Td + (size_t)m * m;
  ARR_HIP(hipMemcpyAsync(Td, T.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, s_));
  std::vector<double> th;
  wk_.jac.solve(m, Td, Vt, th, s_);
  double slast = 0.0;  // last component of the eigenvector of theta_min (last column)
  ARR_HIP(hipMemcpyAsync(&slast, Vt + (size_t)(m - 1) * m + (m - 1), sizeof(double), hipMemcpyDeviceToHost, s_));
  ARR_HIP(hipStreamSynchronize(s_));
  const double tmin = th[m - 1], tmax = th[0];
  const double r = std::fabs(beta[m - 1] * slast);
  a_ = tmin - std::max(r, 1e-3 * (tmax - tmin));
  norm_ = std::max(std::fabs(tmin), std::fabs(tmax));

  // b: smallest Ritz value of the starting block
  Blocks<double> &B = B64_;
  launch_copy<double>(n, w_, B.Ub.as<double>(), B.ldz, B.Zb.as<double>(), B.ldz, s_);
  const Blk<const double> none{nullptr, 0, 0};
  Blk<double> U = orthonormalize<double>(n, B.U(0, w_), B.U(w_, w_), none, wk_, s_, nullptr);
  Blk<double> Wt = (U.p == B.Ub.as<double>()) ? B.U(w_, w_) : B.U(0, w_);
  std::vector<double> ev;
  rayleigh_ritz<double>(A64_, n, Blk<const double>{U.p, U.ld, w_}, Wt, wk_, ev, s_);
  b_ = ev[w_ - 1];
}

int Solver::degree_update(double mu_k, double mu_w) {
  // eq. hat-d / eq. degree with rho_d(t) = psi_d((2t - a - b)/(b - a)), or
  // T_d of eq. cheby-poly at the same point in the Chebyshev mode
  auto rho = [&](int d, double t) {
    const double x = (2.0 * t - a_ - b_) / (b_ - a_);
    if (o_.poly_form == ARR_POLY_CHEBYSHEV) {
      double tp = 1.0, tc = x;
      for (int j = 1; j < d; ++j) {
        const double tn = 2.0 * x * tc - tp;
        tp = tc;
        tc = tn;
      }
      return tc;
    }
    double v = 0.0;
    for (double c : coeffs(d).gamma) v = v * x + c;
    return v;
  };
  for (int d = 3; d <= o_.d_max; ++d) {
    const double num = std::fabs(rho(d, mu_w)), den = std::fabs(rho(d, mu_k));
    if (den > 0.0 && num / den < 0.9) return d;
  }
  return o_.d_max;
}

template <typename T>
void Solver::gather(int64_t n, int w, T *dst, int64_t lddst, const std::vector<const T *> &src,
                    const std::vector<int64_t> &lds, const std::vector<int32_t> &cols) {
  if (w == 0) return;
  char *base = desc_.as<char>();
  const T **dsrc = reinterpret_cast<const T **>(base);
  int64_t *dlds = reinterpret_cast<int64_t *>(base + sizeof(void *) * B64_.ldz);
  int32_t *dcols = reinterpret_cast<int32_t *>(base + (sizeof(void *) + sizeof(int64_t)) * B64_.ldz);
  ARR_HIP(hipMemcpyAsync(dsrc, src.data(), sizeof(void *) * w, hipMemcpyHostToDevice, s_));
  ARR_HIP(hipMemcpyAsync(dlds, lds.data(), sizeof(int64_t) * w, hipMemcpyHostToDevice, s_));
  ARR_HIP(hipMemcpyAsync(dcols, cols.data(), sizeof(int32_t) * w, hipMemcpyHostToDevice, s_));
  launch_gather_columns<T>(n, w, dst, lddst, dsrc, dlds, dcols, s_);
  // the host vectors may be reused right away
  ARR_HIP(hipStreamSynchronize(s_));
}

// Final output: the k leading merged pairs, re-checked with an explicit FP64
// SpMM. Returns the largest of their residuals in the eq. resi scaling. Uses
// only outv_ and the FP64 W block, which no later step of an outer iteration
// reads before writing, so the iteration may continue after it.
template <typename T>
double Solver::finish(Blocks<T> &B, const DevCSR<T> &A, const std::vector<const T *> &src,
                      const std::vector<int64_t> &lds, const std::vector<int32_t> &cols, const std::vector<double> &mu,
                      T *free) {
  (void)A;
  const int64_t n = n_;
  const int k = k_;
  std::vector<const T *> s(src.begin(), src.begin() + k);
  std::vector<int64_t> l(lds.begin(), lds.begin() + k);
  std::vector<int32_t> c(cols.begin(), cols.begin() + k);
  // lean: the vectors in columns [0, k) of a free FP64 block, A X in [k, 2k)
  // (ld >= 2 w >= 2 k); otherwise the output block and the W block
  const bool fp64 = std::is_same<T, double>::value;
  double *AXp;
  int64_t ldax;
  if (lean_) {
    outv_p_ = fp64 ? reinterpret_cast<double *>(free) : B64_.Ub.as<double>();
    outv_ld_ = ldz_;
    AXp = outv_p_ + k;
    ldax = ldz_;
  } else {
    outv_p_ = outv_.as<double>();
    outv_ld_ = k;
    AXp = B64_.Wb.as<double>();
    ldax = ldz_;
  }
  if (fp64) {
    gather<T>(n, k, reinterpret_cast<T *>(outv_p_), outv_ld_, s, l, c);
  } else {
    T *stage = lean_ ? free : B.W(0, k).p;
    gather<T>(n, k, stage, B.ldz, s, l, c);
    launch_convert<double, T>(n, k, outv_p_, outv_ld_, stage, B.ldz, s_);
  }
  // explicit FP64 residuals
  Blk<double> X{outv_p_, outv_ld_, k};
  Blk<double> AX{AXp, ldax, k};
  const Blk<const double> none{nullptr, 0, 0};
  launch_filter_spmm<double>(A64_, Blk<const double>{X.p, X.ld, k}, none, AX, 1.0, 0.0, 0.0, nullptr, s_);
  ARR_HIP(hipMemcpyAsync(mu_.p, mu.data(), sizeof(double) * k, hipMemcpyHostToDevice, s_));
  std::vector<double> rn = residual_norms<double>(n, Blk<const double>{AX.p, AX.ld, k},
                                                  Blk<const double>{X.p, X.ld, k}, mu_.as<double>(), wk_, s_);
  out_vals_.assign(mu.begin(), mu.begin() + k);
  out_res_.resize(k);
  out_rn_.assign(rn.begin(), rn.begin() + k);
  double worst = 0.0, worst_a = 0.0;
  for (int i = 0; i < k; ++i) {
    out_res_[i] = rn[i] / std::max(1.0, std::fabs(mu[i]));
    worst = std::max(worst, out_res_[i]);
    worst_a = std::max(worst_a, rn[i] / norm_);
    if (!(out_res_[i] == out_res_[i])) worst = worst_a = std::numeric_limits<double>::infinity();
  }
  stats.maxres_explicit = worst;
  stats.maxres_norm_a = worst_a;
  if (which_ == ARR_SMALLEST_ALGEBRAIC)
    for (double &v : out_vals_) v = -v;
  return worst;
}

// Test hook of the non-finite guard: a NaN written into X(0, 0) after the
// filter application chosen by debug_nan_poly.
template <typename T>
void Solver::poly_hook(Blk<T> X) {
  ++poly_count_;
  const int at = o_.debug_nan_poly;
  if (at == 0 || X.w == 0) return;
  if ((at > 0 && poly_count_ == at) || (at < 0 && poly_count_ >= -at)) {
    const T nan = std::numeric_limits<T>::quiet_NaN();
    ARR_HIP(hipMemcpyAsync(X.p, &nan, sizeof(T), hipMemcpyHostToDevice, s_));
    ARR_HIP(hipStreamSynchronize(s_));
  }
}

// Outer iterations of Algorithm 8 in block precision T. Returns a status
// (>= 0) when the solve ends, or -100 to hand over to the FP64 stage.
template <typename T>
int Solver::outer(Blocks<T> &B, const DevCSR<T> &A, bool fp32_stage) {
  const int64_t n = n_;
  const int k = k_, w = w_;
  const int fp32_limit = std::max(1, o_.maxit / 2);
  int fp32_iters = 0, fp32_since_best = 0;
  double fp32_best = std::numeric_limits<double>::infinity();
  for (; j_ < o_.maxit;) {
    ++j_;
    stats.outer_iters = j_;
    double t = now();
    // ---- subspace update: MPM on A - aI over [0, b - a] ----
    Blk<T> X = B.Z(0, wp_);
    const Blk<const T> Qc{B.Qb.template as<T>(), B.ldq, nc_};
    {
    // the filter's ping-pong pair: two compact n x ldc blocks in U when they
    // fit (rows of ldc values stream faster than rows strided by ldz)
    const int64_t ldc = round_up((int64_t)wp_, 8);
    const bool compact = 2 * ldc <= B.ldz;
    Blk<T> Ya = compact ? Blk<T>{B.Ub.template as<T>(), ldc, wp_} : B.U(0, wp_);
    Blk<T> Yb = compact ? Blk<T>{B.Ub.template as<T>() + n * ldc, ldc, wp_} : B.U(wp_, wp_);
    wk_.ensure_cols(n, wp_);
    // Non-finite guard: the MPM iterate is kept in W (free until the
    // Rayleigh-Ritz step) at the start of the filter stage. A check that finds
    // a NaN or Inf column norm restores it, renormalizes and restarts the
    // inner loop at half the degree, once per outer iteration.
    const bool mpm = o_.inner_solver != ARR_INNER_GN;
    const Blk<T> snap = lean_ ? B.Z(wp_, wp_) : B.W(0, wp_);  // Z's Krylov columns are free here
    if (mpm) launch_copy<T>(n, wp_, snap.p, snap.ld, X.p, X.ld, s_);
    int retries = 0;
  restart_inner:
    const FilterPoly &g = coeffs(d_);
    double rc = std::numeric_limits<double>::infinity();
    for (int i1 = 0; i1 < o_.maxit1; ++i1) {
      // MPM with Qc empty: X's column normalization is deferred into the last
      // launch of the next filter (the filter is linear in X) and applied on
      // its own only before the inner stop check
      bool pending = false;
      for (int i2 = 0; i2 < o_.maxit2; ++i2) {
        if (o_.inner_solver == ARR_INNER_GN) {
          // GN branch: no normalization; Y in Z's second segment, rho(A) Y in W
          gn_step<T>(A, X, B.Z(wp_, wp_), B.W(0, wp_), Ya, Yb, a_, 0.0, b_ - a_, g, o_.poly_form, wk_, s_);
          poly_hook<T>(X);
          if (nc_) project_out<T>(n, Qc, X, wk_, s_);
        } else {
          // MPM: normalize the columns, then X - Qc (Qc^T X); the scaling rides
          // in the projection's update when Qc is not empty
          poly_apply<T>(A, X, Ya, Yb, a_, 0.0, b_ - a_, g, o_.poly_form, wk_, true, s_,
                        pending ? wk_.colv.as<double>() : nullptr);
          poly_hook<T>(X);
          if (nc_) {
            normalize_and_project<T>(n, Qc, X, wk_, s_);
          } else {
            launch_reduce_groups(wk_.partial.as<double>(), wk_.groups, wp_, wk_.colv.as<double>(), false, s_);
            pending = true;
          }
        }
        stats.poly_calls += 1;
        stats.spmm_degrees += d_;
        stats.spmm_cols += (int64_t)d_ * wp_;
      }
      if (pending) launch_scale_columns<T>(n, X, wk_.colv.as<double>(), true, s_);
      const double rcp = rc;
      rc = rcond_gram<T>(n, Blk<const T>{X.p, X.ld, wp_}, wk_, s_);
      // the last filter application's column norms (MPM) or the Gram (GN)
      bool finite = std::isfinite(rc);
      if (mpm && finite) {
        std::vector<double> cs(wp_);
        ARR_HIP(hipMemcpy(cs.data(), wk_.colv.as<double>(), sizeof(double) * wp_, hipMemcpyDeviceToHost));
        for (double v : cs) finite = finite && std::isfinite(v);
      }
      if (!finite) {
        if (!mpm || retries > 0)
          throw Error(ARR_EBREAKDOWN, "non-finite values in the filtered block (outer iteration " +
                                          std::to_string(j_) + ", degree " + std::to_string(d_) + ")");
        ++retries;
        stats.nan_retries += 1;
        d_ = std::max(1, d_ / 2);
        launch_copy<T>(n, wp_, X.p, X.ld, snap.p, snap.ld, s_);
        normalize<T>(n, X, wk_, s_);
        if (nc_) project_out<T>(n, Qc, X, wk_, s_);
        goto restart_inner;
      }
      const double thr = fp32_stage ? std::max(tol_t_, 1e-6) : tol_t_;
      if (o_.verbose >= 2) {
        std::fprintf(stderr, "[arr]   inner check %d (%d filter calls of degree %d): rcond %.3e\n", i1 + 1,
                     (i1 + 1) * o_.maxit2, d_, rc);
        std::fflush(stderr);
      }
      if (rc <= thr || rc / rcp > 0.99) break;
    }
    }
    ARR_HIP(hipStreamSynchronize(s_));
    stats.t_filter += now() - t;
    t = now();
    // ---- augmentation [X, AX, ..., A^p X] (eq. S:ARR) in Z ----
    const Blk<const T> none{nullptr, 0, 0};
    for (int i = 1; i <= p_; ++i) {
      launch_filter_spmm<T>(A, Blk<const T>{B.Z((i - 1) * wp_, wp_).p, B.ldz, wp_}, none, B.Z(i * wp_, wp_), 1.0,
                            0.0, 0.0, nullptr, s_);
      stats.spmm_degrees += 1;
      stats.spmm_cols += wp_;
    }
    const int m = (p_ + 1) * wp_;
    // ---- RR on the projection onto R(Qc)^perp (Algorithm 1, Sec. 6) ----
    const double td = now();
    // the closing Cholesky QR factor rides in the small Rayleigh-Ritz problem
    const double *rinv = nullptr;
    Blk<T> U = orthonormalize<T>(n, B.Z(0, m), B.U(0, m), Qc, wk_, s_, nullptr, &rinv);
    Blk<T> Pfree = (U.p == B.Zb.template as<T>()) ? B.U(0, m) : B.Z(0, m);
    std::vector<double> ritz;
    if (lean_)
      rayleigh_ritz_chunked<T>(A, n, Blk<const T>{U.p, U.ld, m}, B.Tc(), wk_, ritz, s_, rinv);
    else
      rayleigh_ritz<T>(A, n, Blk<const T>{U.p, U.ld, m}, B.W(0, m), wk_, ritz, s_, rinv);
    stats.t_dense += now() - td;
    stats.arr_calls += 1;
    stats.arr_m2 += (double)m * m;
    // ---- merge with (Qc, Sigma_c): keep the w leading (stable, Qc first) ----
    std::vector<int> order(nc_ + m);
    std::iota(order.begin(), order.end(), 0);
    auto val = [&](int i) { return i < nc_ ? sig_c_[i] : ritz[i - nc_]; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return val(x) > val(y); });
    order.resize(w);
    int cnew = 0;
    for (int i : order)
      if (i >= nc_) cnew = std::max(cnew, i - nc_ + 1);
    // Ritz vectors X_new = U V[:, :cnew] into the free buffer, A X_new = W V into U's
    const double *V = wk_.small.template as<double>() + (size_t)m * m;
    Blk<T> Xn{Pfree.p, Pfree.ld, cnew};
    launch_update<T>(n, Blk<const T>{U.p, U.ld, m}, V, m, cnew, 1.0, 0.0, Xn, s_, false, /*fp32_cores=*/true);
    Blk<T> AXn{U.p, U.ld, cnew};
    if (lean_) {
      const Blk<const T> none{nullptr, 0, 0};
      launch_filter_spmm<T>(A, Blk<const T>{Xn.p, Xn.ld, cnew}, none, AXn, 1.0, 0.0, 0.0, nullptr, s_);
    } else {
      launch_update<T>(n, Blk<const T>{B.W(0, m).p, B.ldz, m}, V, m, cnew, 1.0, 0.0, AXn, s_, false,
                       /*fp32_cores=*/true);
    }
    ARR_HIP(hipMemcpyAsync(mu_.p, ritz.data(), sizeof(double) * cnew, hipMemcpyHostToDevice, s_));
    std::vector<double> rnew = residual_norms<T>(n, Blk<const T>{AXn.p, AXn.ld, cnew},
                                                 Blk<const T>{Xn.p, Xn.ld, cnew}, mu_.as<double>(), wk_, s_);
    std::vector<double> mu(w), res(w);
    std::vector<const T *> src(w);
    std::vector<int64_t> lds(w);
    std::vector<int32_t> cols(w);
    for (int q = 0; q < w; ++q) {
      const int i = order[q];
      if (i < nc_) {
        mu[q] = sig_c_[i];
        res[q] = res_c_[i];
        src[q] = B.Qb.template as<T>();
        lds[q] = B.ldq;
        cols[q] = i;
      } else {
        const int c = i - nc_;
        mu[q] = ritz[c];
        res[q] = rnew[c] / std::max(1.0, std::fabs(ritz[c]));
        src[q] = Xn.p;
        lds[q] = Xn.ld;
        cols[q] = c;
      }
    }
    double maxres = 0.0;
    for (int q = 0; q < k; ++q) maxres = std::max(maxres, res[q]);
    if (!(maxres == maxres)) maxres = std::numeric_limits<double>::infinity();
    stats.maxres = maxres;
    stats.t_arr += now() - t;
    if (fp32_stage) {
      stats.fp32_outer += 1;
      stats.fp32_maxres = maxres;  // the raw FP32-stage figure, before the FP64 closing iterations
      fp32_vals_.assign(mu.begin(), mu.begin() + k);
      fp32_mu_w_ = mu[w - 1];
      // A collapsed block: the w Ritz values within 1e-6 (b - a) of each other.
      // The filter can drive every column onto one isolated dominant
      // eigenvector below FP32 resolution (the FP32 stage cannot lock it
      // out), after which the FP32 pairs (w copies of one vector, with tiny
      // residuals) say nothing about the rest of the wanted set.
      fp32_collapsed_ = !(mu[0] - mu[w - 1] > 1e-6 * (b_ - a_)) || (o_.debug_fp32_collapse && j_ == 1);
      if (which_ == ARR_SMALLEST_ALGEBRAIC)
        for (double &v : fp32_vals_) v = -v;
    }
    if (o_.verbose) {
      std::fprintf(stderr,
                   "[arr] outer %d %s maxres %.3e tol_t %.1e d %d p %d locked %d width %d m %d jacobi_sweeps %d "
                   "t %.3f s (filter %.3f arr %.3f dense %.3f)\n",
                   j_, fp32_stage ? "fp32" : "fp64", maxres, tol_t_, d_, p_, nc_, wp_, m, wk_.last_sweeps, now(),
                   stats.t_filter, stats.t_arr, stats.t_dense);
      std::fflush(stderr);
    }
    // ---- stop rules (eq. out-stop; (i)-(iii) of Sec. 6) ----
    if (maxres < best_maxres_) {
      best_maxres_ = maxres;
      best_mu_k_ = mu[k - 1];
      best_mu_w_ = mu[w - 1];
      since_best_ = 0;
    } else {
      ++since_best_;
    }
    int status = -1;
    double accept = tol_;  // bound the explicit residuals must meet for ARR_OK
    if (!fp32_stage) {
      if (maxres <= tol_) status = ARR_OK;
      if (status < 0 && o_.paper_faithful) {
        int h = 0;
        for (int q = 0; q < k; ++q) h += res[q] < 0.1 * tol_;
        accept = (1.0 + 9.0 * h / k) * tol_;
        if (maxres < accept) status = ARR_OK;
      }
      if (status < 0 && since_best_ >= 3) status = ARR_STAGNATED;
      if (status < 0 && j_ == o_.maxit) status = ARR_NOT_CONVERGED;
    }
    if (status >= 0) {
      const double explicit_max = finish<T>(B, A, src, lds, cols, mu, U.p);
      // an accepted result must also pass the explicit FP64 check; if it does
      // not, iterate on (or report the result as not converged at maxit)
      if (status == ARR_OK && !(explicit_max <= accept)) status = j_ < o_.maxit ? -1 : ARR_NOT_CONVERGED;
    }
    if (status >= 0) {
      stats.final_p = p_;
      stats.final_d = d_;
      stats.n_locked = nc_;
      return status;
    }
    // ---- continuation (eq. contin) ----
    // Not in the FP32 stage: its residuals cannot reach the deflation
    // threshold tol_t^2, so moving b up to mu_w there, with nothing locked,
    // lets the filter amplify the leading directions until the block loses
    // rank in the next sweep. b and tol_t move in the FP64 stage only.
    if (!fp32_stage && maxres <= tol_t_) {
      tol_t_ = std::max(1e-2 * tol_t_, tol_);
      b_ = mu[w - 1];
      early_contin_done_ = true;
    } else if (!fp32_stage && !early_contin_done_ && maxres <= o_.early_contin) {
      // option early_contin: one earlier step of b only (tol_t unchanged)
      b_ = mu[w - 1];
      early_contin_done_ = true;
      stats.early_contin = j_;
    }
    // ---- deflation (eq. defl): Qc re-collected from the merged set ----
    // the FP32 stage locks nothing (its residuals do not reach tol_t^2, and it
    // keeps no Q blocks); the FP64 stage locks at eq. defl's threshold
    const double tol_d = fp32_stage ? -1.0 : std::max(1e-14, tol_t_ * tol_t_);
    std::vector<const T *> qs, xs;
    std::vector<int64_t> ql, xl;
    std::vector<int32_t> qcol, xcol;
    std::vector<double> nsig, nres;
    for (int q = 0; q < w; ++q) {
      if (res[q] <= tol_d) {
        qs.push_back(src[q]); ql.push_back(lds[q]); qcol.push_back(cols[q]);
        nsig.push_back(mu[q]); nres.push_back(res[q]);
      } else {
        xs.push_back(src[q]); xl.push_back(lds[q]); xcol.push_back(cols[q]);
      }
    }
    const int nc_new = (int)qs.size(), wp_new = (int)xs.size();
    // new X -> a scratch block, then into Z; new Qc -> Q2, then swap Q / Q2.
    // The scratch is W, or in the lean mode the block that held the basis and
    // A X_new (both dead now; the sources are X_new and Q): when that block is
    // Z itself the new X goes there directly.
    T *scratch = lean_ ? U.p : B.W(0, wp_new).p;
    gather<T>(n, wp_new, scratch, B.ldz, xs, xl, xcol);
    gather<T>(n, nc_new, B.Q2b.template as<T>(), B.ldq, qs, ql, qcol);
    if (scratch != B.Zb.template as<T>())
      launch_copy<T>(n, wp_new, B.Zb.template as<T>(), B.ldz, scratch, B.ldz, s_);
    std::swap(B.Qb, B.Q2b);
    nc_ = nc_new;
    wp_ = wp_new;
    sig_c_ = nsig;
    res_c_ = nres;
    // ---- augmentation blocks (eq. block) ----
    if (maxresp_ >= 0.0) {
      const double ratio = (mu[w - 1] - a_) / (mu[k - 1] - a_);
      if (ratio > 0.95 && maxres / maxresp_ > 0.1) p_ = std::min(p_ + 1, o_.p_max);
    }
    maxresp_ = maxres;
    // ---- degree (eq. hat-d, eq. degree) ----
    d_ = degree_update(best_mu_k_, best_mu_w_);
    if (wp_ == 0) {  // every pair locked
      std::vector<const T *> s2;
      std::vector<int64_t> l2;
      std::vector<int32_t> c2;
      for (int q = 0; q < nc_; ++q) { s2.push_back(B.Qb.template as<T>()); l2.push_back(B.ldq); c2.push_back(q); }
      const double explicit_max = finish<T>(B, A, s2, l2, c2, sig_c_, B.Ub.template as<T>());
      stats.final_p = p_;
      stats.final_d = d_;
      stats.n_locked = nc_;
      return (maxres <= tol_ && explicit_max <= tol_) ? ARR_OK : ARR_NOT_CONVERGED;
    }
    if (fp32_stage) {
      ++fp32_iters;
      if (maxres < fp32_best * 0.5) {
        fp32_best = maxres;
        fp32_since_best = 0;
      } else {
        ++fp32_since_best;
      }
      if (fp32_collapsed_ || maxres <= o_.mixed_switch || fp32_since_best >= 2 || fp32_iters >= fp32_limit)
        return -100;
    }
  }
  return ARR_NOT_CONVERGED;
}

int Solver::solve() {
  t0_ = std::chrono::steady_clock::now();
  stats = arr_stats_t{};
  solved = false;
  fp32_vals_.clear();
  fp32_collapsed_ = false;
  // the mixed path's handover takes its own step; FP64 takes at most one
  early_contin_done_ = o_.precision == ARR_MIXED;
  ARR_HIP(hipSetDevice(o_.device));
  ensure_device();
  host_results_ = false;
  SpmmTimer timer, gtimer;
  struct Install {
    SpmmTimer *prev, *gprev;
    Install(SpmmTimer *t, SpmmTimer *g) : prev(spmm_timer()), gprev(gemm_timer()) {
      spmm_timer() = t;
      gemm_timer() = g;
    }
    ~Install() {
      spmm_timer() = prev;
      gemm_timer() = gprev;
    }
  } install(o_.timing ? &timer : nullptr, o_.timing ? &gtimer : nullptr);
  if (have_x0_)
    launch_copy<double>(n_, w_, B64_.Zb.as<double>(), B64_.ldz, x0_.as<double>(), w_, s_);
  else
    launch_gaussian(n_, w_, B64_.Zb.as<double>(), B64_.ldz, o_.seed, s_);
  ARR_HIP(hipStreamSynchronize(s_));
  // state of Algorithm 8
  d_ = o_.d0;
  p_ = o_.p0;
  j_ = 0;
  poly_count_ = 0;
  nc_ = 0;
  wp_ = w_;
  sig_c_.clear();
  res_c_.clear();
  best_maxres_ = std::numeric_limits<double>::infinity();
  maxresp_ = -1.0;
  since_best_ = 0;
  tol_t_ = o_.tol1 > 0 ? std::max(o_.tol1, tol_) : (tol_ <= 1e-8 ? 1e-6 : tol_);
  setup_interval();
  ARR_HIP(hipStreamSynchronize(s_));
  stats.t_setup = now();
  if (o_.verbose) {
    std::fprintf(stderr, "[arr] setup n %lld k %d w %d a %.6e b %.6e |A| %.6e t %.3f s\n", (long long)n_, k_, w_, a_,
                 b_, norm_, stats.t_setup);
    std::fflush(stderr);
  }
  int status;
  if (o_.precision == ARR_MIXED) {
    launch_convert<float, double>(n_, w_, B32_.Zb.as<float>(), B32_.ldz, B64_.Zb.as<double>(), B64_.ldz, s_);
    const double b0 = b_, tol_t0 = tol_t_;
    status = outer<float>(B32_, A32_, true);
    if (status == -100 && fp32_collapsed_) {
      // the FP32 stage's block collapsed: Algorithm 8 starts again in FP64
      // from the starting block, which the FP64 Z block still holds
      if (o_.verbose)
        std::fprintf(stderr, "[arr] FP32 stage collapsed (Ritz values within 1e-6 (b - a)): FP64 restarts from the "
                             "starting block\n");
      stats.fp32_collapsed = 1;
      d_ = o_.d0;
      p_ = o_.p0;
      wp_ = w_;
      b_ = b0;
      tol_t_ = tol_t0;
      maxresp_ = -1.0;
      best_maxres_ = std::numeric_limits<double>::infinity();
      since_best_ = 0;
      status = outer<double>(B64_, A64_, false);
    } else if (status == -100) {
      // hand the iterate to the FP64 stage
      ARR_REQUIRE(nc_ == 0, "FP32 stage ended with locked pairs");
      launch_convert<double, float>(n_, wp_, B64_.Zb.as<double>(), B64_.ldz, B32_.Zb.as<float>(), B32_.ldz, s_);
      // the FP64 stage re-derives its stagnation reference
      best_maxres_ = std::numeric_limits<double>::infinity();
      since_best_ = 0;
      // continuation step at the handover: b moves up to the FP32 stage's
      // mu_{k+q}, as eq. contin moves it (tol_t unchanged). The FP32 stage
      // takes no continuation step itself (see outer()).
      if (stats.fp32_maxres <= o_.mixed_contin) {
        if (o_.verbose)
          std::fprintf(stderr, "[arr] handover to FP64 at maxres %.3e: b %.6e -> %.6e\n", stats.fp32_maxres, b_,
                       fp32_mu_w_);
        b_ = fp32_mu_w_;
        stats.handover_contin = 1;
      }
      status = outer<double>(B64_, A64_, false);
    }
  } else {
    status = outer<double>(B64_, A64_, false);
  }
  ARR_HIP(hipStreamSynchronize(s_));
  stats.t_total = now();
  if (o_.timing) {
    timer.flush();
    int best = 0;
    for (int c = 1; c < SpmmTimer::kClasses; ++c)
      if (timer.ms[c] > timer.ms[best]) best = c;
    stats.spmm_launches = timer.launches[best];
    stats.spmm_ms = timer.ms[best];
    stats.spmm_bytes = timer.bytes[best];
    // class = slots + 5 (16-byte loads) + 10 fp64 + 20 flags
    stats.spmm_cols_per_lane = 1 << (best % 5);
    stats.spmm_vec = (best % 10) >= 5 ? ((best % 20) >= 10 ? 2 : 4) : 1;
    stats.spmm_fp64 = (best % 20) >= 10 ? 1 : 0;
    stats.spmm_flags = best / 20;
    int best32 = 0;
    for (int c = 1; c < SpmmTimer::kClasses; ++c)
      if ((c % 20) < 10 && timer.ms[c] > timer.ms[best32]) best32 = c;
    stats.spmm32_launches = timer.launches[best32];
    stats.spmm32_ms = timer.ms[best32];
    stats.spmm32_bytes = timer.bytes[best32];
    stats.spmm32_cols_per_lane = 1 << (best32 % 5);
    stats.spmm32_vec = (best32 % 10) >= 5 ? 4 : 1;
    stats.spmm32_flags = best32 / 20;
    gtimer.flush();
    auto sum = [&](std::initializer_list<int> cls, int64_t &l, double &ms, double &fl) {
      l = 0, ms = 0, fl = 0;
      for (int c : cls) l += gtimer.launches[c], ms += gtimer.ms[c], fl += gtimer.bytes[c];
    };
    sum({kGramF64, kGramF32}, stats.gram64_launches, stats.gram64_ms, stats.gram64_flops);
    sum({kGramF32Cores}, stats.gram32_launches, stats.gram32_ms, stats.gram32_flops);
    sum({kUpdF64, kUpdF32}, stats.upd64_launches, stats.upd64_ms, stats.upd64_flops);
    sum({kUpdF32Cores}, stats.upd32_launches, stats.upd32_ms, stats.upd32_flops);
  }
  stats.status = status;
  stats.a = which_ == ARR_SMALLEST_ALGEBRAIC ? -a_ : a_;
  stats.b = which_ == ARR_SMALLEST_ALGEBRAIC ? -b_ : b_;
  stats.norm_est = norm_;
  solved = true;
  return status;
}

void Solver::get_residuals(double *resid, double *resid_norm_a, double *rnorm) {
  ARR_REQUIRE(solved, "arr_get_residuals called before a successful arr_solve");
  for (int i = 0; i < k_; ++i) {
    if (resid) resid[i] = out_res_[i];
    if (resid_norm_a) resid_norm_a[i] = out_rn_[i] / norm_;
    if (rnorm) rnorm[i] = out_rn_[i];
  }
}

void Solver::get(double *evals, double *evecs, int64_t ldv, double *resid) {
  ARR_REQUIRE(solved, "arr_get_eigpairs called before a successful arr_solve");
  const int k = k_;
  if (evals) std::copy(out_vals_.begin(), out_vals_.end(), evals);
  if (resid) std::copy(out_res_.begin(), out_res_.end(), resid);
  if (evecs) {
    ARR_REQUIRE(ldv >= k, "ldv must be >= k");
    if (host_results_) {
      ARR_REQUIRE(!h_vecs_.empty(), "eigenvectors were not kept for this served request (keep_vectors = 0)");
      for (int64_t i = 0; i < n_; ++i) std::copy(&h_vecs_[i * k], &h_vecs_[i * k] + k, evecs + i * ldv);
    } else {
      ARR_HIP(hipMemcpy2D(evecs, sizeof(double) * ldv, outv_p_, sizeof(double) * outv_ld_, sizeof(double) * k, n_,
                          hipMemcpyDeviceToHost));
    }
    // sign convention: the entry of largest magnitude is positive
    for (int c = 0; c < k; ++c) {
      double best = -1.0, sgn = 1.0;
      for (int64_t i = 0; i < n_; ++i) {
        const double v = evecs[i * ldv + c];
        if (std::fabs(v) > best) {
          best = std::fabs(v);
          sgn = v < 0 ? -1.0 : 1.0;
        }
      }
      if (sgn < 0)
        for (int64_t i = 0; i < n_; ++i) evecs[i * ldv + c] = -evecs[i * ldv + c];
    }
  }
}

template int Solver::outer<double>(Blocks<double> &, const DevCSR<double> &, bool);
template int Solver::outer<float>(Blocks<float> &, const DevCSR<float> &, bool);

}  // namespace arr
