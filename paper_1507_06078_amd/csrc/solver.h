// ARRABIT-MPM solver state (Algorithm 8) behind the C handle.
#pragma once

#include <chrono>
#include <map>
#include <string>
#include <vector>

#include "../../include/arr.h"
#include "steps.h"

namespace arr {

// Device blocks of one precision. Z, U, W are n x ldz: Z holds the iterate X
// in its first w' columns and the Krylov blocks [X, AX, ..., A^p X] of the
// augmentation (eq. S:ARR); U and W hold the orthonormal basis and A U of the
// Rayleigh-Ritz step. Q and Q2 (n x w) hold the locked pairs Qc.
template <typename T>
struct Blocks {
  DevBuf Zb, Ub, Wb, Qb, Q2b, Tb;  // Wb: not allocated in the lean-memory mode; Tb: its chunk buffer (n x ldt)
  int64_t ldt = 0;
  int64_t ldz = 0, ldq = 0;
  bool ready = false;
  void alloc(int64_t n, int64_t ldz_, int64_t ldq_) {
    ldz = ldz_;
    ldq = ldq_;
    Zb.alloc(sizeof(T) * n * ldz);
    Ub.alloc(sizeof(T) * n * ldz);
    Wb.alloc(sizeof(T) * n * ldz);
    Qb.alloc(sizeof(T) * n * ldq);
    Q2b.alloc(sizeof(T) * n * ldq);
    ready = true;
  }
  void release() {
    Zb.release(); Ub.release(); Wb.release(); Qb.release(); Q2b.release(); Tb.release();
    ready = false;
  }
  Blk<T> Z(int c0, int w) const { return Blk<T>{Zb.as<T>() + c0, ldz, w}; }
  Blk<T> U(int c0, int w) const { return Blk<T>{Ub.as<T>() + c0, ldz, w}; }
  Blk<T> W(int c0, int w) const { return Blk<T>{Wb.as<T>() + c0, ldz, w}; }
  Blk<T> Q(int w) const { return Blk<T>{Qb.as<T>(), ldq, w}; }
  Blk<T> Q2(int w) const { return Blk<T>{Q2b.as<T>(), ldq, w}; }
  Blk<T> Tc() const { return Blk<T>{Tb.as<T>(), ldt, (int)ldt}; }
};

class Solver {
 public:
  // Validates the problem and keeps a host copy of the matrix; device memory
  // is allocated by ensure_device() (called by solve() when needed).
  Solver(const arr_csr_t *csr, int64_t n, int k, int which, double tol, const arr_options_t &o);
  ~Solver();
  void set_initial_block(const double *X0, int64_t ld);
  int solve();
  void get(double *evals, double *evecs, int64_t ldv, double *resid);
  void get_residuals(double *resid, double *resid_norm_a, double *rnorm);
  // the k wanted Ritz values of the last FP32-stage iteration (empty if none)
  const std::vector<double> &fp32_stage_values() const { return fp32_vals_; }
  // Device bytes ensure_device() allocates (every buffer of a solve).
  size_t footprint() const { return const_cast<Solver *>(this)->device_plan(false); }
  void ensure_device();
  void release_device();
  // Copy the results to host memory (eigenvectors only if keep_vectors) so that
  // release_device() can return the device memory.
  void stash_results(bool keep_vectors);
  arr_stats_t stats{};
  std::string err;
  bool solved = false;
  int device() const { return o_.device; }
  // Set while a server holds this solver (from submission until the server is
  // destroyed); arr_destroy waits for the request before deleting the solver.
  class Server *server = nullptr;
  uint64_t ticket = 0;
  bool keep_vectors() const { return o_.keep_vectors != 0; }

 private:
  int64_t n_;
  int k_, which_, w_;
  double tol_;
  arr_options_t o_;
  hipStream_t s_ = nullptr;
  DevBuf coef64_, coef32_, fcol_, orp_, ocol_, oval64_, oval32_;  // matrix in the row form of the SpMM
  DevCSR<double> A64_;
  DevCSR<float> A32_;
  Blocks<double> B64_;
  Blocks<float> B32_;
  Work wk_;
  DevBuf desc_, mu_, outv_, x0_;
  // the returned eigenvectors (n x k, leading dimension outv_ld_): outv_, or
  // in the lean-memory mode a free block of the solve
  double *outv_p_ = nullptr;
  int64_t outv_ld_ = 0;
  bool lean_ = false;
  DevBuf lz_V_, lz_w_, lz_h_, lz_part_;  // Lanczos basis and scratch
  bool have_x0_ = false, device_ready_ = false, host_results_ = false;
  int64_t ldz_ = 0, ldq_ = 0;
  int lanczos_L_ = 0;
  RowSplit h_split_;  // the working operator in the row form of the SpMM
  std::vector<double> h_x0_, h_vecs_;
  int64_t nnz_ = 0;  // entries of the whole matrix
  size_t device_plan(bool allocate);
  std::map<int, FilterPoly> coef_;

  // iteration state (Algorithm 8)
  int nc_ = 0, wp_ = 0, d_ = 3, p_ = 1, j_ = 0;
  double a_ = 0, b_ = 0, norm_ = 0, tol_t_ = 0;
  std::vector<double> sig_c_, res_c_;
  double best_maxres_ = 0, maxresp_ = -1, best_mu_k_ = 0, best_mu_w_ = 0;
  int since_best_ = 0;
  std::vector<double> out_vals_, out_res_, out_rn_, fp32_vals_;
  double fp32_mu_w_ = 0;  // mu_{k+q} of the last FP32-stage iteration
  bool fp32_collapsed_ = false;  // its Ritz values collapsed (see outer())
  bool early_contin_done_ = false;  // option early_contin's step taken (or not wanted)
  int poly_count_ = 0;  // filter applications so far (for the debug_nan_poly hook)

  const FilterPoly &coeffs(int d);
  void setup_interval();
  template <typename T>
  int outer(Blocks<T> &B, const DevCSR<T> &A, bool fp32_stage);
  // free: a block of the solve not holding any source (n x ldz, T); in the
  // lean-memory mode it receives the output vectors
  template <typename T>
  double finish(Blocks<T> &B, const DevCSR<T> &A, const std::vector<const T *> &src, const std::vector<int64_t> &lds,
                const std::vector<int32_t> &cols, const std::vector<double> &mu, T *free);
  template <typename T>
  void poly_hook(Blk<T> X);
  template <typename T>
  void gather(int64_t n, int w, T *dst, int64_t lddst, const std::vector<const T *> &src,
              const std::vector<int64_t> &lds, const std::vector<int32_t> &cols);
  int degree_update(double mu_k, double mu_w) ;
  double now() const;
  std::chrono::steady_clock::time_point t0_;
};

}  // namespace arr
