// Internal declarations of the gfx950 ARRABIT library: device buffers, kernel
// launchers and the small helpers they share. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

namespace arr {

// Error raised by a failed HIP call or a violated precondition; the C ABI
// turns it into a return code and a message.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define ARR_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::arr::Error(-3, std::string(#call) + " failed: " + hipGetErrorString(e_) +     \
                                 " at " __FILE__ ":" + std::to_string(__LINE__));           \
  } while (0)

#define ARR_REQUIRE(cond, msg)                                  \
  do {                                                          \
    if (!(cond)) throw ::arr::Error(-1, std::string(msg));      \
  } while (0)

// Device matrix in the row form the SpMM kernels read. Per row i: coef[8i ..
// 8i+7] = {A[i][i-1], A[i][i], A[i][i+1], f0, f1, f2, f3, a_p} (zero where an
// entry is absent) and fcol[4i .. 4i+3] the columns of the first four other
// ("far") entries f0..f3 (unused slots: column i, value 0). Far entries past
// the fourth are an overflow CSR (orp int64 [n+1], ocol int32, oval in T);
// orp is null when no row has more than four. nnz counts every entry of the
// matrix.
//
// Paired form (pair = P > 0): rows are grouped in blocks of 2P; row i is an
// "upper" row when i mod 2P < P, with partner i + P, else a "lower" row with
// partner i - P. a_p = A[i][partner(i)] (0 if absent or out of range) and the
// partner entry is not among the far entries. A wave then processes a run of
// upper rows together with the lower run P rows below it, so each row's
// partner term comes from the other run's register window instead of a
// gather. Only matrices whose rows then fit the far slots without overflow
// use it; kf (1 or 3) is the number of far slots the kernel gathers (slots
// past kf are unused in every row). In the plain form pair = 0, a_p = 0 and
// kf = 4.
template <typename T>
struct DevCSR {
  int64_t n = 0, nnz = 0;
  const T *coef = nullptr;
  const int32_t *fcol = nullptr;
  const int64_t *orp = nullptr;
  const int32_t *ocol = nullptr;
  const T *oval = nullptr;
  int64_t pair = 0;
  int kf = 4;
  // grid form (gx > 0): see split_rows; fcol and the overflow CSR are unused
  int64_t gx = 0, gy = 0, gz = 0;
};

// Host form of the same split (FP64 values); orp is left empty when no row
// has more than four far entries.
struct RowSplit {
  std::vector<double> coef;
  std::vector<int32_t> fcol;
  std::vector<int64_t> orp;
  std::vector<int32_t> ocol;
  std::vector<double> oval;
  int64_t pair = 0;
  int kf = 4;
  int64_t gx = 0, gy = 0, gz = 0;
};

// Rows per run of the paired form (a wave does two runs at once).
constexpr int64_t kPairRun = 20;

// Host split of a CSR with strictly increasing columns per row. form 3 (grid)
// chooses the grid form when every entry is a neighbour of its row in a
// 7-point stencil on a gx x gy x gz grid, or a 5-point stencil on a gx x gz
// grid (gy = 1), lexicographic with x fastest; form 0 (automatic) does so for
// the 2D case only. In the grid form the record of row i is
// then {A[i][i - gx gy], A[i][i - gx], A[i][i - 1], A[i][i], A[i][i + 1],
// A[i][i + gx], A[i][i + gx gy], 0} (zero for a neighbour outside the grid;
// for gy = 1 the +-gx entries take the first and seventh slots) and fcol is
// empty. Otherwise, and with form 2 (paired), the paired form when the matrix
// has a frequent far offset P >= kPairRun (entries A[i][i+P] in at least half
// of the rows), the runs of kPairRun rows cover a half block of P rows with
// at most P/8 rows computed twice, and every row then has at most three far
// entries besides its partner; otherwise, and with form 1, the plain form.
void split_rows(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, RowSplit &out,
                int form = 0);

// A row-major view of columns [0, w) of a device block with leading
// dimension ld.
template <typename T>
struct Blk {
  T *p = nullptr;
  int64_t ld = 0;
  int w = 0;
  Blk cols(int c0, int wc) const { return Blk{p + c0, ld, wc}; }
};

// Bump allocator over one pre-reserved device block. While a pool is
// installed for the calling thread (see device_pool()), every DevBuf
// allocation of that thread is carved from it and never returned
// individually: the whole block goes back at once when its owner is done.
struct Pool {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  void *take(size_t b) {
    b = (b + 255) / 256 * 256;
    if (used + b > cap)
      throw Error(-2, "device pool exhausted: need " + std::to_string(used + b) + " of " + std::to_string(cap) +
                          " reserved bytes");
    void *p = base + used;
    used += b;
    return p;
  }
};
Pool *&device_pool();

// Owned device allocation (hipMalloc, or a slice of the thread's pool).
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  bool pooled = false;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), pooled(o.pooled) { o.p = nullptr; o.bytes = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; pooled = o.pooled;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    if (Pool *pool = device_pool()) {
      p = pool->take(b);
      bytes = b;
      pooled = true;
      return;
    }
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(-2, "hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = b;
    pooled = false;
  }
  void ensure(size_t b) {
    if (b <= bytes) return;
    // a pooled buffer is sized once from the request's footprint; growing it
    // would take memory the request did not reserve
    if (pooled) throw Error(-2, "pooled device buffer of " + std::to_string(bytes) + " bytes asked to grow to " +
                                    std::to_string(b) + " (footprint under-estimate)");
    alloc(b);
  }
  void release() {
    if (p && !pooled) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    pooled = false;
  }
  template <typename T> T *as() const { return static_cast<T *>(p); }
  // A view of `b` bytes of memory owned elsewhere (never freed here).
  void view(void *q, size_t b) {
    release();
    p = q;
    bytes = b;
    pooled = true;
  }
};

// ---- launchers (spmm.hip) ----------------------------------------------------

// Yout = alpha*A*Yin + beta*Yin + gamma*Z on the w columns of the views; if
// partial != nullptr, per-workgroup column sums of squares of Yout are written
// to partial[g*w + c] for g < returned group count. With colss (device, w
// values; needs partial) column c of Yout is also divided by sqrt(colss[c])
// before it is stored and summed. Returns the number of workgroups (rows of
// `partial`).
template <typename T>
int launch_filter_spmm(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, double alpha,
                       double beta, double gamma, double *partial, hipStream_t s, const double *colss = nullptr);
// Optional HIP-event timing of kernel launches, per launch class, with the
// algorithmic work of each launch (bytes for the SpMM, flops for the GEMMs).
// Installed per thread by the solver. SpMM classes: columns per lane (0..4
// for 1..16) + 5 for 16-byte loads + 10 for FP64 data + 20 * flags (1 Z term,
// 2 overflow rows, 4 column sums, 8 paired form, 16 paired with one far slot).
// GEMM classes: see GemmClass. Flag 32 marks the grid form, 64 its 2D tile.
struct SpmmTimer {
  struct Pending { hipEvent_t a, b; int cls; double bytes; };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  static constexpr int kClasses = 2048;
  int64_t launches[kClasses] = {};
  double ms[kClasses] = {}, bytes[kClasses] = {};
  hipEvent_t get();
  void flush();  // waits for the recorded events and accumulates
  void reset();
  ~SpmmTimer();
  // brackets one launch on stream s (no-op on a null timer)
  struct Scope {
    SpmmTimer *t;
    Pending p{};
    hipStream_t s;
    Scope(SpmmTimer *t_, int cls, double work, hipStream_t s_);
    ~Scope();
  };
};
SpmmTimer *&spmm_timer();
// Timer of the Gram (X^T Y) and block-update (X W) launches.
SpmmTimer *&gemm_timer();
enum GemmClass { kGramF64 = 0, kGramF32 = 1, kGramF32Cores = 2, kUpdF64 = 3, kUpdF32 = 4, kUpdF32Cores = 5 };
// Groups that launch_filter_spmm / launch_colsumsq use for n rows (sizes the
// partial buffer: groups * w doubles).
int spmm_groups(int64_t n);

// ---- multi-request filter SpMM ----------------------------------------------
// One launch of the plain- or paired-form SpMM kernel, as its arguments
// (pointers already offset to the launch's column chunk), for the
// multi-request kernel: groups is the grid the launch would have had.
struct SpmmTask {
  int64_t n, P, ldy, ldz, ldo;
  const void *coef;
  const int32_t *fcol;
  const int64_t *orp;
  const int32_t *ocol;
  const void *oval;
  const void *Yin;
  const void *Z;
  void *Yout;
  double alpha, beta, gamma;
  double *partial;
  const double *colss;
  int32_t w, wtot, c0, groups;
};
// Runs ntasks workgroup tasks {launch index into desc, workgroup of that
// launch} of one kernel variant on s.
using SpmmTaskLauncher = void (*)(const SpmmTask *desc, const int2 *tasks, int ntasks, hipStream_t s);

// While a batch is installed on the calling thread (spmm_batch()),
// launch_filter_spmm hands its plain- and paired-form launches to the batch
// instead of launching them (grid-form launches still go to their stream,
// and no SpMM timing is taken). run() then executes every collected launch:
// one persistent launch per kernel variant, whose workgroups take the
// collected launches' workgroups from a task table, interleaved over the
// launches. Each workgroup of a collected launch runs the same code on the
// same rows as in its own launch, so results are bitwise those of separate
// launches. The tables go through one device buffer of cap bytes (so
// successive run() calls must use one stream) and a ring of kRing pinned
// staging buffers: run() waits on the host only for the copy kRing runs
// back.
struct SpmmBatch {
  explicit SpmmBatch(size_t cap_bytes = (size_t)4 << 20);
  ~SpmmBatch();
  SpmmBatch(const SpmmBatch &) = delete;
  SpmmBatch &operator=(const SpmmBatch &) = delete;
  void add(const SpmmTask &t, SpmmTaskLauncher launcher);
  // Launches the collected work on s and forgets it; returns the number of
  // launches it replaced.
  int run(hipStream_t s);
  bool empty() const { return tasks_.empty(); }

 private:
  static constexpr int kRing = 8;
  std::vector<SpmmTask> tasks_;
  std::vector<SpmmTaskLauncher> launchers_;
  DevBuf dev_;
  char *host_ = nullptr;  // kRing staging buffers of cap_ bytes
  size_t cap_ = 0;
  hipEvent_t staged_[kRing] = {};
  int slot_ = 0;
};
SpmmBatch *&spmm_batch();

// A receiver of the calling thread's SpMMs (the serving loop installs one on
// each request's thread): launch_filter_spmm hands it the whole call as
// `launch` (its arguments copied; it performs the call's launches on the
// stream it is given) and returns what the call would return. The sink must
// leave the caller's stream s ordered after those launches: at once, or,
// inside a chain (begin_chain .. end_chain, calls on s with nothing else
// enqueued on s in between), by end_chain.
struct SpmmSink {
  virtual ~SpmmSink() = default;
  virtual void run(std::function<void(hipStream_t)> launch, hipStream_t s) = 0;
  virtual void begin_chain() {}
  virtual void end_chain(hipStream_t) {}
  virtual void drop_chain() {}
};
SpmmSink *&spmm_sink();

// Marks a run of filter SpMMs on s with nothing else enqueued on s in between
// (one filter application) for the calling thread's sink, which may hand them
// on together; close() ends the run. A chain left without close() (an
// exception) is dropped.
class SpmmChain {
 public:
  explicit SpmmChain(hipStream_t s) : s_(s), k_(spmm_sink()) {
    if (k_) k_->begin_chain();
  }
  SpmmChain(const SpmmChain &) = delete;
  SpmmChain &operator=(const SpmmChain &) = delete;
  void close() {
    SpmmSink *k = k_;
    k_ = nullptr;
    if (k) k->end_chain(s_);
  }
  ~SpmmChain() {
    if (k_) k_->drop_chain();
  }

 private:
  hipStream_t s_;
  SpmmSink *k_;
};
// y = A x for one vector (Lanczos).
template <typename T>
void launch_spmv(const DevCSR<T> &A, const T *x, T *y, hipStream_t s);

// ---- launchers (gemm.hip) ----------------------------------------------------

// G (FP64, mx x my, row-major, ld = my) = X^T Y with X n x mx and Y n x my.
// `work` must hold gram_work_doubles(n, mx, my) doubles. If sym, X^T Y is
// known to be symmetric (mx == my): only its upper triangle is computed, then
// mirrored. fp32_cores (FP32 data only): FP32 matrix cores on 32-row slices,
// for well-conditioned products; otherwise products and sums are FP64.
// work_cap > 0: work holds only work_cap doubles; the split count is capped to
// fit, and a product whose single split does not fit is rejected (ARR_EINVAL).
template <typename T>
void launch_gram(int64_t n, Blk<const T> X, Blk<const T> Y, double *G, double *work, bool sym,
                 hipStream_t s, bool fp32_cores = false, int64_t work_cap = 0);
size_t gram_work_doubles(int64_t n, int mx, int my);
// Upper bound of gram_work_doubles over all mx, my <= m_max.
size_t gram_work_bound(int64_t n, int m_max);
// Y = beta*Y + alpha * X * W with W FP64 (m x c, ldw) on the device; w_upper:
// W is upper triangular (its zero blocks are skipped). Y must not alias X.
// fp32_cores (FP32 data only): W rounded to FP32 and FP32 matrix cores, for a
// well-conditioned W such as an orthogonal rotation. colss (device, c values,
// may be null): column j of the result is divided by sqrt(colss[j]).
template <typename T>
void launch_update(int64_t n, Blk<const T> X, const double *W, int64_t ldw, int c, double alpha,
                   double beta, Blk<T> Y, hipStream_t s, bool w_upper = false, bool fp32_cores = false,
                   const double *colss = nullptr);

// ---- launchers (misc.hip) ----------------------------------------------------

// Per-group column sums of squares of (P - Q diag(mu)) (Q, mu may be null),
// written to partial[g*w + c]. Returns the group count.
template <typename T>
int launch_colsumsq(int64_t n, Blk<const T> P, Blk<const T> Q, const double *mu, double *partial,
                    hipStream_t s);
// out[c] = sum_g partial[g*w + c] (fixed order), optionally sqrt.
void launch_reduce_groups(const double *partial, int groups, int w, double *out, bool take_sqrt,
                          hipStream_t s);
// X[:, c] *= scale[c] (scale FP64 on device); if inv_sqrt, X[:, c] /= sqrt(scale[c]).
template <typename T>
void launch_scale_columns(int64_t n, Blk<T> X, const double *scale, bool inv_sqrt, hipStream_t s);
// dst[:, j] = src_j[:, col_j] for j < w; srcs/cols/lds are device arrays of length w.
template <typename T>
void launch_gather_columns(int64_t n, int w, T *dst, int64_t lddst, const T *const *srcs,
                           const int64_t *lds, const int32_t *cols, hipStream_t s);
template <typename TD, typename TS>
void launch_convert(int64_t n, int w, TD *dst, int64_t lddst, const TS *src, int64_t ldsrc,
                    hipStream_t s);
// Gaussian N(0,1) block from a counter-based generator (Philox4x32-10 +
// Box-Muller), entry (i, j) depends only on (seed, i, j).
void launch_gaussian(int64_t n, int w, double *X, int64_t ld, uint64_t seed, hipStream_t s);
template <typename T>
void launch_fill(T *p, int64_t count, T v, hipStream_t s);
// copy a block (same dtype)
template <typename T>
void launch_copy(int64_t n, int w, T *dst, int64_t lddst, const T *src, int64_t ldsrc, hipStream_t s);

// ---- launchers (dense.hip): small FP64 matrices, row-major, on the device ----

// In-place lower Cholesky of the m x m SPD matrix A (upper part left
// untouched). info (device int) = 0 on success, j+1 if the pivot of column j
// was not positive. `shift` is added to the diagonal first.
void launch_cholesky(int m, double *A, int64_t lda, double shift, int *info, hipStream_t s);
// Winv = L^{-T} (upper triangular, full m x m written, zeros below) for the
// lower-triangular L (in A's lower part). scratch >= 2 m^2 doubles.
void launch_tri_inv_t(int m, const double *L, int64_t ldl, double *Winv, int64_t ldw, double *scratch,
                      hipStream_t s);
// rcond(G) = 1/(|G|_1 |G^-1|_1) for the m x m matrix G (device, ld m), or 0
// if G is not numerically positive definite. work >= 5 m^2 doubles; info is a
// device int; the result goes to *rc (device).
void rcond_device(int m, const double *G, double *work, int *info, double *rc, hipStream_t s);
// C = beta C + alpha A B for small device matrices with arbitrary strides:
// A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj]; lower: skip 64 x 64
// tiles strictly above the diagonal.
void small_gemm(int m1, int m2, int kk, double alpha, const double *A, int64_t sai, int64_t sak, const double *B,
                int64_t sbk, int64_t sbj, double beta, double *C, int64_t ldc, bool lower, hipStream_t s);
// C <- (C - I) / 2 (m x m, ld m)
void launch_half_minus_identity(int m, double *C, hipStream_t s);
// max |diag| and Frobenius norm of a small matrix -> out[0], out[1]
void launch_diag_max(int m, const double *A, int64_t lda, double *out, hipStream_t s);
// Symmetrize: A = (A + A^T)/2

// Parallel cyclic Jacobi eigensolver; see dense.hip.
struct Jacobi {
  DevBuf bufA, bufB, bufV, bufOff, bufEval;
  std::vector<double> h_eval;
  int mcap = 0;
  // Device bytes of the buffers for matrices of order <= m, and allocation.
  static size_t reserve_bytes(int m);
  void reserve(int m);
  // H (m x m, row-major, ld = m) is read; on return the eigenvalues in
  // descending order are in evals_host (size m) and the matching unit
  // eigenvectors are the COLUMNS of V (m x m row-major, ld = m):
  // H = V diag(evals) V^T.
  void solve(int m, const double *H, double *V, std::vector<double> &evals_host, hipStream_t s,
             int *sweeps_out = nullptr);
};

// ---- host helpers ------------------------------------------------------------

// Chebyshev-interpolant coefficients Gamma_d (leading first), Sec. 5.
std::vector<double> filter_coefficients(int d);
// psi_d in both forms: monomial coefficients (leading first) for Algorithm 7's
// Horner recurrence, and lead * prod (t - roots[i]) with the real roots in
// Leja order for the product form.
struct FilterPoly {
  std::vector<double> gamma, roots;
  double lead = 0.0;
};
FilterPoly filter_poly(int d);
// Form of the filter application: the product of d linear factors (2 block
// passes per degree) or Algorithm 7's Horner recurrence (3 block passes); or
// the classic Chebyshev polynomial T_d (eq. cheby-poly) in place of psi_d.
enum PolyForm { kPolyProduct = 0, kPolyHorner = 1, kPolyChebyshev = 2 };
// The same interpolant in the Chebyshev basis: psi_d = sum_k c[k] T_k.
std::vector<double> filter_chebyshev_coefficients(int d);

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace arr
