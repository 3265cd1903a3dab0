// extern "C" entry points declared in include/arr.h. Each one converts
// exceptions into return codes and keeps the message for arr_last_error /
// arr_last_global_error.
#include <cstring>
#include <memory>
#include <mutex>

#include "server.h"

// Split-K partial tiles of arr_gram_noalloc: a fixed device array, so that the
// call allocates nothing. Host code never passes this name to a kernel (on the
// host it is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device (scratch_on_device).
constexpr int64_t kNoallocScratchDoubles = int64_t(1) << 22;  // 32 MiB on each device
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

struct arr_solver {
  std::unique_ptr<arr::Solver> s;
  std::string err;
};

struct arr_server {
  std::unique_ptr<arr::Server> s;
};

namespace {

thread_local std::string g_err;

template <typename F>
int guarded(std::string *err, F &&f) {
  try {
    return f();
  } catch (const arr::Error &e) {
    g_err = e.what();
    if (err) *err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    if (err) *err = g_err;
    return ARR_ENOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    if (err) *err = e.what();
    return ARR_EDEVICE;
  }
}

// The caller's device CSR in the row form of the SpMM kernels: downloaded,
// checked (row pointers, column range and order), split on the host and
// uploaded into buffers this object owns.
template <typename T>
struct SplitDev {
  arr::DevBuf coef, fcol, orp, ocol, oval;
  arr::DevCSR<T> M;
};

template <typename T>
std::unique_ptr<SplitDev<T>> dev_split(const arr_dev_csr_t *A) {
  ARR_REQUIRE(A && A->rowptr && A->n > 0 && A->nnz >= 0, "device CSR is NULL or empty");
  ARR_REQUIRE(A->nnz == 0 || (A->colind && A->val), "device CSR arrays are NULL");
  ARR_REQUIRE(A->row_form >= ARR_ROW_AUTO && A->row_form <= ARR_ROW_GRID,
              "unknown row form");
  const int64_t n = A->n, nnz = A->nnz;
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> ci(nnz);
  std::vector<T> vt(nnz);
  ARR_HIP(hipMemcpy(rp.data(), A->rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz) {
    ARR_HIP(hipMemcpy(ci.data(), A->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    ARR_HIP(hipMemcpy(vt.data(), A->val, sizeof(T) * nnz, hipMemcpyDeviceToHost));
  }
  ARR_REQUIRE(rp[0] == 0 && rp[n] == nnz, "rowptr[0] must be 0 and rowptr[n] must equal nnz");
  for (int64_t i = 0; i < n; ++i) {
    ARR_REQUIRE(rp[i] <= rp[i + 1], "rowptr must be non-decreasing");
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
      ARR_REQUIRE(ci[q] >= 0 && ci[q] < n, "column index out of range");
      ARR_REQUIRE(q == rp[i] || ci[q - 1] < ci[q], "column indices must be strictly increasing within a row");
    }
  }
  std::vector<double> v(vt.begin(), vt.end());
  arr::RowSplit sp;
  arr::split_rows(n, rp.data(), ci.data(), v.data(), sp, A->row_form);
  std::vector<T> cv(sp.coef.begin(), sp.coef.end()), ov(sp.oval.begin(), sp.oval.end());
  auto d = std::make_unique<SplitDev<T>>();
  const int64_t no = (int64_t)sp.ocol.size();
  d->coef.alloc(sizeof(T) * 8 * n);
  ARR_HIP(hipMemcpy(d->coef.p, cv.data(), sizeof(T) * 8 * n, hipMemcpyHostToDevice));
  if (!sp.gx) {
    d->fcol.alloc(sizeof(int32_t) * 4 * n);
    ARR_HIP(hipMemcpy(d->fcol.p, sp.fcol.data(), sizeof(int32_t) * 4 * n, hipMemcpyHostToDevice));
  }
  if (no) {
    d->orp.alloc(sizeof(int64_t) * (n + 1));
    d->ocol.alloc(sizeof(int32_t) * no);
    d->oval.alloc(sizeof(T) * no);
    ARR_HIP(hipMemcpy(d->orp.p, sp.orp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    ARR_HIP(hipMemcpy(d->ocol.p, sp.ocol.data(), sizeof(int32_t) * no, hipMemcpyHostToDevice));
    ARR_HIP(hipMemcpy(d->oval.p, ov.data(), sizeof(T) * no, hipMemcpyHostToDevice));
  }
  d->M = arr::DevCSR<T>{n,
                        nnz,
                        (const T *)d->coef.p,
                        (const int32_t *)d->fcol.p,
                        no ? (const int64_t *)d->orp.p : nullptr,
                        no ? (const int32_t *)d->ocol.p : nullptr,
                        no ? (const T *)d->oval.p : nullptr,
                        sp.pair,
                        sp.kf,
                        sp.gx,
                        sp.gy,
                        sp.gz};
  return d;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Checks a host CSR (row pointers, column range and order) and splits it into
// the row form `form` (arr_row_form_t) selects.
void host_row_split(const arr_csr_t *csr, int32_t form, arr::RowSplit &sp);

// Device address of `scratch` on the current device, looked up once per device
// (each device holds its own copy of the array at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

double *scratch_on_device() {
  int dev = -1;
  ARR_HIP(hipGetDevice(&dev));
  ARR_REQUIRE(dev >= 0 && dev < kMaxDevices, "device ordinal out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    ARR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ARR_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

void arr_options_default(arr_options_t *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->w = 0;
  o->p0 = 1;
  o->p_max = 3;
  o->d0 = 3;
  o->d_max = 15;
  o->maxit = 30;
  o->maxit1 = 10;
  o->maxit2 = 5;
  o->tol1 = 0.0;
  o->precision = ARR_FP64;
  o->paper_faithful = 0;
  o->lanczos_steps = 100;
  o->device = 0;
  o->seed = 2;
  o->mixed_switch = 1e-2;
  o->mixed_contin = 1e-2;
  o->verbose = 0;
  o->timing = 0;
  o->keep_vectors = 1;
}

int arr_row_form(const arr_csr_t *csr, int32_t form, int64_t *pair, int32_t *far_slots, int64_t *overflow) {
  return guarded(nullptr, [&]() {
    arr::RowSplit sp;
    host_row_split(csr, form, sp);
    if (pair) *pair = sp.pair;
    if (far_slots) *far_slots = sp.kf;
    if (overflow) *overflow = (int64_t)sp.ocol.size();
    return ARR_OK;
  });
}

int arr_row_grid(const arr_csr_t *csr, int32_t form, int64_t *dims) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(dims != nullptr, "dims is NULL");
    arr::RowSplit sp;
    host_row_split(csr, form, sp);
    dims[0] = sp.gx;
    dims[1] = sp.gy;
    dims[2] = sp.gz;
    return ARR_OK;
  });
}

}  // extern "C"

namespace {
void host_row_split(const arr_csr_t *csr, int32_t form, arr::RowSplit &sp) {
  {
    ARR_REQUIRE(csr && csr->n > 0 && csr->nnz >= 0 && csr->rowptr, "csr is NULL or empty");
    ARR_REQUIRE(csr->nnz == 0 || csr->colind, "csr arrays are NULL");
    ARR_REQUIRE(form >= ARR_ROW_AUTO && form <= ARR_ROW_GRID, "unknown row form");
    const int64_t n = csr->n, *rp = csr->rowptr;
    ARR_REQUIRE(rp[0] == 0 && rp[n] == csr->nnz, "rowptr[0] must be 0 and rowptr[n] must equal nnz");
    for (int64_t i = 0; i < n; ++i) {
      ARR_REQUIRE(rp[i] <= rp[i + 1], "rowptr must be non-decreasing");
      for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
        ARR_REQUIRE(csr->colind[q] >= 0 && csr->colind[q] < n, "column index out of range");
        ARR_REQUIRE(q == rp[i] || csr->colind[q - 1] < csr->colind[q],
                    "column indices must be strictly increasing within a row");
      }
    }
    // the form depends on the pattern only: unit values stand in when val is NULL
    std::vector<double> ones;
    const double *val = csr->val;
    if (!val) {
      ones.assign((size_t)csr->nnz, 1.0);
      val = ones.data();
    }
    arr::split_rows(n, rp, csr->colind, val, sp, form);
  }
}
}  // namespace

extern "C" {

int arr_create_ex(const arr_csr_t *csr, int64_t n, int32_t k, arr_which_t which, double tol,
                  const arr_options_t *opts, arr_handle_t *out) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    arr_options_t o;
    if (opts)
      o = *opts;
    else
      arr_options_default(&o);
    auto h = std::make_unique<arr_solver>();
    h->s = std::make_unique<arr::Solver>(csr, n, k, (int)which, tol, o);
    *out = h.release();
    return ARR_OK;
  });
}

int arr_create(const arr_csr_t *csr, int64_t n, int32_t k, arr_which_t which, double tol, arr_handle_t *out) {
  return arr_create_ex(csr, n, k, which, tol, nullptr, out);
}

int arr_set_initial_block(arr_handle_t h, const double *X0, int64_t ld) {
  if (!h) return ARR_EINVAL;
  return guarded(&h->err, [&]() {
    h->s->set_initial_block(X0, ld);
    return ARR_OK;
  });
}

int arr_solve(arr_handle_t h) {
  if (!h) return ARR_EINVAL;
  return guarded(&h->err, [&]() { return h->s->solve(); });
}

int arr_get_eigpairs(arr_handle_t h, double *evals, double *evecs, int64_t ldv, double *resid) {
  if (!h) return ARR_EINVAL;
  if (!h->s->solved) {
    h->err = "arr_get_eigpairs called before arr_solve";
    return ARR_ESTATE;
  }
  return guarded(&h->err, [&]() {
    h->s->get(evals, evecs, ldv, resid);
    return ARR_OK;
  });
}

int arr_get_residuals(arr_handle_t h, double *resid, double *resid_norm_a, double *rnorm) {
  if (!h) return ARR_EINVAL;
  if (!h->s->solved) {
    h->err = "arr_get_residuals called before arr_solve";
    return ARR_ESTATE;
  }
  return guarded(&h->err, [&]() {
    h->s->get_residuals(resid, resid_norm_a, rnorm);
    return ARR_OK;
  });
}

int arr_get_fp32_stage_values(arr_handle_t h, double *evals) {
  if (!h || !evals) return ARR_EINVAL;
  if (!h->s->solved || h->s->fp32_stage_values().empty()) {
    h->err = h->s->solved ? "arr_get_fp32_stage_values: the solve had no FP32 stage"
                          : "arr_get_fp32_stage_values called before arr_solve";
    return ARR_ESTATE;
  }
  const std::vector<double> &v = h->s->fp32_stage_values();
  std::copy(v.begin(), v.end(), evals);
  return ARR_OK;
}

int arr_get_stats(arr_handle_t h, arr_stats_t *s) {
  if (!h || !s) return ARR_EINVAL;
  *s = h->s->stats;
  return ARR_OK;
}

const char *arr_last_error(arr_handle_t h) { return h ? h->err.c_str() : g_err.c_str(); }
const char *arr_last_global_error(void) { return g_err.c_str(); }

void arr_destroy(arr_handle_t h) {
  if (!h) return;
  // a request still held by a server must finish before its solver goes away
  if (arr::Server *srv = h->s->server) {
    try {
      srv->wait(h->s->ticket, nullptr);
    } catch (...) {
    }
  }
  delete h;
}

// ---- serving -------------------------------------------------------------------

void arr_server_opts_default(arr_server_opts_t *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget_bytes = 0;
  o->max_slots = 4;
  o->device = 0;
  o->batch_spmm = 0;
}

int arr_server_create(const arr_server_opts_t *o, arr_server_t *out) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    arr_server_opts_t d;
    if (o)
      d = *o;
    else
      arr_server_opts_default(&d);
    ARR_REQUIRE(d.max_slots >= 0, "max_slots must be >= 0");
    ARR_REQUIRE(d.batch_spmm == 0 || d.batch_spmm == 1, "batch_spmm must be 0 or 1");
    ARR_REQUIRE(d.reserved == 0, "reserved must be 0");
    auto s = std::make_unique<arr_server>();
    s->s = std::make_unique<arr::Server>(d);
    *out = s.release();
    return ARR_OK;
  });
}

int arr_footprint(arr_handle_t h, uint64_t *bytes) {
  if (!h || !bytes) return ARR_EINVAL;
  return guarded(&h->err, [&]() {
    *bytes = h->s->footprint();
    return ARR_OK;
  });
}

int arr_submit(arr_server_t s, arr_handle_t h, uint64_t *ticket) {
  if (!s || !h || !ticket) return ARR_EINVAL;
  return guarded(nullptr, [&]() {
    *ticket = s->s->submit(h->s.get());
    return ARR_OK;
  });
}

int arr_poll(arr_server_t s, uint64_t ticket, int *done) {
  if (!s || !done) return ARR_EINVAL;
  return guarded(nullptr, [&]() {
    *done = s->s->poll(ticket, nullptr) ? 1 : 0;
    return ARR_OK;
  });
}

int arr_wait(arr_server_t s, uint64_t ticket) {
  if (!s) return ARR_EINVAL;
  return guarded(nullptr, [&]() {
    std::string e;
    const int st = s->s->wait(ticket, &e);
    if (st < 0) throw arr::Error(st, e.empty() ? std::string("request failed") : e);
    return st;
  });
}

int arr_request_times(arr_server_t s, uint64_t ticket, double *t_submit, double *t_admit, double *t_done) {
  if (!s) return ARR_EINVAL;
  return guarded(nullptr, [&]() {
    s->s->times(ticket, t_submit, t_admit, t_done);
    return ARR_OK;
  });
}

int arr_server_batch_stats(arr_server_t s, int64_t *batches, int64_t *launches) {
  if (!s || !batches || !launches) return ARR_EINVAL;
  s->s->batch_stats(batches, launches);
  return ARR_OK;
}

void arr_server_destroy(arr_server_t s) { delete s; }

// ---- step-level entry points ----------------------------------------------

int arr_filter_step(const arr_dev_csr_t *A, int64_t w, const void *Yin, int64_t ldy, const void *Z, int64_t ldz,
                    void *Yout, int64_t ldo, double alpha, double beta, double gamma, double *colsumsq,
                    void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(A && w >= 0 && ldy >= w && ldo >= w && (!Z || ldz >= w), "filter_step: bad sizes");
    ARR_REQUIRE(Yin && Yout && Yin != Yout, "filter_step: Yin/Yout NULL or aliased");
    hipStream_t s = as_stream(stream);
    arr::DevBuf part;
    double *pp = nullptr;
    if (colsumsq) {
      part.alloc(sizeof(double) * arr::spmm_groups(A->n) * std::max<int64_t>(1, w));
      pp = part.as<double>();
    }
    int groups;
    if (A->dtype == 0) {
      auto S = dev_split<double>(A);
      groups = arr::launch_filter_spmm<double>(S->M, arr::Blk<const double>{(const double *)Yin, ldy, (int)w},
                                               arr::Blk<const double>{(const double *)Z, ldz, Z ? (int)w : 0},
                                               arr::Blk<double>{(double *)Yout, ldo, (int)w}, alpha, beta, gamma, pp, s);
    } else {
      ARR_REQUIRE(A->dtype == 1, "dtype must be 0 (FP64) or 1 (FP32)");
      auto S = dev_split<float>(A);
      groups = arr::launch_filter_spmm<float>(S->M, arr::Blk<const float>{(const float *)Yin, ldy, (int)w},
                                              arr::Blk<const float>{(const float *)Z, ldz, Z ? (int)w : 0},
                                              arr::Blk<float>{(float *)Yout, ldo, (int)w}, alpha, beta, gamma, pp, s);
    }
    if (colsumsq) arr::launch_reduce_groups(pp, groups, (int)w, colsumsq, false, s);
    ARR_HIP(hipStreamSynchronize(s));  // before the temporary buffers go
    return ARR_OK;
  });
}

int arr_filter_step_batch(int32_t count, const arr_dev_csr_t *const *A, const int64_t *w, const void *const *Yin,
                          const int64_t *ldy, const void *const *Z, const int64_t *ldz, void *const *Yout,
                          const int64_t *ldo, const double *alpha, const double *beta, const double *gamma,
                          double *const *colsumsq, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(count >= 1 && A && w && Yin && ldy && ldz && Yout && ldo && alpha && beta && gamma,
                "filter_step_batch: NULL array or count < 1");
    hipStream_t s = as_stream(stream);
    std::vector<std::unique_ptr<SplitDev<double>>> m64(count);
    std::vector<std::unique_ptr<SplitDev<float>>> m32(count);
    std::vector<arr::DevBuf> part(count);
    std::vector<int> groups(count, 0);
    for (int i = 0; i < count; ++i) {
      const void *Zi = Z ? Z[i] : nullptr;
      ARR_REQUIRE(A[i] && w[i] >= 0 && ldy[i] >= w[i] && ldo[i] >= w[i] && (!Zi || ldz[i] >= w[i]),
                  "filter_step_batch: bad sizes in item " + std::to_string(i));
      ARR_REQUIRE(Yin[i] && Yout[i] && Yin[i] != Yout[i],
                  "filter_step_batch: Yin/Yout NULL or aliased in item " + std::to_string(i));
      ARR_REQUIRE(A[i]->dtype == 0 || A[i]->dtype == 1, "dtype must be 0 (FP64) or 1 (FP32)");
      if (A[i]->dtype == 0)
        m64[i] = dev_split<double>(A[i]);
      else
        m32[i] = dev_split<float>(A[i]);
      if (colsumsq && colsumsq[i]) part[i].alloc(sizeof(double) * arr::spmm_groups(A[i]->n) * std::max<int64_t>(1, w[i]));
    }
    // task table: at most one launch per 64 columns of an item, each with at
    // most spmm_groups(n) workgroups
    size_t cap = 4096;
    for (int i = 0; i < count; ++i)
      cap += ((size_t)w[i] / 64 + 1) * (sizeof(arr::SpmmTask) + 256 + sizeof(int2) * arr::spmm_groups(A[i]->n));
    arr::SpmmBatch batch(cap);
    struct Install {
      arr::SpmmBatch *prev;
      explicit Install(arr::SpmmBatch *b) : prev(arr::spmm_batch()) { arr::spmm_batch() = b; }
      ~Install() { arr::spmm_batch() = prev; }
    };
    {
      Install in(&batch);
      for (int i = 0; i < count; ++i) {
        const void *Zi = Z ? Z[i] : nullptr;
        double *pp = part[i].as<double>();
        const int wi = (int)w[i];
        if (A[i]->dtype == 0)
          groups[i] = arr::launch_filter_spmm<double>(
              m64[i]->M, arr::Blk<const double>{(const double *)Yin[i], ldy[i], wi},
              arr::Blk<const double>{(const double *)Zi, ldz[i], Zi ? wi : 0},
              arr::Blk<double>{(double *)Yout[i], ldo[i], wi}, alpha[i], beta[i], gamma[i], pp, s);
        else
          groups[i] = arr::launch_filter_spmm<float>(
              m32[i]->M, arr::Blk<const float>{(const float *)Yin[i], ldy[i], wi},
              arr::Blk<const float>{(const float *)Zi, ldz[i], Zi ? wi : 0},
              arr::Blk<float>{(float *)Yout[i], ldo[i], wi}, alpha[i], beta[i], gamma[i], pp, s);
      }
    }
    batch.run(s);
    for (int i = 0; i < count; ++i)
      if (colsumsq && colsumsq[i])
        arr::launch_reduce_groups(part[i].as<double>(), groups[i], (int)w[i], colsumsq[i], false, s);
    ARR_HIP(hipStreamSynchronize(s));  // before the temporary buffers go
    return ARR_OK;
  });
}

int arr_filter_coefficients(int32_t d, double *out) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(out && d >= 1 && d <= 32, "filter_coefficients: need 1 <= d <= 32");
    const std::vector<double> g = arr::filter_coefficients(d);
    std::copy(g.begin(), g.end(), out);
    return ARR_OK;
  });
}

int arr_poly(const arr_dev_csr_t *A, int64_t w, void *X, int64_t ld, double shift, double lo, double hi,
             const double *gamma, int32_t d, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(A && X && gamma && d >= 1 && w >= 0 && ld >= w, "poly: bad arguments");
    hipStream_t s = as_stream(stream);
    std::vector<double> g(gamma, gamma + d + 1);
    arr::Work wk;
    wk.ensure_cols(A->n, (int)w);
    const int64_t n = A->n;
    if (A->dtype == 0) {
      arr::DevBuf tmp(sizeof(double) * n * 2 * std::max<int64_t>(1, w));
      double *t = tmp.as<double>();
      auto S = dev_split<double>(A);
      arr::poly_apply_horner<double>(S->M, arr::Blk<double>{(double *)X, ld, (int)w},
                              arr::Blk<double>{t, 2 * w, (int)w}, arr::Blk<double>{t + w, 2 * w, (int)w}, shift, lo,
                              hi, g, wk, false, s);
    } else {
      arr::DevBuf tmp(sizeof(float) * n * 2 * std::max<int64_t>(1, w));
      float *t = tmp.as<float>();
      auto S = dev_split<float>(A);
      arr::poly_apply_horner<float>(S->M, arr::Blk<float>{(float *)X, ld, (int)w},
                             arr::Blk<float>{t, 2 * w, (int)w}, arr::Blk<float>{t + w, 2 * w, (int)w}, shift, lo, hi,
                             g, wk, false, s);
    }
    ARR_HIP(hipStreamSynchronize(s));
    return ARR_OK;
  });
}

int arr_filter_roots(int32_t d, double *roots, double *lead) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(roots && lead && d >= 1 && d <= 64, "filter_roots: bad arguments");
    const arr::FilterPoly fp = arr::filter_poly(d);
    std::copy(fp.roots.begin(), fp.roots.end(), roots);
    *lead = fp.lead;
    return ARR_OK;
  });
}

int arr_filter(const arr_dev_csr_t *A, int64_t w, void *X, int64_t ld, double shift, double lo, double hi,
               int32_t d, int32_t form, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(A && X && d >= 1 && d <= 64 && w >= 0 && ld >= w, "filter: bad arguments");
    ARR_REQUIRE(form == ARR_POLY_PRODUCT || form == ARR_POLY_HORNER || form == ARR_POLY_CHEBYSHEV,
                "filter: unknown form");
    hipStream_t s = as_stream(stream);
    const arr::FilterPoly fp = arr::filter_poly(d);
    arr::Work wk;
    const int64_t n = A->n;
    ARR_REQUIRE(n > 0, "filter: empty matrix");
    wk.ensure_cols(n, (int)w);
    const int iw = (int)w;
    auto run = [&](auto *Xp, auto tag) {
      using T = decltype(tag);
      arr::DevBuf tmp(sizeof(T) * n * 2 * std::max<int64_t>(1, w));
      T *t = tmp.as<T>();
      auto S = dev_split<T>(A);
      arr::poly_apply<T>(S->M, arr::Blk<T>{Xp, ld, iw}, arr::Blk<T>{t, 2 * w, iw}, arr::Blk<T>{t + w, 2 * w, iw},
                         shift, lo, hi, fp, form, wk, false, s);
      ARR_HIP(hipStreamSynchronize(s));
    };
    if (A->dtype == 0)
      run((double *)X, double{});
    else {
      ARR_REQUIRE(A->dtype == 1, "dtype must be 0 (FP64) or 1 (FP32)");
      run((float *)X, float{});
    }
    return ARR_OK;
  });
}

int arr_gn_step(const arr_dev_csr_t *A, int64_t w, void *X, int64_t ld, double shift, double lo, double hi,
                const double *gamma, int32_t d, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(A && X && gamma && d >= 1 && w >= 1 && ld >= w, "gn_step: bad arguments");
    hipStream_t s = as_stream(stream);
    std::vector<double> g(gamma, gamma + d + 1);
    arr::Work wk;
    const int64_t n = A->n;
    ARR_REQUIRE(n > 0, "gn_step: empty matrix");
    wk.ensure_cols(n, (int)w);
    const int iw = (int)w;
    auto run = [&](auto *Xp, auto tag) {
      using T = decltype(tag);
      arr::DevBuf tmp(sizeof(T) * n * 4 * w);
      T *t = tmp.as<T>();
      auto S = dev_split<T>(A);
      auto blk = [&](int q) { return arr::Blk<T>{t + q * w, 4 * w, iw}; };
      arr::FilterPoly fp;
      fp.gamma = g;  // the caller's coefficients, applied by Algorithm 7's recurrence
      arr::gn_step<T>(S->M, arr::Blk<T>{Xp, ld, iw}, blk(0), blk(1), blk(2), blk(3), shift, lo, hi, fp,
                      arr::kPolyHorner, wk, s);
      ARR_HIP(hipStreamSynchronize(s));
    };
    if (A->dtype == 0)
      run((double *)X, double{});
    else {
      ARR_REQUIRE(A->dtype == 1, "dtype must be 0 (FP64) or 1 (FP32)");
      run((float *)X, float{});
    }
    return ARR_OK;
  });
}

int arr_gram(int32_t dtype, int64_t n, const void *X, int64_t ldx, int32_t mx, const void *Y, int64_t ldy, int32_t my,
             double *G, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(X && Y && G && mx >= 0 && my >= 0 && ldx >= mx && ldy >= my && n >= 0, "gram: bad arguments");
    hipStream_t s = as_stream(stream);
    arr::DevBuf work(sizeof(double) * std::max<size_t>(1, arr::gram_work_doubles(n, mx, my)));
    const bool sym = (X == Y && ldx == ldy && mx == my);
    ARR_REQUIRE(dtype >= 0 && dtype <= 2, "gram: dtype must be 0, 1 or 2");
    if (dtype == 0)
      arr::launch_gram<double>(n, arr::Blk<const double>{(const double *)X, ldx, mx},
                               arr::Blk<const double>{(const double *)Y, ldy, my}, G, work.as<double>(), sym, s);
    else
      arr::launch_gram<float>(n, arr::Blk<const float>{(const float *)X, ldx, mx},
                              arr::Blk<const float>{(const float *)Y, ldy, my}, G, work.as<double>(), sym, s,
                              dtype == 2);
    ARR_HIP(hipStreamSynchronize(s));
    return ARR_OK;
  });
}

int arr_gram_noalloc(int32_t dtype, int64_t n, const void *X, int64_t ldx, int32_t mx, const void *Y, int64_t ldy,
                     int32_t my, double *G, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(X && Y && G && mx >= 0 && my >= 0 && ldx >= mx && ldy >= my && n >= 0, "gram_noalloc: bad arguments");
    ARR_REQUIRE(dtype >= 0 && dtype <= 2, "gram_noalloc: dtype must be 0, 1 or 2");
    ARR_REQUIRE((int64_t)mx * my <= kNoallocScratchDoubles,
                "gram_noalloc: mx * my = " + std::to_string((int64_t)mx * my) + " exceeds the scratch array (" +
                    std::to_string(kNoallocScratchDoubles) + " doubles); use arr_gram");
    hipStream_t s = as_stream(stream);
    double *work = scratch_on_device();
    const bool sym = (X == Y && ldx == ldy && mx == my);
    if (dtype == 0)
      arr::launch_gram<double>(n, arr::Blk<const double>{(const double *)X, ldx, mx},
                               arr::Blk<const double>{(const double *)Y, ldy, my}, G, work, sym, s, false,
                               kNoallocScratchDoubles);
    else
      arr::launch_gram<float>(n, arr::Blk<const float>{(const float *)X, ldx, mx},
                              arr::Blk<const float>{(const float *)Y, ldy, my}, G, work, sym, s, dtype == 2,
                              kNoallocScratchDoubles);
    return ARR_OK;
  });
}

int arr_block_update(int32_t dtype, int64_t n, int32_t m, int32_t c, double alpha, const void *X, int64_t ldx,
                     const double *W, int64_t ldw, double beta, void *Y, int64_t ldy, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(X && W && Y && X != Y && m >= 0 && c >= 0 && ldx >= m && ldw >= c && ldy >= c, "block_update: bad arguments");
    hipStream_t s = as_stream(stream);
    ARR_REQUIRE(dtype >= 0 && dtype <= 2, "block_update: dtype must be 0, 1 or 2");
    if (dtype == 0)
      arr::launch_update<double>(n, arr::Blk<const double>{(const double *)X, ldx, m}, W, ldw, c, alpha, beta,
                                 arr::Blk<double>{(double *)Y, ldy, c}, s);
    else
      arr::launch_update<float>(n, arr::Blk<const float>{(const float *)X, ldx, m}, W, ldw, c, alpha, beta,
                                arr::Blk<float>{(float *)Y, ldy, c}, s, false, dtype == 2);
    return ARR_OK;
  });
}

int arr_rcond_gram(int32_t dtype, int64_t n, int32_t w, const void *X, int64_t ld, double *rc, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(X && rc && w > 0 && ld >= w, "rcond_gram: bad arguments");
    arr::Work wk;
    hipStream_t s = as_stream(stream);
    if (dtype == 0)
      *rc = arr::rcond_gram<double>(n, arr::Blk<const double>{(const double *)X, ld, w}, wk, s);
    else
      *rc = arr::rcond_gram<float>(n, arr::Blk<const float>{(const float *)X, ld, w}, wk, s);
    return ARR_OK;
  });
}

int arr_orthonormalize(int64_t n, int32_t m, double *Z, int64_t ld, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(Z && m > 0 && ld >= m && n >= m, "orthonormalize: bad arguments");
    hipStream_t s = as_stream(stream);
    arr::Work wk;
    arr::DevBuf alt(sizeof(double) * n * m);
    const arr::Blk<const double> none{nullptr, 0, 0};
    arr::Blk<double> U = arr::orthonormalize<double>(n, arr::Blk<double>{Z, ld, m}, arr::Blk<double>{alt.as<double>(), m, m},
                                                     none, wk, s, nullptr);
    if (U.p != Z) arr::launch_copy<double>(n, m, Z, ld, U.p, U.ld, s);
    ARR_HIP(hipStreamSynchronize(s));
    return ARR_OK;
  });
}

int arr_syev(int32_t m, double *H, double *evals, double *V, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(H && evals && V && m > 0, "syev: bad arguments");
    hipStream_t s = as_stream(stream);
    arr::Jacobi jac;
    std::vector<double> ev;
    jac.solve(m, H, V, ev, s);
    ARR_HIP(hipMemcpyAsync(evals, ev.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
    ARR_HIP(hipStreamSynchronize(s));
    return ARR_OK;
  });
}

int arr_augmented_rr(const arr_dev_csr_t *A, int64_t w, const double *X, int64_t ld, int32_t p, const double *Qc,
                     int64_t ldq, int32_t nc, double *Y, int64_t ldy, double *ritz_vals, void *stream) {
  return guarded(nullptr, [&]() {
    ARR_REQUIRE(A && A->dtype == 0 && X && Y && ritz_vals && w > 0 && p >= 0 && ld >= w && ldy >= w, "augmented_rr: bad arguments");
    ARR_REQUIRE(nc == 0 || (Qc && ldq >= nc), "augmented_rr: bad Qc");
    const int64_t n = A->n;
    const int m = (int)((p + 1) * w);
    ARR_REQUIRE(m <= n, "augmented_rr: (p+1) w must not exceed n");
    hipStream_t s = as_stream(stream);
    auto S = dev_split<double>(A);
    const arr::DevCSR<double> &M = S->M;
    arr::Work wk;
    arr::DevBuf zb(sizeof(double) * n * m), ub(sizeof(double) * n * m), wb(sizeof(double) * n * m);
    const int iw = (int)w;
    arr::Blk<double> Z{zb.as<double>(), m, m};
    arr::launch_copy<double>(n, iw, Z.p, m, X, ld, s);
    const arr::Blk<const double> none{nullptr, 0, 0};
    for (int i = 1; i <= p; ++i)
      arr::launch_filter_spmm<double>(M, arr::Blk<const double>{Z.p + (i - 1) * iw, m, iw}, none,
                                      arr::Blk<double>{Z.p + i * iw, m, iw}, 1.0, 0.0, 0.0, nullptr, s);
    const arr::Blk<const double> Q{Qc, ldq, nc};
    if (nc) arr::project_out<double>(n, Q, Z, wk, s);
    const double *rinv = nullptr;
    arr::Blk<double> U =
        arr::orthonormalize<double>(n, Z, arr::Blk<double>{ub.as<double>(), m, m}, Q, wk, s, nullptr, &rinv);
    std::vector<double> ev;
    arr::rayleigh_ritz<double>(M, n, arr::Blk<const double>{U.p, U.ld, m}, arr::Blk<double>{wb.as<double>(), m, m}, wk,
                               ev, s, rinv);
    const double *V = wk.small.as<double>() + (size_t)m * m;
    arr::launch_update<double>(n, arr::Blk<const double>{U.p, U.ld, m}, V, m, iw, 1.0, 0.0, arr::Blk<double>{Y, ldy, iw}, s);
    std::copy(ev.begin(), ev.begin() + iw, ritz_vals);
    ARR_HIP(hipStreamSynchronize(s));
    return ARR_OK;
  });
}

}  // extern "C"
