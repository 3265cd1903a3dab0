"""Thin ctypes binding of libarr.so (include/arr.h). Argument marshalling only:
every step of the solver runs in the HIP library. Device buffers for the
step-level calls are torch tensors on a ROCm device (torch is used for device
memory and streams only).

Loading fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libarr.so")

ARR_OK = 0
ARR_NOT_CONVERGED = 1
ARR_STAGNATED = 2
ARR_EINVAL = -1
ARR_ENOMEM = -2
ARR_EDEVICE = -3
ARR_ESTATE = -4
ARR_EBREAKDOWN = -5
LARGEST = 0
SMALLEST = 1
FP64 = 0
MIXED = 1
INNER_MPM = 0
INNER_GN = 1
POLY_PRODUCT = 0
POLY_HORNER = 1
POLY_CHEBYSHEV = 2
ROW_AUTO = 0
ROW_PLAIN = 1
ROW_PAIRED = 2
ROW_GRID = 3


class ArrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"arr error {code}: {msg}")
        self.code = code


class arr_csr_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class arr_dev_csr_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("row_form", ctypes.c_int32)]


class arr_options_t(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("p0", ctypes.c_int32), ("p_max", ctypes.c_int32),
                ("d0", ctypes.c_int32), ("d_max", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("maxit1", ctypes.c_int32), ("maxit2", ctypes.c_int32), ("tol1", ctypes.c_double),
                ("precision", ctypes.c_int32), ("paper_faithful", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("device", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("mixed_switch", ctypes.c_double), ("verbose", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("keep_vectors", ctypes.c_int32),
                ("inner_solver", ctypes.c_int32),
                ("poly_form", ctypes.c_int32),
                ("row_form", ctypes.c_int32),
                ("debug_nan_poly", ctypes.c_int32),
                ("lean_memory", ctypes.c_int32),
                ("mixed_contin", ctypes.c_double),
                ("debug_fp32_collapse", ctypes.c_int32),
                ("early_contin", ctypes.c_double)]


class arr_server_opts_t(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32), ("device", ctypes.c_int32),
                ("batch_spmm", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class arr_stats_t(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("arr_calls", ctypes.c_int32),
                ("poly_calls", ctypes.c_int32), ("final_p", ctypes.c_int32), ("final_d", ctypes.c_int32),
                ("n_locked", ctypes.c_int32), ("fp32_outer", ctypes.c_int32),
                ("spmm_degrees", ctypes.c_int64), ("spmm_cols", ctypes.c_int64),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("norm_est", ctypes.c_double),
                ("maxres", ctypes.c_double), ("t_total", ctypes.c_double), ("t_setup", ctypes.c_double),
                ("t_filter", ctypes.c_double), ("t_arr", ctypes.c_double), ("t_dense", ctypes.c_double),
                ("spmm_launches", ctypes.c_int64), ("spmm_ms", ctypes.c_double), ("spmm_bytes", ctypes.c_double),
                ("spmm_cols_per_lane", ctypes.c_int32), ("spmm_fp64", ctypes.c_int32),
                ("spmm_vec", ctypes.c_int32),
                ("gram64_launches", ctypes.c_int64), ("gram32_launches", ctypes.c_int64),
                ("upd64_launches", ctypes.c_int64), ("upd32_launches", ctypes.c_int64),
                ("gram64_ms", ctypes.c_double), ("gram64_flops", ctypes.c_double),
                ("gram32_ms", ctypes.c_double), ("gram32_flops", ctypes.c_double),
                ("upd64_ms", ctypes.c_double), ("upd64_flops", ctypes.c_double),
                ("upd32_ms", ctypes.c_double), ("upd32_flops", ctypes.c_double),
                ("spmm32_launches", ctypes.c_int64), ("spmm32_ms", ctypes.c_double), ("spmm32_bytes", ctypes.c_double),
                ("spmm32_cols_per_lane", ctypes.c_int32), ("spmm32_vec", ctypes.c_int32),
                ("fp32_maxres", ctypes.c_double), ("spmm_flags", ctypes.c_int32), ("spmm32_flags", ctypes.c_int32),
                ("nan_retries", ctypes.c_int32), ("maxres_explicit", ctypes.c_double),
                ("maxres_norm_a", ctypes.c_double), ("arr_m2", ctypes.c_double),
                ("handover_contin", ctypes.c_int32), ("fp32_collapsed", ctypes.c_int32),
                ("early_contin", ctypes.c_int32)]


EXPORTS = ["arr_options_default", "arr_create", "arr_create_ex", "arr_set_initial_block", "arr_solve",
           "arr_get_eigpairs", "arr_get_residuals", "arr_get_fp32_stage_values", "arr_get_stats", "arr_last_error",
           "arr_last_global_error", "arr_destroy",
           "arr_filter_step", "arr_filter_step_batch", "arr_poly", "arr_filter", "arr_filter_roots", "arr_gn_step",
           "arr_filter_coefficients", "arr_gram", "arr_gram_noalloc", "arr_block_update",
           "arr_rcond_gram", "arr_orthonormalize", "arr_syev", "arr_augmented_rr", "arr_server_opts_default",
           "arr_server_create", "arr_footprint", "arr_submit", "arr_poll", "arr_wait", "arr_request_times",
           "arr_server_destroy", "arr_server_batch_stats", "arr_row_form", "arr_row_grid"]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libarr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1507_06078_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.arr_options_default.argtypes = [P(arr_options_t)]
    L.arr_options_default.restype = None
    L.arr_create.argtypes = [P(arr_csr_t), i64, i32, i32, f64, P(vp)]
    L.arr_create_ex.argtypes = [P(arr_csr_t), i64, i32, i32, f64, P(arr_options_t), P(vp)]
    L.arr_set_initial_block.argtypes = [vp, vp, i64]
    L.arr_solve.argtypes = [vp]
    L.arr_get_eigpairs.argtypes = [vp, vp, vp, i64, vp]
    L.arr_get_residuals.argtypes = [vp, vp, vp, vp]
    L.arr_get_fp32_stage_values.argtypes = [vp, vp]
    L.arr_get_stats.argtypes = [vp, P(arr_stats_t)]
    L.arr_last_error.argtypes = [vp]
    L.arr_last_error.restype = ctypes.c_char_p
    L.arr_last_global_error.argtypes = []
    L.arr_last_global_error.restype = ctypes.c_char_p
    L.arr_destroy.argtypes = [vp]
    L.arr_destroy.restype = None
    L.arr_filter_step.argtypes = [P(arr_dev_csr_t), i64, vp, i64, vp, i64, vp, i64, f64, f64, f64, vp, vp]
    L.arr_filter_step_batch.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.arr_poly.argtypes = [P(arr_dev_csr_t), i64, vp, i64, f64, f64, f64, vp, i32, vp]
    L.arr_gn_step.argtypes = [P(arr_dev_csr_t), i64, vp, i64, f64, f64, f64, vp, i32, vp]
    L.arr_filter.argtypes = [P(arr_dev_csr_t), i64, vp, i64, f64, f64, f64, i32, i32, vp]
    L.arr_filter_roots.argtypes = [i32, vp, vp]
    L.arr_filter_coefficients.argtypes = [i32, vp]
    L.arr_row_form.argtypes = [P(arr_csr_t), i32, vp, vp, vp]
    L.arr_row_grid.argtypes = [P(arr_csr_t), i32, vp]
    L.arr_gram.argtypes = [i32, i64, vp, i64, i32, vp, i64, i32, vp, vp]
    L.arr_gram_noalloc.argtypes = [i32, i64, vp, i64, i32, vp, i64, i32, vp, vp]
    L.arr_block_update.argtypes = [i32, i64, i32, i32, f64, vp, i64, vp, i64, f64, vp, i64, vp]
    L.arr_rcond_gram.argtypes = [i32, i64, i32, vp, i64, vp, vp]
    L.arr_orthonormalize.argtypes = [i64, i32, vp, i64, vp]
    L.arr_syev.argtypes = [i32, vp, vp, vp, vp]
    L.arr_augmented_rr.argtypes = [P(arr_dev_csr_t), i64, vp, i64, i32, vp, i64, i32, vp, i64, vp, vp]
    L.arr_server_opts_default.argtypes = [P(arr_server_opts_t)]
    L.arr_server_opts_default.restype = None
    L.arr_server_create.argtypes = [P(arr_server_opts_t), P(vp)]
    L.arr_footprint.argtypes = [vp, P(ctypes.c_uint64)]
    L.arr_submit.argtypes = [vp, vp, P(ctypes.c_uint64)]
    L.arr_poll.argtypes = [vp, ctypes.c_uint64, P(ctypes.c_int)]
    L.arr_wait.argtypes = [vp, ctypes.c_uint64]
    L.arr_request_times.argtypes = [vp, ctypes.c_uint64, vp, vp, vp]
    L.arr_server_destroy.argtypes = [vp]
    L.arr_server_destroy.restype = None
    L.arr_server_batch_stats.argtypes = [vp, vp, vp]
    void_fns = ("arr_options_default", "arr_destroy", "arr_last_error", "arr_last_global_error",
                "arr_server_opts_default", "arr_server_destroy")
    for name in EXPORTS:
        if name not in void_fns:
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(code: int, handle=None) -> int:
    if code < 0:
        L = lib()
        msg = (L.arr_last_error(handle) if handle else L.arr_last_global_error()) or b""
        raise ArrError(code, msg.decode(errors="replace"))
    return code


# ---- whole-solve API -------------------------------------------------------

def arr_options_default() -> arr_options_t:
    o = arr_options_t()
    lib().arr_options_default(ctypes.byref(o))
    return o


class Handle:
    """Owns an arr_handle_t; keeps the host CSR arrays alive only during create."""

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "ptr", None):
            lib().arr_destroy(self.ptr)
            self.ptr = None


def _host_csr(csr) -> tuple[arr_csr_t, tuple]:
    rowptr = np.ascontiguousarray(csr.rowptr, dtype=np.int64)
    colind = np.ascontiguousarray(csr.colind, dtype=np.int32)
    val = np.ascontiguousarray(csr.val, dtype=np.float64)
    c = arr_csr_t(int(csr.n), int(rowptr[-1]), rowptr.ctypes.data, colind.ctypes.data, val.ctypes.data)
    return c, (rowptr, colind, val)


def arr_create(csr, n: int, k: int, which: int, tol: float, opts: arr_options_t | None = None) -> Handle:
    c, keep = _host_csr(csr)
    h = ctypes.c_void_p()
    if opts is None:
        code = lib().arr_create(ctypes.byref(c), int(n), int(k), int(which), float(tol), ctypes.byref(h))
    else:
        code = lib().arr_create_ex(ctypes.byref(c), int(n), int(k), int(which), float(tol), ctypes.byref(opts),
                                   ctypes.byref(h))
    _check(code)
    del keep
    return Handle(h.value)


def arr_row_form(csr, form: int = ROW_AUTO):
    """Row form the SpMM kernels use for a host CSR: (pair offset P, 0 for
    the plain form; far entries gathered per row; overflow entries)."""
    c, keep = _host_csr(csr)
    pair, far, ovf = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().arr_row_form(ctypes.byref(c), int(form), ctypes.addressof(pair), ctypes.addressof(far),
                              ctypes.addressof(ovf)))
    del keep
    return pair.value, far.value, ovf.value


def arr_row_grid(csr, form: int = ROW_AUTO):
    """Grid dimensions (gx, gy, gz) of the grid row form for a host CSR, or
    (0, 0, 0) when the kernels do not use it."""
    c, keep = _host_csr(csr)
    dims = np.zeros(3, dtype=np.int64)
    _check(lib().arr_row_grid(ctypes.byref(c), int(form), dims.ctypes.data))
    del keep
    return tuple(int(d) for d in dims)


def arr_set_initial_block(h: Handle, X0: np.ndarray) -> None:
    X0 = np.ascontiguousarray(X0, dtype=np.float64)
    _check(lib().arr_set_initial_block(h.ptr, X0.ctypes.data, X0.shape[1]), h.ptr)


def arr_solve(h: Handle) -> int:
    return _check(lib().arr_solve(h.ptr), h.ptr)


def arr_get_eigpairs(h: Handle, k: int, n: int, vectors: bool = True):
    ev = np.zeros(k)
    res = np.zeros(k)
    X = np.zeros((n, k)) if vectors else None
    _check(lib().arr_get_eigpairs(h.ptr, ev.ctypes.data, X.ctypes.data if vectors else None, k, res.ctypes.data),
           h.ptr)
    return ev, X, res


def arr_get_residuals(h: Handle, k: int):
    """(resid, resid_norm_a, rnorm): ||r|| / max(1, |lambda|) (eq. resi),
    ||r|| / ||A||_2 (Lanczos estimate) and ||r||, each k values."""
    out = [np.zeros(k) for _ in range(3)]
    _check(lib().arr_get_residuals(h.ptr, *(o.ctypes.data for o in out)), h.ptr)
    return tuple(out)


def arr_get_fp32_stage_values(h: Handle, k: int) -> np.ndarray:
    """The k Ritz values the FP32 stage of a mixed solve handed over."""
    out = np.zeros(k)
    _check(lib().arr_get_fp32_stage_values(h.ptr, out.ctypes.data), h.ptr)
    return out


def arr_get_stats(h: Handle) -> dict:
    s = arr_stats_t()
    _check(lib().arr_get_stats(h.ptr, ctypes.byref(s)), h.ptr)
    return {name: getattr(s, name) for name, _ in arr_stats_t._fields_}


# ---- serving -------------------------------------------------------------------

class Server:
    """Owns an arr_server_t (continuous batching of solves on one GPU)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 4, device: int = 0, batch_spmm: bool = False):
        o = arr_server_opts_t()
        lib().arr_server_opts_default(ctypes.byref(o))
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.max_slots = int(max_slots)
        o.device = int(device)
        o.batch_spmm = 1 if batch_spmm else 0
        p = ctypes.c_void_p()
        _check(lib().arr_server_create(ctypes.byref(o), ctypes.byref(p)))
        self.ptr = p.value

    def submit(self, h: Handle) -> int:
        t = ctypes.c_uint64()
        _check(lib().arr_submit(self.ptr, h.ptr, ctypes.byref(t)))
        # keep the handle alive while the server may use it
        self._held = getattr(self, "_held", [])
        self._held.append(h)
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _check(lib().arr_poll(self.ptr, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> int:
        return _check(lib().arr_wait(self.ptr, ctypes.c_uint64(ticket)))

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().arr_request_times(self.ptr, ctypes.c_uint64(ticket), ctypes.addressof(a), ctypes.addressof(b),
                                       ctypes.addressof(c)))
        return a.value, b.value, c.value

    def batch_stats(self):
        """(multi-request launch rounds, single-request launches they replaced)."""
        b, n = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().arr_server_batch_stats(self.ptr, ctypes.addressof(b), ctypes.addressof(n)))
        return b.value, n.value

    def close(self):
        if getattr(self, "ptr", None):
            lib().arr_server_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        self.close()


def arr_footprint(h: Handle) -> int:
    b = ctypes.c_uint64()
    _check(lib().arr_footprint(h.ptr, ctypes.byref(b)), h.ptr)
    return b.value


def arr_filter_coefficients(d: int) -> np.ndarray:
    out = np.zeros(d + 1)
    _check(lib().arr_filter_coefficients(int(d), out.ctypes.data))
    return out


# ---- step-level API on device tensors ---------------------------------------

def _ptr(t):
    return None if t is None else t.data_ptr()


def _ld(t):
    return 0 if t is None else int(t.stride(0))


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class DeviceCSR:
    """A CSR matrix resident on the device (torch tensors) plus its descriptor."""

    def __init__(self, csr, dtype=None, device="cuda", row_form=ROW_AUTO):
        import torch
        dtype = dtype or torch.float64
        self.n = int(csr.n)
        self.rowptr = torch.as_tensor(np.asarray(csr.rowptr, dtype=np.int64)).to(device)
        self.colind = torch.as_tensor(np.asarray(csr.colind, dtype=np.int32)).to(device)
        self.val = torch.as_tensor(np.asarray(csr.val, dtype=np.float64)).to(device=device, dtype=dtype)
        self.desc = arr_dev_csr_t(self.n, int(self.colind.numel()), self.rowptr.data_ptr(),
                                  self.colind.data_ptr(), self.val.data_ptr(), _dtype_code(self.val),
                                  int(row_form))


def arr_filter_step(A: DeviceCSR, Yin, Z, Yout, alpha: float, beta: float, gamma: float, colsumsq=None):
    w = int(Yout.shape[1])
    _check(lib().arr_filter_step(ctypes.byref(A.desc), w, _ptr(Yin), _ld(Yin), _ptr(Z), _ld(Z), _ptr(Yout),
                                 _ld(Yout), float(alpha), float(beta), float(gamma), _ptr(colsumsq), _stream()))


def arr_filter_step_batch(items):
    """arr_filter_step on every item of `items`, a list of tuples
    (A, Yin, Z, Yout, alpha, beta, gamma, colsumsq), in one multi-request
    launch per kernel variant."""
    cnt = len(items)
    arrs = lambda ctype, vals: (ctype * cnt)(*vals)
    descs = [it[0].desc for it in items]
    A = (ctypes.POINTER(arr_dev_csr_t) * cnt)(*[ctypes.pointer(d) for d in descs])
    vp = ctypes.c_void_p
    _check(lib().arr_filter_step_batch(
        cnt, A, arrs(ctypes.c_int64, [int(it[3].shape[1]) for it in items]),
        arrs(vp, [_ptr(it[1]) for it in items]), arrs(ctypes.c_int64, [_ld(it[1]) for it in items]),
        arrs(vp, [_ptr(it[2]) for it in items]), arrs(ctypes.c_int64, [_ld(it[2]) for it in items]),
        arrs(vp, [_ptr(it[3]) for it in items]), arrs(ctypes.c_int64, [_ld(it[3]) for it in items]),
        arrs(ctypes.c_double, [float(it[4]) for it in items]), arrs(ctypes.c_double, [float(it[5]) for it in items]),
        arrs(ctypes.c_double, [float(it[6]) for it in items]), arrs(vp, [_ptr(it[7]) for it in items]), _stream()))


def arr_poly(A: DeviceCSR, X, shift: float, lo: float, hi: float, gamma: np.ndarray):
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    _check(lib().arr_poly(ctypes.byref(A.desc), int(X.shape[1]), _ptr(X), _ld(X), float(shift), float(lo),
                          float(hi), g.ctypes.data, len(g) - 1, _stream()))


def arr_filter_roots(d: int):
    """Roots of psi_d (Leja order) and its leading coefficient."""
    r = np.zeros(d)
    lead = ctypes.c_double()
    _check(lib().arr_filter_roots(int(d), r.ctypes.data, ctypes.addressof(lead)))
    return r, lead.value


def arr_filter(A: DeviceCSR, X, shift: float, lo: float, hi: float, d: int, form: int = POLY_PRODUCT):
    _check(lib().arr_filter(ctypes.byref(A.desc), int(X.shape[1]), _ptr(X), _ld(X), float(shift), float(lo),
                            float(hi), int(d), int(form), _stream()))


def arr_gn_step(A: DeviceCSR, X, shift: float, lo: float, hi: float, gamma: np.ndarray):
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    _check(lib().arr_gn_step(ctypes.byref(A.desc), int(X.shape[1]), _ptr(X), _ld(X), float(shift), float(lo),
                             float(hi), g.ctypes.data, len(g) - 1, _stream()))


def arr_gram(X, Y, G, fp32_cores: bool = False):
    code = 2 if (fp32_cores and _dtype_code(X) == 1) else _dtype_code(X)
    _check(lib().arr_gram(code, int(X.shape[0]), _ptr(X), _ld(X), int(X.shape[1]), _ptr(Y), _ld(Y),
                          int(Y.shape[1]), _ptr(G), _stream()))


def arr_gram_noalloc(X, Y, G, fp32_cores: bool = False):
    """arr_gram through the allocation-free entry point (asynchronous on the
    current stream)."""
    code = 2 if (fp32_cores and _dtype_code(X) == 1) else _dtype_code(X)
    _check(lib().arr_gram_noalloc(code, int(X.shape[0]), _ptr(X), _ld(X), int(X.shape[1]), _ptr(Y), _ld(Y),
                                  int(Y.shape[1]), _ptr(G), _stream()))


def arr_block_update(X, W, Y, alpha: float = 1.0, beta: float = 0.0, fp32_cores: bool = False):
    code = 2 if (fp32_cores and _dtype_code(X) == 1) else _dtype_code(X)
    _check(lib().arr_block_update(code, int(X.shape[0]), int(X.shape[1]), int(Y.shape[1]), float(alpha),
                                  _ptr(X), _ld(X), _ptr(W), _ld(W), float(beta), _ptr(Y), _ld(Y), _stream()))


def arr_rcond_gram(X) -> float:
    rc = ctypes.c_double()
    _check(lib().arr_rcond_gram(_dtype_code(X), int(X.shape[0]), int(X.shape[1]), _ptr(X), _ld(X),
                                ctypes.addressof(rc), _stream()))
    return rc.value


def arr_orthonormalize(Z):
    _check(lib().arr_orthonormalize(int(Z.shape[0]), int(Z.shape[1]), _ptr(Z), _ld(Z), _stream()))


def arr_syev(H, evals, V):
    _check(lib().arr_syev(int(H.shape[0]), _ptr(H), _ptr(evals), _ptr(V), _stream()))


def arr_augmented_rr(A: DeviceCSR, X, p: int, Qc, Y) -> np.ndarray:
    w = int(X.shape[1])
    vals = np.zeros(w)
    nc = 0 if Qc is None else int(Qc.shape[1])
    _check(lib().arr_augmented_rr(ctypes.byref(A.desc), w, _ptr(X), _ld(X), int(p), _ptr(Qc), _ld(Qc), nc,
                                  _ptr(Y), _ld(Y), vals.ctypes.data, _stream()))
    return vals
