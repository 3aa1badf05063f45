"""Randomized HALS for nonnegative matrix factorisation on AMD MI355X.

Python binding of ``librnmf.so`` (C ABI in ``include/rnmf.h``).  This module
only marshals arguments: it allocates device memory through PyTorch, passes
raw device pointers and the current HIP stream to the library, and turns
status codes into exceptions.  Every step of the method runs in the library's
HIP kernels; if the library is missing this module raises instead of falling
back to anything else.

Method: Erichson, Mendible, Wihlborn, Kutz, "Randomized Nonnegative Matrix
Factorization", arXiv:1711.02037 (Sec. 2.3 randomized QB; Sec. 3.2 and
Algorithm 1 randomized HALS; Sec. 3.3 projected-gradient stop).
"""

import ctypes
import os

__all__ = [
    "RnmfError", "lib", "available", "make_opts", "sketch_width", "workspace_bytes",
    "sketch", "compress", "hals_step", "rel_error", "factorize", "cast_bf16",
    "status_string", "read_status", "hals", "svd_init", "Batch", "backward", "backward_workspace_bytes",
    "unrolled_forward", "unroll", "rand_hals_fn", "hals_ordered", "order_blocked", "order_interleaved",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librnmf.so")

# status codes (include/rnmf.h)
OK, ERR_ARG, ERR_SHAPE, ERR_DTYPE, ERR_WORKSPACE, ERR_NONFINITE, ERR_NEGATIVE_INPUT, \
    ERR_NOT_SPD, ERR_HIP, ERR_DEVICE_TIMEOUT, NOT_CONVERGED = range(11)
F64, F32, BF16 = 0, 1, 2
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
GRAM = {"full": 0, "lowdim": 1, "mixed": 2}
ORDER = {"h_first": 0, "w_first": 1}
OMEGA = {"gaussian": 0, "uniform": 1}
FLAG_CHECK_INPUT, FLAG_NO_SHIFT, FLAG_EXACT_Q, FLAG_TRACE, FLAG_SHIFTED_QR3 = 0x1, 0x2, 0x4, 0x8, 0x10
FLAG_SVD_INIT = 0x20
FLAG_GAUSS_INIT = 0x40
OP_SKETCH, OP_COMPRESS, OP_HALS_STEP, OP_FACTORIZE, OP_REL_ERROR, OP_HALS, OP_SVD_INIT = range(7)

EXPORTS = [
    "rnmf_default_opts", "rnmf_workspace_bytes", "rnmf_status_string", "rnmf_last_error",
    "rnmf_sketch_width", "rnmf_sketch", "rnmf_compress", "rnmf_hals_step", "rnmf_rel_error",
    "rnmf_factorize", "rnmf_cast_bf16", "rnmf_read_status", "rnmf_hals", "rnmf_svd_init",
    "rnmf_batch_workspace_bytes", "rnmf_batch_plan", "rnmf_batch_run", "rnmf_batch_results",
    "rnmf_batch_autotune", "rnmf_backward_workspace_bytes", "rnmf_backward", "rnmf_unroll",
    "rnmf_hals_ordered_workspace_bytes", "rnmf_hals_ordered", "rnmf_random", "rnmf_philox4x32_10",
    "rnmf_hals_step_noalloc", "rnmf_sweep_plan", "rnmf_batch_set_tuning", "rnmf_batch_get_tuning",
]


class Opts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("prec", ctypes.c_int32), ("omega_dist", ctypes.c_int32), ("gram_mode", ctypes.c_int32),
                ("order", ctypes.c_int32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32),
                ("alpha_w", ctypes.c_double), ("alpha_h", ctypes.c_double), ("beta_w", ctypes.c_double),
                ("beta_h", ctypes.c_double)]


class Problem(ctypes.Structure):
    """rnmf_problem: one problem of a batched run (device pointers)."""
    _fields_ = [("X", ctypes.c_void_p), ("Omega", ctypes.c_void_p), ("W0", ctypes.c_void_p),
                ("H0", ctypes.c_void_p), ("W", ctypes.c_void_p), ("H", ctypes.c_void_p),
                ("Q", ctypes.c_void_p), ("B", ctypes.c_void_p), ("Z", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("k", ctypes.c_int32), ("l", ctypes.c_int32), ("prec", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("l_eff", ctypes.c_int32), ("q_eff", ctypes.c_int32),
                ("qr_path", ctypes.c_int32), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rel_err", ctypes.c_double), ("pg_ratio", ctypes.c_double), ("ms_qb", ctypes.c_double),
                ("ms_sweeps", ctypes.c_double), ("ms_error", ctypes.c_double), ("comp_err", ctypes.c_double)]


class RnmfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"rnmf status {status} ({status_string(status)}): {message}")
        self.status = status


_lib = None


def lib():
    """The loaded librnmf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1711_02037_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.rnmf_hals_step_noalloc.argtypes = [vp, vp, i64, i64, i32, i32, vp, vp, vp, i32, ctypes.POINTER(Opts),
                                             vp, vp, vp]
        L.rnmf_hals_step_noalloc.restype = ctypes.c_int
        L.rnmf_sweep_plan.argtypes = [i64, i64, i32, i32, ctypes.POINTER(Opts), vp]
        L.rnmf_sweep_plan.restype = ctypes.c_int
        L.rnmf_random.argtypes = [vp, ctypes.c_int, i64, i64, ctypes.c_uint64, ctypes.c_uint32, i32, vp]
        L.rnmf_random.restype = ctypes.c_int
        L.rnmf_philox4x32_10.argtypes = [vp, vp, vp, i64, vp]
        L.rnmf_philox4x32_10.restype = ctypes.c_int
        L.rnmf_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.rnmf_default_opts.restype = None
        L.rnmf_workspace_bytes.argtypes = [ctypes.c_int, i64, i64, ctypes.POINTER(Opts)]
        L.rnmf_workspace_bytes.restype = sz
        L.rnmf_status_string.argtypes = [ctypes.c_int]
        L.rnmf_status_string.restype = ctypes.c_char_p
        L.rnmf_last_error.argtypes = []
        L.rnmf_last_error.restype = ctypes.c_char_p
        L.rnmf_sketch_width.argtypes = [i32, i32, i64, i64]
        L.rnmf_sketch_width.restype = i32
        L.rnmf_sketch.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, ctypes.POINTER(Opts), vp,
                                  ctypes.POINTER(i32), vp, sz, vp]
        L.rnmf_sketch.restype = ctypes.c_int
        L.rnmf_compress.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i32, ctypes.POINTER(Opts), vp,
                                    vp, sz, vp]
        L.rnmf_compress.restype = ctypes.c_int
        L.rnmf_hals_step.argtypes = [vp, vp, i64, i64, i32, i32, vp, vp, vp, i32, ctypes.POINTER(Opts),
                                     vp, vp, sz, vp]
        L.rnmf_hals_step.restype = ctypes.c_int
        L.rnmf_rel_error.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, vp, i32, ctypes.POINTER(Opts),
                                     vp, vp, sz, vp]
        L.rnmf_rel_error.restype = ctypes.c_int
        L.rnmf_factorize.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.POINTER(Opts), vp, vp, vp,
                                     vp, vp, ctypes.POINTER(Report), vp, sz, vp]
        L.rnmf_factorize.restype = ctypes.c_int
        L.rnmf_hals.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, vp, i32, ctypes.POINTER(Opts), vp, sz, vp]
        L.rnmf_hals.restype = ctypes.c_int
        L.rnmf_svd_init.argtypes = [vp, vp, i64, i64, i32, i32, vp, vp, ctypes.POINTER(Opts), vp, sz, vp]
        L.rnmf_svd_init.restype = ctypes.c_int
        L.rnmf_batch_workspace_bytes.argtypes = [i32]
        L.rnmf_batch_workspace_bytes.restype = sz
        L.rnmf_batch_plan.argtypes = [ctypes.POINTER(Problem), i32, vp, sz, vp]
        L.rnmf_batch_plan.restype = ctypes.c_int
        L.rnmf_batch_run.argtypes = [i32, i32, i32, vp, sz, vp]
        L.rnmf_batch_run.restype = ctypes.c_int
        L.rnmf_batch_results.argtypes = [i32, vp, sz, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), vp]
        L.rnmf_batch_results.restype = ctypes.c_int
        L.rnmf_batch_autotune.argtypes = [ctypes.POINTER(Problem), i32, i32, vp, sz, ctypes.POINTER(i32), vp]
        L.rnmf_batch_autotune.restype = ctypes.c_int
        L.rnmf_backward_workspace_bytes.argtypes = [i64, i64, i32, i32, i32, i32, ctypes.POINTER(Opts)]
        L.rnmf_backward_workspace_bytes.restype = sz
        L.rnmf_backward.argtypes = [vp, vp, i64, i64, i32, i32, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp,
                                    ctypes.POINTER(Opts), vp, sz, vp]
        L.rnmf_unroll.argtypes = [vp, vp, i64, i64, i32, i32, vp, vp, vp, i32, vp, ctypes.POINTER(Opts), vp, sz, vp]
        L.rnmf_hals_ordered_workspace_bytes.argtypes = [i64, i64, i32, i32]
        L.rnmf_hals_ordered_workspace_bytes.restype = sz
        L.rnmf_hals_ordered.argtypes = [vp, vp, i64, i64, i32, i32, vp, vp, vp, i32, ctypes.POINTER(i32),
                                        ctypes.POINTER(Opts), vp, sz, vp]
        L.rnmf_hals_ordered.restype = ctypes.c_int
        L.rnmf_unroll.restype = ctypes.c_int
        L.rnmf_backward.restype = ctypes.c_int
        L.rnmf_cast_bf16.argtypes = [vp, i64, i64, i64, vp, vp]
        L.rnmf_cast_bf16.restype = ctypes.c_int
        L.rnmf_read_status.argtypes = [vp, sz, vp]
        L.rnmf_read_status.restype = ctypes.c_int
        _lib = L
    return _lib


def available():
    try:
        lib()
        return True
    except (RuntimeError, OSError):
        return False


def status_string(s):
    return lib().rnmf_status_string(int(s)).decode()


def _check(status, allow=()):
    if status != OK and status not in allow:
        raise RnmfError(status, lib().rnmf_last_error().decode())
    return status


def make_opts(k, p=20, q=2, max_iter=200, tol=0.0, seed=0, precision="fp32", omega="gaussian",
              gram="full", order="h_first", check_input=True, shift=True, exact_q=False, reg=None):
    """rnmf_opts from keyword arguments.  reg: None or a mapping with any of
    alpha_w, alpha_h (ridge) and beta_w, beta_h (LASSO) weights (Sec. 3.4)."""
    o = Opts()
    lib().rnmf_default_opts(ctypes.byref(o))
    o.k, o.p, o.q, o.max_iter = int(k), int(p), int(q), int(max_iter)
    o.tol, o.seed = float(tol), int(seed) & 0xFFFFFFFFFFFFFFFF
    o.prec, o.omega_dist = PREC[precision], OMEGA[omega]
    o.gram_mode, o.order = GRAM[gram], ORDER[order]
    # shift: True = shifted pass only where a Gram is not positive definite,
    # False = never, "always" = shifted CholeskyQR3 for every QR
    o.flags = (FLAG_CHECK_INPUT if check_input else 0) | (0 if shift else FLAG_NO_SHIFT) | \
        (FLAG_SHIFTED_QR3 if shift == "always" else 0) | (FLAG_EXACT_Q if exact_q else 0)
    if reg:
        unknown = set(reg) - set(REG_KEYS)
        if unknown:
            raise ValueError(f"unknown regularization keys {sorted(unknown)}")
        for key in REG_KEYS:
            setattr(o, key, float(reg.get(key, 0.0)))
    return o


REG_KEYS = ("alpha_w", "alpha_h", "beta_w", "beta_h")


def sketch_width(k, p, m, n):
    return int(lib().rnmf_sketch_width(int(k), int(p), int(m), int(n)))


def workspace_bytes(op, m, n, opts):
    b = lib().rnmf_workspace_bytes(int(op), int(m), int(n), ctypes.byref(opts))
    if b == 0:
        raise RnmfError(ERR_ARG, lib().rnmf_last_error().decode())
    return int(b)


# ---------------------------------------------------------------------------
# torch marshalling
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _xt(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


def _fdtype(precision):
    torch = _torch()
    return torch.float64 if precision == "fp64" else torch.float32


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need_dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")


def _rowmajor(t, name):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D tensor with unit column stride")
    return t


def _packed(t, name):
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _workspace(nbytes, device):
    torch = _torch()
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf[off:off + nbytes]


def sketch(X, k, p=20, q=2, omega=None, precision="fp32", seed=0, omega_dist="gaussian", ws=None, **kw):
    """Orthonormal basis Q (m x l) of the range of X (rnmf_sketch)."""
    torch = _torch()
    _need_dev(X, "X"); _rowmajor(X, "X")
    m, n = X.shape
    o = make_opts(k, p, q, seed=seed, precision=precision, omega=omega_dist, **kw)
    l = sketch_width(k, p, m, n)
    dt = _fdtype(precision)
    if omega is not None:
        _packed(omega, "omega")
        if omega.shape != (n, l) or omega.dtype != dt:
            raise ValueError(f"omega must be {n} x {l} of {dt}")
    Q = torch.empty((m, l), dtype=dt, device=X.device)
    nb = workspace_bytes(OP_SKETCH, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, X.device)
    lo = ctypes.c_int32(0)
    _check(lib().rnmf_sketch(_ptr(X), _xt(X), m, n, X.stride(0), _ptr(omega), ctypes.byref(o), _ptr(Q),
                             ctypes.byref(lo), _ptr(w), w.numel(), _stream(X.device)))
    return Q


def compress(X, Q, precision="fp32", ws=None):
    """B = Q^T X (rnmf_compress)."""
    torch = _torch()
    _need_dev(X, "X"); _rowmajor(X, "X"); _packed(Q, "Q")
    m, n = X.shape
    l = Q.shape[1]
    if Q.shape[0] != m:
        raise ValueError("Q must have as many rows as X")
    o = make_opts(1, l - 1, 0, precision=precision)
    B = torch.empty((l, n), dtype=Q.dtype, device=X.device)
    nb = workspace_bytes(OP_COMPRESS, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, X.device)
    _check(lib().rnmf_compress(_ptr(X), _xt(X), m, n, X.stride(0), _ptr(Q), l, ctypes.byref(o), _ptr(B),
                               _ptr(w), w.numel(), _stream(X.device)))
    return B


def hals_step(Q, B, W, Wt, H, nsweeps=1, tol=0.0, gram="full", order="h_first", precision=None, ws=None,
              trace=False, reg=None):
    """nsweeps compressed HALS sweeps in place on W, Wt, H (rnmf_hals_step);
    reg: optional ridge / LASSO weights (see make_opts).
    Returns (sweeps done, pg^2 at entry, pg^2 at exit), plus the list of phase
    timestamps in microseconds when trace is set."""
    torch = _torch()
    for t, nm in ((Q, "Q"), (B, "B"), (W, "W"), (Wt, "Wt"), (H, "H")):
        _need_dev(t, nm); _packed(t, nm)
    m, l = Q.shape
    k, n = H.shape
    prec = precision or ("fp64" if Q.dtype == torch.float64 else "fp32")
    o = make_opts(k, l - k, 0, tol=tol, precision=prec, gram=gram, order=order, reg=reg)
    if trace:
        o.flags |= FLAG_TRACE
    nb = workspace_bytes(OP_HALS_STEP, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, Q.device)
    stats = torch.zeros(4, dtype=torch.float64, device=Q.device)
    _check(lib().rnmf_hals_step(_ptr(Q), _ptr(B), m, n, l, k, _ptr(W), _ptr(Wt), _ptr(H), int(nsweeps),
                                ctypes.byref(o), _ptr(stats), _ptr(w), w.numel(), _stream(Q.device)))
    s = stats.cpu().tolist()
    _check(lib().rnmf_read_status(_ptr(w), w.numel(), _stream(Q.device)))
    if trace:
        ts = w[1024:1024 + 8 * 128].cpu().view(torch.int64).tolist()
        t0 = ts[0]
        return int(s[0]), s[1], s[2], [(x - t0) / 100.0 if x else None for x in ts]
    return int(s[0]), s[1], s[2]


def sweep_plan(m, n, l, k, precision="fp32", tol=0.0):
    """Launch plan rnmf_hals_step would use for this shape on the current
    device (rnmf_sweep_plan): dict with the workgroup count, W rows and H
    columns per workgroup, the Q-slab path ("registers" or "lds"), whether
    the W rows stay in global memory, the exchange owners and the LDS bytes."""
    o = make_opts(k, l - k, 0, tol=tol, precision=precision)
    out = (ctypes.c_int32 * 8)()
    _check(lib().rnmf_sweep_plan(int(m), int(n), int(l), int(k), ctypes.byref(o), out))
    return dict(workgroups=out[0], rows_per=out[1], cols_per=out[2],
                q_slab="registers" if out[3] else "lds", w_global=bool(out[4]), owners=out[5],
                lds_bytes=out[6], q_rows_in_lds=out[7])


def hals_step_noalloc(Q, B, W, Wt, H, nsweeps=1, tol=0.0, gram="full", order="h_first", precision=None, reg=None):
    """hals_step through rnmf_hals_step_noalloc: the same sweeps with the
    library's fixed per-GPU scratch instead of a workspace (the library
    allocates nothing).  Returns (sweeps done, pg^2 at entry, pg^2 at exit,
    device status bits)."""
    torch = _torch()
    for t, nm in ((Q, "Q"), (B, "B"), (W, "W"), (Wt, "Wt"), (H, "H")):
        _need_dev(t, nm); _packed(t, nm)
    m, l = Q.shape
    k, n = H.shape
    prec = precision or ("fp64" if Q.dtype == torch.float64 else "fp32")
    o = make_opts(k, l - k, 0, tol=tol, precision=prec, gram=gram, order=order, reg=reg)
    stats = torch.zeros(4, dtype=torch.float64, device=Q.device)
    status = torch.zeros(1, dtype=torch.int32, device=Q.device)
    _check(lib().rnmf_hals_step_noalloc(_ptr(Q), _ptr(B), m, n, l, k, _ptr(W), _ptr(Wt), _ptr(H), int(nsweeps),
                                        ctypes.byref(o), _ptr(stats), _ptr(status), _stream(Q.device)))
    s = stats.cpu().tolist()
    return int(s[0]), s[1], s[2], int(status.cpu().item())


def hals(X, W, H, nsweeps=1, order="h_first", ws=None, reg=None):
    """nsweeps sweeps of deterministic HALS on X itself, in place on W and H
    (rnmf_hals; Sec. 3.1, regularized form of Sec. 3.4 when reg is given).
    X, W, H: FP32 or FP64 (all the same dtype)."""
    torch = _torch()
    _need_dev(X, "X"); _rowmajor(X, "X")
    for t, nm in ((W, "W"), (H, "H")):
        _need_dev(t, nm); _packed(t, nm)
    m, n = X.shape
    k = H.shape[0]
    if W.shape != (m, k) or H.shape != (k, n) or W.dtype != X.dtype or H.dtype != X.dtype:
        raise ValueError("need W (m x k) and H (k x n) in the dtype of X")
    prec = "fp64" if X.dtype == torch.float64 else "fp32"
    o = make_opts(k, 0, 0, precision=prec, order=order, reg=reg)
    nb = workspace_bytes(OP_HALS, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, X.device)
    _check(lib().rnmf_hals(_ptr(X), _xt(X), m, n, X.stride(0), _ptr(W), _ptr(H), int(nsweeps), ctypes.byref(o),
                           _ptr(w), w.numel(), _stream(X.device)))
    _check(lib().rnmf_read_status(_ptr(w), w.numel(), _stream(X.device)))


def order_blocked(k, w_first=False):
    """One sweep's block list for a blocked order: rows of H then columns of
    W (Algorithm 1), or columns of W first.  Entry e < k is column e of W,
    entry e >= k is row e - k of H."""
    w = list(range(k))
    h = [k + j for j in range(k)]
    return w + h if w_first else h + w


def order_interleaved(k, perm=None):
    """One sweep's block list for the interleaved order W(:,j) -> H(j,:) with
    j = perm[0], perm[1], ... (0..k-1 by default; a random perm gives the
    shuffled order)."""
    perm = range(k) if perm is None else perm
    out = []
    for j in perm:
        out += [int(j), k + int(j)]
    return out


def hals_ordered(Q, B, W, Wt, H, orders, ws=None):
    """Compressed HALS sweeps with explicit block orders, in place on W, Wt,
    H (rnmf_hals_ordered): `orders` holds one list per sweep, each a
    permutation of 0..2k-1 (see order_blocked, order_interleaved)."""
    import numpy as np
    torch = _torch()
    for t, nm in ((Q, "Q"), (B, "B"), (W, "W"), (Wt, "Wt"), (H, "H")):
        _need_dev(t, nm); _packed(t, nm)
    m, l = Q.shape
    k, n = H.shape
    arr = np.ascontiguousarray(np.asarray(orders, dtype=np.int32).reshape(-1, 2 * k))
    prec = "fp64" if Q.dtype == torch.float64 else "fp32"
    o = make_opts(k, l - k, 0, precision=prec)
    nb = lib().rnmf_hals_ordered_workspace_bytes(m, n, l, k)
    if nb == 0:
        raise RnmfError(ERR_ARG, lib().rnmf_last_error().decode())
    keep, w = ws if ws is not None else _workspace(nb, Q.device)
    _check(lib().rnmf_hals_ordered(_ptr(Q), _ptr(B), m, n, l, k, _ptr(W), _ptr(Wt), _ptr(H), arr.shape[0],
                                   arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(o), _ptr(w),
                                   w.numel(), _stream(Q.device)))
    _check(lib().rnmf_read_status(_ptr(w), w.numel(), _stream(Q.device)))


def svd_init(Q, B, k, ws=None):
    """W0 (m x k) and H0 (k x n) by the SVD-based initialization
    (rnmf_svd_init: nonnegative double SVD of the randomized SVD Q B)."""
    torch = _torch()
    for t, nm in ((Q, "Q"), (B, "B")):
        _need_dev(t, nm); _packed(t, nm)
    m, l = Q.shape
    n = B.shape[1]
    if B.shape[0] != l or B.dtype != Q.dtype:
        raise ValueError("need B (l x n) in the dtype of Q")
    prec = "fp64" if Q.dtype == torch.float64 else "fp32"
    o = make_opts(k, l - k, 0, precision=prec)
    nb = workspace_bytes(OP_SVD_INIT, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, Q.device)
    W = torch.empty((m, k), dtype=Q.dtype, device=Q.device)
    H = torch.empty((k, n), dtype=Q.dtype, device=Q.device)
    _check(lib().rnmf_svd_init(_ptr(Q), _ptr(B), m, n, l, int(k), _ptr(W), _ptr(H), ctypes.byref(o), _ptr(w),
                               w.numel(), _stream(Q.device)))
    return W, H


def backward_workspace_bytes(m, n, l, k, T, ckpt_every, precision="fp32"):
    o = make_opts(k, l - k, 0, precision=precision)
    b = lib().rnmf_backward_workspace_bytes(int(m), int(n), int(l), int(k), int(T), int(ckpt_every),
                                            ctypes.byref(o))
    if b == 0:
        raise RnmfError(ERR_ARG, lib().rnmf_last_error().decode())
    return int(b)


def backward(Q, B, W0, Wt0, H0, T, gW, gH, ckpt_every=None, states=None, want_gX=False, ws=None):
    """Gradients through T unrolled compressed sweeps with Q fixed
    (rnmf_backward).  Q, B, W0, Wt0, H0 in the factor dtype (FP32 or FP64),
    gW (m x k) and gH (k x n) FP64: the upstream gradients of (W_T, H_T).
    With `states` (the record of unroll) nothing is recomputed; otherwise the
    forward is recomputed from checkpoints every `ckpt_every` sweeps (default
    T: all states of one pass kept).  Returns FP64 (gB, gW0, gH0, gX), gX =
    Q gB or None."""
    torch = _torch()
    for t, nm in ((Q, "Q"), (B, "B"), (W0, "W0"), (Wt0, "Wt0"), (H0, "H0"), (gW, "gW"), (gH, "gH")):
        _need_dev(t, nm); _packed(t, nm)
    m, l = Q.shape
    k, n = H0.shape
    if B.shape != (l, n) or W0.shape != (m, k) or Wt0.shape != (l, k):
        raise ValueError("need B (l x n), W0 (m x k), Wt0 (l x k) for Q (m x l), H0 (k x n)")
    for t, nm in ((B, "B"), (W0, "W0"), (Wt0, "Wt0"), (H0, "H0")):
        if t.dtype != Q.dtype:
            raise ValueError(f"{nm} must have the dtype of Q")
    if gW.shape != (m, k) or gH.shape != (k, n) or gW.dtype != torch.float64 or gH.dtype != torch.float64:
        raise ValueError("gW (m x k) and gH (k x n) must be float64")
    if states is not None:
        _need_dev(states, "states"); _packed(states, "states")
        if states.dtype != Q.dtype or states.numel() < int(T) * (m * k + l * k + k * n):
            raise ValueError("states must hold T recorded states in the dtype of Q")
        ckpt = 0
    else:
        ckpt = int(ckpt_every) if ckpt_every else max(1, int(T))
    prec = "fp64" if Q.dtype == torch.float64 else "fp32"
    o = make_opts(k, l - k, 0, precision=prec)
    nb = backward_workspace_bytes(m, n, l, k, T, ckpt, prec)
    keep, w = ws if ws is not None else _workspace(nb, Q.device)
    dev = Q.device
    gB = torch.empty((l, n), dtype=torch.float64, device=dev)
    gW0 = torch.empty((m, k), dtype=torch.float64, device=dev)
    gH0 = torch.empty((k, n), dtype=torch.float64, device=dev)
    gX = torch.empty((m, n), dtype=torch.float64, device=dev) if want_gX else None
    _check(lib().rnmf_backward(_ptr(Q), _ptr(B), m, n, l, k, _ptr(W0), _ptr(Wt0), _ptr(H0), int(T), ckpt,
                               _ptr(states), _ptr(gW), _ptr(gH), _ptr(gB), _ptr(gW0), _ptr(gH0), _ptr(gX),
                               ctypes.byref(o), _ptr(w), w.numel(), _stream(dev)))
    _check(lib().rnmf_read_status(_ptr(w), w.numel(), _stream(dev)))
    return gB, gW0, gH0, gX


def state_elems(m, n, l, k):
    """Elements of one recorded state: W (m x k), Wt (l x k), H (k x n)."""
    return m * k + l * k + k * n


def unroll(Q, B, W, Wt, H, T, record=True, ws=None):
    """T sweeps, one launch each, in place on W, Wt, H (rnmf_unroll).  With
    `record`, returns the T states after each sweep in one flat tensor of the
    factor dtype (the layout rnmf_backward reads), else None."""
    torch = _torch()
    for t, nm in ((Q, "Q"), (B, "B"), (W, "W"), (Wt, "Wt"), (H, "H")):
        _need_dev(t, nm); _packed(t, nm)
    m, l = Q.shape
    k, n = H.shape
    prec = "fp64" if Q.dtype == torch.float64 else "fp32"
    o = make_opts(k, l - k, 0, precision=prec)
    nb = workspace_bytes(OP_HALS_STEP, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, Q.device)
    states = (torch.empty(max(1, int(T)) * state_elems(m, n, l, k), dtype=Q.dtype, device=Q.device)
              if record else None)
    _check(lib().rnmf_unroll(_ptr(Q), _ptr(B), m, n, l, k, _ptr(W), _ptr(Wt), _ptr(H), int(T), _ptr(states),
                             ctypes.byref(o), _ptr(w), w.numel(), _stream(Q.device)))
    _check(lib().rnmf_read_status(_ptr(w), w.numel(), _stream(Q.device)))
    return states


def unrolled_forward(Q, B, W0, Wt0, H0, T, ws=None):
    """(W_T, Wt_T, H_T) after T compressed sweeps from copies of (W0, Wt0, H0),
    one sweep per launch: the states rnmf_backward reads or recomputes."""
    W, Wt, H = W0.clone(), Wt0.clone(), H0.clone()
    unroll(Q, B, W, Wt, H, T, record=False, ws=ws)
    return W, Wt, H


def _make_autograd():
    torch = _torch()

    class RandHALS(torch.autograd.Function):
        """(W_T, H_T) = T compressed HALS sweeps from (W0, H0) on B = Q^T X with
        the basis Q held fixed (no gradient flows into Q).  Both passes run in
        librnmf: the forward through rnmf_compress and rnmf_unroll, the
        backward through rnmf_backward.
        Call as RandHALS.apply(X, Q, W0, H0, T, ckpt_every): with ckpt_every
        None the forward records all T states (rnmf_unroll) and the backward
        reads them; with a number it records nothing and the backward
        recomputes from checkpoints."""

        @staticmethod
        def forward(ctx, X, Q, W0, H0, T, ckpt_every=None):
            Q = Q.contiguous()
            prec = "fp64" if Q.dtype == torch.float64 else "fp32"
            B = compress(X, Q, precision=prec)
            W0c = W0.detach().to(Q.dtype).contiguous()
            H0c = H0.detach().to(Q.dtype).contiguous()
            Wt0 = compress(W0c, Q, precision=prec)
            W, Wt, H = W0c.clone(), Wt0.clone(), H0c.clone()
            # without ckpt_every every state is recorded and the backward
            # recomputes nothing; with it, nothing is recorded
            states = unroll(Q, B, W, Wt, H, T, record=ckpt_every is None)
            ctx.save_for_backward(Q, B, W0c, Wt0, H0c, states)
            ctx.T, ctx.ckpt = int(T), ckpt_every
            ctx.dtypes = (X.dtype, W0.dtype, H0.dtype)
            return W, H

        @staticmethod
        def backward(ctx, gW, gH):
            Q, B, W0, Wt0, H0, states = ctx.saved_tensors
            m, k = W0.shape
            n = H0.shape[1]
            gW = (torch.zeros((m, k), dtype=torch.float64, device=Q.device) if gW is None
                  else gW.to(torch.float64).contiguous())
            gH = (torch.zeros((k, n), dtype=torch.float64, device=Q.device) if gH is None
                  else gH.to(torch.float64).contiguous())
            want_x = ctx.needs_input_grad[0]
            gB, gW0, gH0, gX = backward(Q, B, W0, Wt0, H0, ctx.T, gW, gH, ctx.ckpt, states=states, want_gX=want_x)
            xd, wd, hd = ctx.dtypes
            return (gX.to(xd) if want_x else None, None, gW0.to(wd), gH0.to(hd), None, None)

    return RandHALS


_rand_hals = None


def rand_hals_fn():
    """The torch.autograd.Function over T unrolled sweeps (see RandHALS)."""
    global _rand_hals
    if _rand_hals is None:
        _rand_hals = _make_autograd()
    return _rand_hals


def batch_tuning(table=None):
    """The batch autotune table (8 ints: X-pass column groups for l <= 16,
    32, 48, 64, then the H-phase tile widths); with table given, set it first
    (rnmf_batch_set_tuning).  Returns the table now in force."""
    if table is not None:
        t = (ctypes.c_int32 * 8)(*[int(x) for x in table])
        _check(lib().rnmf_batch_set_tuning(t))
    out = (ctypes.c_int32 * 8)()
    _check(lib().rnmf_batch_get_tuning(out))
    return list(out)


class Batch:
    """Batched randomized HALS (rnmf_batch_*): many independent problems in one
    persistent launch.  problems: list of (X, Omega, W0, H0) FP32 device
    tensors (X m x n with unit column stride, Omega n x l, W0 m x k, H0 k x n).
    precision: "fp32" (FP32 arithmetic) or "bf16" (X passes on bf16 matrix
    cores from the FP32 X, one more subspace iteration).
    Holds the outputs W, H, Q, B of every problem and the workspace."""

    def __init__(self, problems, autotune=False, q=2, precision="fp32"):
        if precision not in ("fp32", "bf16"):
            raise ValueError("precision must be 'fp32' or 'bf16'")
        torch = _torch()
        self.problems = []
        descs = (Problem * len(problems))()
        for i, (X, Om, W0, H0) in enumerate(problems):
            for t, nm in ((X, "X"), (Om, "Omega"), (W0, "W0"), (H0, "H0")):
                _need_dev(t, nm)
                if t.dtype != torch.float32:
                    raise ValueError(f"problem {i}: {nm} must be float32")
            _rowmajor(X, "X")
            for t, nm in ((Om, "Omega"), (W0, "W0"), (H0, "H0")):
                _packed(t, nm)
            m, n = X.shape
            l = Om.shape[1]
            k = W0.shape[1]
            if Om.shape[0] != n or W0.shape[0] != m or H0.shape != (k, n):
                raise ValueError(f"problem {i}: inconsistent shapes")
            dev = X.device
            out = dict(X=X, Omega=Om, W0=W0, H0=H0,
                       W=torch.empty((m, k), dtype=torch.float32, device=dev),
                       H=torch.empty((k, n), dtype=torch.float32, device=dev),
                       Q=torch.empty((m, l), dtype=torch.float32, device=dev),
                       B=torch.empty((l, n), dtype=torch.float32, device=dev),
                       Z=torch.empty(n * l + k * ((m + 31) // 32) * 32 + 32, dtype=torch.float32,
                                     device=dev))
            self.problems.append(out)
            d = descs[i]
            for key in ("X", "Omega", "W0", "H0", "W", "H", "Q", "B", "Z"):
                setattr(d, key, out[key].data_ptr())
            d.m, d.n, d.ldx, d.k, d.l = m, n, X.stride(0), k, l
            d.prec = PREC[precision]
        self.descs = descs
        self.n = len(problems)
        self.device = problems[0][0].device
        nb = lib().rnmf_batch_workspace_bytes(self.n)
        if nb == 0:
            raise RnmfError(ERR_ARG, lib().rnmf_last_error().decode())
        self.keep, self.ws = _workspace(nb, self.device)
        self.tiling = None
        if autotune:
            tab = (ctypes.c_int32 * 8)()
            _check(lib().rnmf_batch_autotune(descs, self.n, int(q), _ptr(self.ws), self.ws.numel(), tab,
                                             _stream(self.device)))
            self.tiling = list(tab)
        else:
            _check(lib().rnmf_batch_plan(descs, self.n, _ptr(self.ws), self.ws.numel(), _stream(self.device)))

    def run(self, q=2, nsweeps=100):
        """One persistent launch (plus a counter reset); asynchronous."""
        _check(lib().rnmf_batch_run(self.n, int(q), int(nsweeps), _ptr(self.ws), self.ws.numel(),
                                    _stream(self.device)))

    def results(self):
        """(rel_err list, status list) of the last run; synchronises."""
        rel = (ctypes.c_double * self.n)()
        st = (ctypes.c_int32 * self.n)()
        _check(lib().rnmf_batch_results(self.n, _ptr(self.ws), self.ws.numel(), rel, st, _stream(self.device)))
        return list(rel), list(st)

    def capture(self, q=2, nsweeps=100):
        """A HIP graph (torch.cuda.CUDAGraph) holding one run; replay() reruns it."""
        torch = _torch()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.run(q, nsweeps)  # warm-up outside the graph sets the kernel attribute
        torch.cuda.current_stream(self.device).wait_stream(s)
        torch.cuda.synchronize(self.device)
        with torch.cuda.graph(g):
            self.run(q, nsweeps)
        return g


def rel_error(X, W, H, ws=None):
    """||X - W H||_F / ||X||_F with FP64 accumulation (rnmf_rel_error)."""
    torch = _torch()
    _need_dev(X, "X"); _rowmajor(X, "X")
    m, n = X.shape
    k = W.shape[1]
    prec = "fp64" if W.dtype == torch.float64 else ("bf16" if X.dtype == torch.bfloat16 else "fp32")
    o = make_opts(1, 0, 0, precision=prec)
    nb = workspace_bytes(OP_REL_ERROR, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, X.device)
    out = torch.zeros(2, dtype=torch.float64, device=X.device)
    _check(lib().rnmf_rel_error(_ptr(X), _xt(X), m, n, X.stride(0), _ptr(W), _ptr(H), k, ctypes.byref(o),
                                _ptr(out), _ptr(w), w.numel(), _stream(X.device)))
    se, sx = out.cpu().tolist()
    return (se / sx) ** 0.5 if sx > 0 else 0.0


def factorize(X, k, p=20, q=2, max_iter=200, tol=0.0, precision="fp32", seed=0, omega=None, W0=None,
              H0=None, gram="full", order="h_first", omega_dist="gaussian", check_input=True, shift=True,
              exact_q=False, ws=None, reg=None, init="random"):
    """Algorithm 1 end to end (rnmf_factorize).  Returns (W, H, report dict).
    reg: optional ridge / LASSO weights (Sec. 3.4; see make_opts).
    init: "random" (W0, H0 given or uniform from seed), "gauss" (W0, H0
    given or standard normal from seed with the negative entries set to zero)
    or "svd" (the SVD-based initialization on this run's Q and B)."""
    torch = _torch()
    _need_dev(X, "X"); _rowmajor(X, "X")
    m, n = X.shape
    o = make_opts(k, p, q, max_iter, tol, seed, precision, omega_dist, gram, order, check_input, shift,
                  exact_q, reg)
    if init == "svd":
        o.flags |= FLAG_SVD_INIT
    elif init == "gauss":
        o.flags |= FLAG_GAUSS_INIT
    elif init != "random":
        raise ValueError("init must be 'random', 'gauss' or 'svd'")
    dt = _fdtype(precision)
    for t, nm in ((omega, "omega"), (W0, "W0"), (H0, "H0")):
        if t is not None:
            _need_dev(t, nm); _packed(t, nm)
            if t.dtype != dt:
                raise ValueError(f"{nm} must be {dt}")
    W = torch.empty((m, k), dtype=dt, device=X.device)
    H = torch.empty((k, n), dtype=dt, device=X.device)
    nb = workspace_bytes(OP_FACTORIZE, m, n, o)
    keep, w = ws if ws is not None else _workspace(nb, X.device)
    rep = Report()
    st = lib().rnmf_factorize(_ptr(X), _xt(X), m, n, X.stride(0), ctypes.byref(o), _ptr(omega), _ptr(W0),
                              _ptr(H0), _ptr(W), _ptr(H), ctypes.byref(rep), _ptr(w), w.numel(),
                              _stream(X.device))
    _check(st, allow=(NOT_CONVERGED,))
    info = dict(iters=rep.iters, l=rep.l_eff, q=rep.q_eff, shifted_qr=bool(rep.qr_path & 1),
                status=rep.status, rel_err=rep.rel_err, pg_ratio=rep.pg_ratio, ms_qb=rep.ms_qb,
                ms_sweeps=rep.ms_sweeps, ms_error=rep.ms_error, comp_err=rep.comp_err)
    return W, H, info


def cast_bf16(X):
    """Packed bfloat16 copy of an FP32 matrix, round to nearest even (rnmf_cast_bf16)."""
    torch = _torch()
    _need_dev(X, "X"); _rowmajor(X, "X")
    m, n = X.shape
    Xb = torch.empty((m, n), dtype=torch.bfloat16, device=X.device)
    _check(lib().rnmf_cast_bf16(_ptr(X), m, n, X.stride(0), _ptr(Xb), _stream(X.device)))
    return Xb


DISTS = {"gaussian": 0, "uniform": 1, "gauss_clipped": 2}


def random(rows, cols, seed, stream_id, dist="gaussian", dtype=None, device="cuda:0"):
    """The library's seeded random matrix (rnmf_random): rows x cols, FP32 by
    default; stream ids 3, 4, 5 are the ones rnmf_factorize uses for Omega,
    W0 and H0."""
    torch = _torch()
    dt = dtype or torch.float32
    if dt not in (torch.float32, torch.float64):
        raise ValueError("dtype must be float32 or float64")
    out = torch.empty((rows, cols), dtype=dt, device=device)
    _check(lib().rnmf_random(_ptr(out), 0 if dt == torch.float64 else 1, rows, cols, int(seed) & (2**64 - 1),
                             int(stream_id), DISTS[dist], _stream(out.device)))
    return out


def philox4x32_10(ctr, key):
    """The Philox4x32-10 block function (rnmf_philox4x32_10) on device int32
    tensors ctr (count x 4) and key (count x 2); returns count x 4 words
    (int32 storage of the unsigned words)."""
    torch = _torch()
    _need_dev(ctr, "ctr"); _need_dev(key, "key")
    if ctr.dtype != torch.int32 or key.dtype != torch.int32:
        raise ValueError("ctr and key must be int32 tensors")
    if ctr.dim() != 2 or ctr.shape[1] != 4 or key.shape != (ctr.shape[0], 2):
        raise ValueError("ctr must be count x 4 and key count x 2")
    ctr, key = ctr.contiguous(), key.contiguous()
    out = torch.empty_like(ctr)
    _check(lib().rnmf_philox4x32_10(_ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0], _stream(ctr.device)))
    return out


def read_status(ws):
    return _check(lib().rnmf_read_status(_ptr(ws), ws.numel(), None))
