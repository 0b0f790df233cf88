"""MI355X-native Gaussian kernel ridge regression (arXiv 1905.10587) — Python binding.

This module only marshals arguments into the C ABI of ``libkrr.so`` (declared in
include/krr.h): it converts torch tensors to contiguous FP64 device buffers,
passes their pointers and torch's current HIP stream, and routes the library's
device allocations through PyTorch's caching allocator.  Every step of the solver
runs in the library's HIP kernels; there is no CPU or eager-PyTorch fallback: if
the library is not built, every call raises.

Entry points (names follow the C ABI):
  kernel_mv      K(Xt, Xs) V, optionally + shift*V, K' = (D^2/eps) K       (Sec. 2.4, computed exactly)
  sketch         Algorithm 1 / Algorithm 2 sketch Y                          (Sec. 3)
  qrcp           pivoted QR of Y^T: anchors and |R_jj|                       (Sec. 3)
  Preconditioner ID / Nystrom / Woodbury preconditioner (Algorithms 1-4), .apply()
  pcg_solve      Algorithm 5 for a block of right-hand sides
  grad           validation-loss gradient w.r.t. log eps and log beta (adjoint)
  KRRValLoss     torch.autograd.Function wrapping grad
  autotune       kernel-variant search
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

__all__ = ["load", "KRRError", "kernel_mv", "sketch", "qrcp", "Preconditioner", "pcg_solve", "grad",
           "KRRValLoss", "autotune", "autotune_save", "autotune_load", "set_variant", "num_variants", "kmv_variant",
           "kmv_last_launch", "set_cull", "cull_stats", "set_pcg_mode", "radix_sort_pairs", "fps", "rank_for_cond",
           "PREC", "library_path"]

PREC = {"fp64": 0, "fp32": 1, "mixed": 2}
_STATUS = {0: "KRR_OK", -1: "KRR_EINVAL", -2: "KRR_ENOMEM", -3: "KRR_EHIP", -4: "KRR_ENOTSPD",
           -5: "KRR_EBREAKDOWN", 1: "KRR_ENOCONV"}
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_CALLBACKS = None


def library_path() -> str:
    return os.path.join(_HERE, "libkrr.so")


class KRRError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class SolveStats(ctypes.Structure):
    _fields_ = [("iters_max", ctypes.c_int32), ("n_mvm", ctypes.c_int32), ("n_mvm_fp64", ctypes.c_int32),
                ("n_replace", ctypes.c_int32), ("t_total_ms", ctypes.c_double), ("t_mvm_ms", ctypes.c_double),
                ("t_mvm_fp64_ms", ctypes.c_double), ("t_precond_ms", ctypes.c_double),
                ("kappa_est", ctypes.c_double), ("t_mvm_kernel_ms", ctypes.c_double),
                ("lam_min_est", ctypes.c_double), ("lam_max_est", ctypes.c_double),
                ("n_graph_cycles", ctypes.c_int32), ("n_graph_iters", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _i64, _i32, _f64, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "krr_version": ([], _i32),
    "krr_init": ([_vp], _i32),
    "krr_last_error": ([], ctypes.c_char_p),
    "krr_set_allocator": ([_vp, _vp, _vp], _i32),
    "krr_kernel_mv": ([_vp, _i64, _vp, _i64, _i32, _f64, _vp, _i32, _vp, _i32, _i32, _vp, _vp], _i32),
    "krr_sketch": ([_vp, _i64, _i32, _f64, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp], _i32),
    "krr_qrcp": ([_vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp], _i32),
    "krr_build_precond": ([_vp, _i64, _i32, _f64, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _f64, _i32, _i32,
                           ctypes.POINTER(_vp), _vp], _i32),
    "krr_build_precond_anchors": ([_vp, _i64, _i32, _f64, _vp, _i32, _vp, _i32, _i64, _f64, _i32,
                                   ctypes.POINTER(_vp), _vp], _i32),
    "krr_fps": ([_vp, _i64, _i32, _i32, _i64, _vp, _vp, _vp], _i32),
    "krr_radix_sort_pairs": ([_vp, _vp, _vp, _vp, _i64, _i32, _vp], _i32),
    "krr_rank_for_cond": ([_vp, _i64, _i32, _f64, _f64, _f64, _f64, _vp, _vp, _vp, _vp], _i32),
    "krr_precond_info": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "krr_precond_get": ([_vp, _i32, _i32, _vp, _sz, _vp], _i32),
    "krr_precond_timings": ([_vp, _vp, _vp], _i32),
    "krr_precond_apply": ([_vp, _vp, _i32, _vp, _i32, _vp, _vp], _i32),
    "krr_precond_apply_noalloc": ([_vp, _vp, _i32, _vp, _i32, _vp, _vp], _i32),
    "krr_precond_free": ([_vp], None),
    "krr_pcg_solve": ([_vp, _i64, _i32, _f64, _vp, _i32, _vp, _vp, _f64, _i32, _i32, _i32, _vp, _vp, _vp, _vp,
                       _i32, _vp], _i32),
    "krr_grad": ([_vp, _i64, _vp, _vp, _i64, _vp, _i32, _f64, _f64, _vp, _f64, _i32, _i32, _i32, _vp, _vp, _vp,
                  _vp, _vp, _vp, _vp], _i32),
    "krr_autotune": ([_i32, _i32, _i32, _i64, _vp, _vp], _i32),
    "krr_autotune_save": ([ctypes.c_char_p], _i32),
    "krr_autotune_load": ([ctypes.c_char_p], _i32),
    "krr_set_variant": ([_i32, _i32, _i32, _i32], _i32),
    "krr_num_variants": ([_i32, _i32], _i32),
    "krr_kmv_variant": ([_i32, _i32, _i32, _i32, _i32, _i64, _vp, _vp], _i32),
    "krr_kmv_last_launch": ([_vp, _vp, _vp], _i32),
    "krr_set_cull": ([_i32], _i32),
    "krr_set_pcg_mode": ([_i32], _i32),
    "krr_cull_stats": ([_vp, _vp, _vp], _i32),
}


def _alloc_cb(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(max(int(nbytes), 1), torch.cuda.current_device(),
                                                  int(stream or 0))
    except Exception:   # out of memory: the library reports KRR_ENOMEM
        return None


def _free_cb(ptr, ctx):
    torch.cuda.caching_allocator_delete(int(ptr))


def load():
    """Load libkrr.so (raises if it is not built) and register torch's caching allocator."""
    global _LIB, _CALLBACKS
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1905_10587_amd.build` "
                           "(the solver has no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if torch.cuda.is_available():
        ALLOC = ctypes.CFUNCTYPE(_vp, _sz, _vp, _vp)
        FREE = ctypes.CFUNCTYPE(None, _vp, _vp)
        _CALLBACKS = (ALLOC(_alloc_cb), FREE(_free_cb))
        _chk(lib, lib.krr_set_allocator(ctypes.cast(_CALLBACKS[0], _vp), ctypes.cast(_CALLBACKS[1], _vp), None))
        _chk(lib, lib.krr_init(_stream()))
    _LIB = lib
    return lib


def _chk(lib, status):
    if status < 0:
        raise KRRError(status, lib.krr_last_error().decode())
    return status


def _tensor(t):
    return t if isinstance(t, torch.Tensor) else torch.as_tensor(t)


def _need(cond, msg):
    """Shape checks of the binding: the C ABI takes plain pointers and sizes and cannot see a buffer's extent,
    so a mismatched shape would make the library read or write past it."""
    if not cond:
        raise ValueError(msg)


def _points(X, name="X", d=None):
    X = _tensor(X)
    _need(X.dim() == 2 and X.shape[0] >= 1 and X.shape[1] >= 1, f"{name} must be a non-empty n x d matrix")
    _need(d is None or X.shape[1] == d, f"{name} has {X.shape[1]} columns, expected d = {d}")
    return X


def _rows(V, n, name):
    V = _tensor(V)
    _need(V.dim() in (1, 2) and V.shape[0] == n, f"{name} must have {n} rows (got shape {tuple(V.shape)})")
    return V


def _betas(betas, R):
    betas = [float(betas)] * R if isinstance(betas, (int, float)) else [float(b) for b in betas]
    _need(len(betas) == R, f"{R} columns need {R} betas (got {len(betas)})")
    return betas


def _dev(t, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    if not t.is_cuda:
        t = t.to("cuda")
    return t.to(dtype).contiguous()


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host_f64(vals):
    vals = [float(v) for v in vals]
    return (ctypes.c_double * len(vals))(*vals), len(vals)


def _prec(prec):
    return PREC[prec] if isinstance(prec, str) else int(prec)


# ---------------------------------------------------------------------------------------------
def kernel_mv(Xt, Xs, eps: float, V, shift=None, deriv: int = 0, prec="fp64"):
    """U = K(Xt, Xs) V (+ shift * V); deriv=1: K' V, deriv=2: [K V, K' V] (m x 2R)."""
    lib = load()
    Xt = _points(Xt, "Xt")
    Xs = None if Xs is None else _points(Xs, "Xs", Xt.shape[1])
    V = _rows(V, Xt.shape[0] if Xs is None else Xs.shape[0], "V")
    shift = None if shift is None else _betas(shift, 1 if V.dim() == 1 else V.shape[1])
    Xt, Xs = _dev(Xt), (None if Xs is None else _dev(Xs))
    same = Xs is None
    if same:
        Xs = Xt
    V = _dev(V)
    vec = V.dim() == 1
    V2 = V.reshape(V.shape[0], -1)
    m, d = Xt.shape
    n = Xs.shape[0]
    R = V2.shape[1]
    cols = 2 * R if deriv == 2 else R
    U = torch.empty((m, cols), dtype=torch.float64, device=Xt.device)
    sh = None
    if shift is not None:
        sh, _ = _host_f64(shift)
    _chk(lib, lib.krr_kernel_mv(_p(Xt), m, _p(Xs), n, d, float(eps), _p(V2), R, sh, deriv, _prec(prec), _p(U),
                                _stream()))
    if vec and deriv != 2:
        return U[:, 0]
    return U


def sketch(X, eps: float, omega=None, idx=None, sign=None, prec="fp64"):
    """Algorithm 1 (omega: n x l Gaussian) or Algorithm 2 (idx/sign: l x r) sketch Y (n x l)."""
    lib = load()
    X = _points(X)
    n, d = X.shape
    _check_draws(n, omega, idx, sign)
    X = _dev(X)
    if omega is not None:
        omega = _dev(omega)
        l, r = omega.shape[1], 0
    else:
        idx, sign = _dev(idx, torch.int64), _dev(sign)
        l, r = idx.shape
    Y = torch.empty((n, l), dtype=torch.float64, device=X.device)
    _chk(lib, lib.krr_sketch(_p(X), n, d, float(eps), _p(omega), _p(idx), _p(sign), l, r, _prec(prec), _p(Y),
                             _stream()))
    return Y


def _check_draws(n, omega, idx, sign, l=None):
    """Shapes of the sketch randomness: omega n x l, or idx and sign both l x r."""
    if omega is not None:
        omega = _tensor(omega)
        _need(omega.dim() == 2 and omega.shape[0] == n, f"omega must be n x l with n = {n}")
        _need(l is None or omega.shape[1] == l, f"omega must have l = {l} columns")
        return
    _need(idx is not None and sign is not None, "give omega, or idx and sign")
    idx, sign = _tensor(idx), _tensor(sign)
    _need(idx.dim() == 2 and tuple(sign.shape) == tuple(idx.shape), "idx and sign must both be l x r")
    _need(l is None or idx.shape[0] == l, f"idx and sign must have l = {l} rows")


def qrcp(Y, k: int, prec="fp64"):
    """First k pivots of the column-pivoted QR of Y^T (Y is n x l). Returns (piv int64 k, rdiag k)."""
    lib = load()
    Y = _dev(_points(Y, "Y"))
    n, l = Y.shape
    piv = torch.empty(k, dtype=torch.int64, device=Y.device)
    rdiag = torch.empty(k, dtype=torch.float64, device=Y.device)
    _chk(lib, lib.krr_qrcp(_p(Y), n, l, k, _prec(prec), _p(piv), _p(rdiag), _stream()))
    return piv, rdiag


def fps(X, k: int, start: int = 0):
    """Farthest point sampling on the device: (S int64 k, dsel float64 k), dsel[0] = inf."""
    lib = load()
    X = _dev(_points(X))
    n, d = X.shape
    S = torch.empty(int(k), dtype=torch.int64, device="cuda")
    dsel = torch.empty(int(k), dtype=torch.float64, device="cuda")
    _chk(lib, lib.krr_fps(_p(X), n, d, int(k), int(start), _p(S), _p(dsel), _stream()))
    return S, dsel


def radix_sort_pairs(keys, vals, end_bit: int = 64):
    """Stable device sort of (uint64 key, int64 value) pairs by key bits [0, end_bit): (keys, vals) sorted.
    keys: a torch.int64 tensor holding the uint64 bit patterns; vals: torch.int64."""
    lib = load()
    keys = keys.to(device="cuda", dtype=torch.int64).contiguous()
    vals = vals.to(device="cuda", dtype=torch.int64).contiguous()
    if keys.shape != vals.shape or keys.dim() != 1:
        raise ValueError("keys and vals must be 1-D tensors of one length")
    ko, vo = torch.empty_like(keys), torch.empty_like(vals)
    _chk(lib, lib.krr_radix_sort_pairs(_p(keys), _p(ko), _p(vals), _p(vo), keys.numel(), int(end_bit), _stream()))
    return ko, vo


def rank_for_cond(X, eps: float, beta: float, xi: float, Mbar: Optional[float] = None):
    """Corollary tradeoff on the data: (gamma, k bound as a float, bounding-box side lengths q)."""
    lib = load()
    X = _dev(_points(X))
    n, d = X.shape
    g, kb = ctypes.c_double(), ctypes.c_double()
    q = (ctypes.c_double * d)()
    _chk(lib, lib.krr_rank_for_cond(_p(X), n, d, float(eps), float(beta), float(xi),
                                    0.0 if Mbar is None else float(Mbar), ctypes.byref(g), ctypes.byref(kb), q,
                                    _stream()))
    return g.value, kb.value, list(q)


class Preconditioner:
    """ID / Nystrom / Woodbury preconditioner (Algorithms 1-4) owned by the library."""

    W64, W32, LCORE, SKETCH, MCORE = 0, 1, 2, 3, 4

    def __init__(self, X, eps: float, betas: Sequence[float], k: int, l: Optional[int] = None, *, omega=None,
                 idx=None, sign=None, anchors=None, fps_start: int = 0, tau: float = 0.0, prec="fp64",
                 keep_sketch: bool = False):
        """anchors=None: Algorithm 1 (omega) or 2 (idx, sign) with l sketch columns and the pivoted QR;
        anchors="fps": farthest point sampling from fps_start; anchors=<k indices>: those points
        (random sampling: the caller draws them)."""
        lib = load()
        self._lib = lib
        self._h = None
        X = _points(X)
        self.n, self.d = X.shape
        if anchors is None and l is not None:
            _check_draws(self.n, omega, idx, sign, int(l))
        X = _dev(X)
        self.eps = float(eps)
        self.betas = [float(b) for b in betas]
        self.k = int(k)
        self.prec = _prec(prec)
        bh, nb = _host_f64(self.betas)
        h = ctypes.c_void_p()
        if anchors is not None:
            self.l = 0
            S = None if isinstance(anchors, str) and anchors == "fps" else _dev(anchors, torch.int64)
            if S is not None and S.numel() != self.k:
                raise ValueError("anchors must hold k indices")
            _chk(lib, lib.krr_build_precond_anchors(_p(X), self.n, self.d, self.eps, bh, nb, _p(S), self.k,
                                                    int(fps_start), float(tau), self.prec, ctypes.byref(h),
                                                    _stream()))
            self._h = h
            return
        if l is None:
            raise ValueError("l (sketch columns) is required unless anchors are given")
        self.l = int(l)
        if omega is not None:
            omega, r = _dev(omega), 0
        else:
            idx, sign = _dev(idx, torch.int64), _dev(sign)
            r = idx.shape[1]
        _chk(lib, lib.krr_build_precond(_p(X), self.n, self.d, self.eps, bh, nb, self.k, self.l, _p(omega),
                                        _p(idx), _p(sign), r, float(tau), self.prec, 1 if keep_sketch else 0,
                                        ctypes.byref(h), _stream()))
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self):
        k = self.k
        S = (ctypes.c_int64 * k)()
        lam = (ctypes.c_double * k)()
        rd = (ctypes.c_double * k)()
        kept = ctypes.c_int32()
        _chk(self._lib, self._lib.krr_precond_info(self._h, S, ctypes.byref(kept), lam, rd, None, None))
        return {"S": list(S), "kept": kept.value, "lam": list(lam), "rdiag": list(rd)}

    def timings(self):
        """Build phases in ms: sketch, qr, evd, factor, core, total (and the Jacobi sweep count)."""
        ms = (ctypes.c_double * 6)()
        sw = ctypes.c_int32()
        _chk(self._lib, self._lib.krr_precond_timings(self._h, ms, ctypes.byref(sw)))
        keys = ("sketch", "qr", "evd", "factor", "core", "total")
        return {**{k: ms[i] for i, k in enumerate(keys)}, "jacobi_sweeps": sw.value}

    def get(self, what: int, bidx: int = 0):
        info = self.info()
        kept = info["kept"]
        shapes = {0: ((self.n, kept), torch.float64), 1: ((self.n, kept), torch.float32),
                  2: ((kept, kept), torch.float64), 3: ((self.n, self.l), torch.float64),
                  4: ((kept, kept), torch.float64)}
        shape, dt = shapes[what]
        out = torch.empty(shape, dtype=dt, device="cuda")
        _chk(self._lib, self._lib.krr_precond_get(self._h, what, bidx, _p(out), out.numel() * out.element_size(),
                                                  _stream()))
        return out

    def apply(self, x, betas=None, prec=None):
        x = _dev(_rows(x, self.n, "x"))
        vec = x.dim() == 1
        x2 = x.reshape(x.shape[0], -1)
        R = x2.shape[1]
        betas = [self.betas[0]] * R if betas is None else _betas(betas, R)
        bh, _ = _host_f64(betas)
        out = torch.empty_like(x2)
        _chk(self._lib, self._lib.krr_precond_apply(self._h, _p(x2), R, bh,
                                                    self.prec if prec is None else _prec(prec), _p(out),
                                                    _stream()))
        return out[:, 0] if vec else out

    def apply_noalloc(self, x, out, betas=None, prec=None):
        """The Woodbury apply into the caller's `out` (n or n x R FP64 on the device, same shape as x) through
        krr_precond_apply_noalloc: the library allocates nothing (its scratch is a fixed device array)."""
        vec = x.dim() == 1
        _rows(x, self.n, "x")
        x2 = x.reshape(x.shape[0], -1)
        R = x2.shape[1]
        if x2.dtype != torch.float64 or not x2.is_cuda or not x2.is_contiguous():
            raise ValueError("x must be a contiguous FP64 device tensor")
        if out.shape != x.shape or out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous FP64 device tensor shaped like x")
        betas = [self.betas[0]] * R if betas is None else _betas(betas, R)
        bh, _ = _host_f64(betas)
        _chk(self._lib, self._lib.krr_precond_apply_noalloc(self._h, _p(x2), R, bh,
                                                            self.prec if prec is None else _prec(prec), _p(out),
                                                            _stream()))
        return out

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            try:
                torch.cuda.current_stream().synchronize()
                self._lib.krr_precond_free(self._h)
            except Exception:
                pass
            self._h = None


def pcg_solve(X, Y, eps: float, betas, P: Optional[Preconditioner] = None, *, tol=1e-8, maxit=10000,
              replace_every=0, prec="fp64", x0=None, timing=False):
    """Algorithm 5 for R right-hand sides. Returns (alpha, iters list, relres list, stats dict, status)."""
    lib = load()
    X = _points(X)
    n, d = X.shape
    Y = _rows(Y, n, "Y")
    R = 1 if Y.dim() == 1 else Y.shape[1]
    _need(x0 is None or _tensor(x0).numel() == n * R, f"x0 must hold n x R = {n} x {R} values")
    _need(P is None or (P.n, P.d) == (n, d), "the preconditioner was built for another point set")
    betas = _betas(betas, R)
    X, Y = _dev(X), _dev(Y)
    vec = Y.dim() == 1
    Y2 = Y.reshape(Y.shape[0], -1)
    bh, _ = _host_f64(betas)
    alpha = torch.zeros_like(Y2) if x0 is None else _dev(x0).reshape(n, R).clone()
    iters = (ctypes.c_int32 * R)()
    relres = (ctypes.c_double * R)()
    st = SolveStats()
    status = _chk(lib, lib.krr_pcg_solve(_p(X), n, d, float(eps), _p(Y2), R, bh, None if P is None else P.handle,
                                         float(tol), int(maxit), int(replace_every), _prec(prec), _p(alpha), iters,
                                         relres, ctypes.byref(st), 1 if timing else 0, _stream()))
    out = alpha[:, 0] if vec else alpha
    return out, list(iters), list(relres), st.as_dict(), status


def grad(Xtr, ytr, Xval, yval, eps: float, beta: float, P: Optional[Preconditioner] = None, *, tol=1e-8,
         maxit=10000, replace_every=0, prec="fp64", return_stats=False):
    """(loss, dL/dlog eps, dL/dlog beta, alpha, lambda, status) by the adjoint method.

    status is KRR_OK (0) or KRR_ENOCONV (1: the forward or the adjoint solve stopped before tol, so the
    loss and gradients come from unconverged iterates); errors raise KRRError.  With return_stats, a
    seventh element: the forward and adjoint solves' statistics (two dicts)."""
    lib = load()
    Xtr = _points(Xtr, "Xtr")
    n, d = Xtr.shape
    Xval = _points(Xval, "Xval", d)
    m = Xval.shape[0]
    _need(_tensor(ytr).numel() == n, f"ytr must hold n = {n} values")
    _need(_tensor(yval).numel() == m, f"yval must hold m = {m} values")
    _need(P is None or (P.n, P.d) == (n, d), "the preconditioner was built for another point set")
    Xtr, ytr, Xval, yval = _dev(Xtr), _dev(ytr), _dev(Xval), _dev(yval)
    loss, ge, gb = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    alpha = torch.empty(n, dtype=torch.float64, device=Xtr.device)
    lam = torch.empty(n, dtype=torch.float64, device=Xtr.device)
    st = (SolveStats * 2)()
    status = _chk(lib, lib.krr_grad(_p(Xtr), n, _p(ytr), _p(Xval), m, _p(yval), d, float(eps), float(beta),
                                    None if P is None else P.handle, float(tol), int(maxit), int(replace_every),
                                    _prec(prec), ctypes.byref(loss), ctypes.byref(ge), ctypes.byref(gb), _p(alpha),
                                    _p(lam), st if return_stats else None, _stream()))
    out = (loss.value, ge.value, gb.value, alpha, lam, status)
    if return_stats:
        return out + ([st[0].as_dict(), st[1].as_dict()],)
    return out


class KRRValLoss(torch.autograd.Function):
    """L(log eps, log beta) = 1/2 ||K(Xval, Xtr) alpha - yval||^2 with alpha = (K + beta I)^{-1} ytr.

    forward(log_eps, log_beta, Xtr, ytr, Xval, yval, P, opts) -> scalar loss; backward returns the
    adjoint gradients for log_eps and log_beta (X and y are not differentiated).  opts are grad()'s keyword
    arguments plus "allow_noconv": a solve that stops before tol raises KRRError(KRR_ENOCONV) unless it is
    True, in which case a RuntimeWarning is issued and the unconverged values are returned.
    """

    @staticmethod
    def forward(ctx, log_eps, log_beta, Xtr, ytr, Xval, yval, P=None, opts=None):
        opts = dict(opts or {})
        allow = bool(opts.pop("allow_noconv", False))
        eps, beta = float(torch.exp(log_eps)), float(torch.exp(log_beta))
        loss, ge, gb, _, _, status = grad(Xtr, ytr, Xval, yval, eps, beta, P, **opts)
        if status != 0:
            msg = load().krr_last_error().decode()
            if not allow:
                raise KRRError(status, msg)
            import warnings
            warnings.warn(f"KRRValLoss: {_STATUS.get(status, status)}: {msg}", RuntimeWarning, stacklevel=2)
        ctx.save_for_backward(torch.tensor([ge, gb], dtype=torch.float64))
        return torch.tensor(loss, dtype=torch.float64, device=log_eps.device)

    @staticmethod
    def backward(ctx, g):
        (gr,) = ctx.saved_tensors
        gr = gr.to(g.device)
        return g * gr[0], g * gr[1], None, None, None, None, None, None


def autotune(d: int, R: int = 1, prec="mixed", n: int = 65536) -> int:
    lib = load()
    best = ctypes.c_int32()
    _chk(lib, lib.krr_autotune(d, R, _prec(prec), n, ctypes.byref(best), _stream()))
    return best.value


def set_variant(d: int, R: int, prec, variant: int):
    lib = load()
    _chk(lib, lib.krr_set_variant(d, R, _prec(prec), variant))


def num_variants(prec, R: int = 1) -> int:
    lib = load()
    return lib.krr_num_variants(_prec(prec), R)


def kmv_variant(d: int, R: int = 1, prec="mixed", *, deriv: int = 0, square: bool = True, n: int = 0):
    """(variant, symmetric): the kernel variant a product of n sources would run (n = 0: size unknown) and
    whether it is the symmetric form."""
    lib = load()
    v, sym = ctypes.c_int32(), ctypes.c_int32()
    _chk(lib, lib.krr_kmv_variant(d, R, deriv, _prec(prec), 1 if square else 0, int(n), ctypes.byref(v),
                                  ctypes.byref(sym)))
    return v.value, bool(sym.value)


def kmv_last_launch():
    """(variant, split, symmetric) of the last kernel MVM launched on this thread."""
    lib = load()
    v, sp, sym = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _chk(lib, lib.krr_kmv_last_launch(ctypes.byref(v), ctypes.byref(sp), ctypes.byref(sym)))
    return v.value, sp.value, bool(sym.value)


def set_cull(mode: int):
    """Exact far-tile culling of square one-column mixed products: -1 automatic, 0 off, 1 on, 2 spatial order
    without skipping."""
    lib = load()
    _chk(lib, lib.krr_set_cull(int(mode)))


def set_pcg_mode(mode: int):
    """PCG driver: -1 automatic, 0 host loop (one synchronisation per iteration), 1 graph-captured cycles of
    replace_every iterations (one synchronisation per cycle).  Both give bit-identical results."""
    lib = load()
    _chk(lib, lib.krr_set_pcg_mode(int(mode)))


def cull_stats():
    """(pairs_total, pairs_skipped) of the last kernel MVM launched on this thread."""
    lib = load()
    tot, sk = ctypes.c_int64(), ctypes.c_int64()
    _chk(lib, lib.krr_cull_stats(ctypes.byref(tot), ctypes.byref(sk), _stream()))
    return tot.value, sk.value


def autotune_save(path: str):
    lib = load()
    _chk(lib, lib.krr_autotune_save(os.fsencode(path)))


def autotune_load(path: str):
    lib = load()
    _chk(lib, lib.krr_autotune_load(os.fsencode(path)))
