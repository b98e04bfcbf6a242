"""Python binding of libfkkec (include/fkkec.h): fKK-EC on MI355X.

Argument marshalling only.  Device buffers are torch tensors on a ROCm
device; the library reads their data pointers and runs on the current torch
stream.  Every computation happens inside the library: if it is not built,
importing works but every call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfkkec.so")

FKK_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "device error",
          -4: "invalid intensities", -5: "basis / data mismatch", -7: "rank not available",
          -8: "internal numerical failure", -9: "busy"}
DETREND_ALS, DETREND_WHITTAKER = 0, 1
SEC_SAVGOL, SEC_MEAN = 0, 1
PAD_EDGE, PAD_ZERO = 0, 1
F_ONE, F_NOISE = 0, 1
OUT_IM, OUT_RE, OUT_ABS = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_FP64, PREC_SPLIT = 0, 1, 2, 3
SVD_GRAM, SVD_RANDOMIZED = 0, 1
TRIDIAG_NONE, TRIDIAG_RESIDENT, TRIDIAG_PER_COLUMN = 0, 1, 2
SEC_FORM_LOG, SEC_FORM_RE = 0, 1
OP_FIT, OP_TRANSFORM, OP_PLAIN = 0, 1, 2

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)


class Params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32), ("f_mode", ctypes.c_int32), ("alpha", ctypes.c_double),
        ("sigma_g", ctypes.c_double), ("pad_mode", ctypes.c_int32), ("fft_len", ctypes.c_int32),
        ("detrend", ctypes.c_int32), ("als_lambda", ctypes.c_double), ("als_p", ctypes.c_double),
        ("als_iters", ctypes.c_int32), ("ridge_rel", ctypes.c_double), ("sec_mode", ctypes.c_int32),
        ("sg_window", ctypes.c_int32), ("sg_order", ctypes.c_int32), ("ml_lambda", ctypes.c_double),
        ("ratio_floor", ctypes.c_double), ("strict", ctypes.c_int32), ("gram_prec", ctypes.c_int32),
        ("recon_prec", ctypes.c_int32), ("output", ctypes.c_int32),
        ("q_override", _c_int64_p), ("n_q_override", ctypes.c_int32),
        ("svd_mode", ctypes.c_int32), ("sec_form", ctypes.c_int32), ("rrf_oversample", ctypes.c_int32),
        ("rrf_power_iters", ctypes.c_int32),
        ("rrf_seed", ctypes.c_uint64), ("rrf_omega", _c_double_p), ("q_between", ctypes.c_int32),
    ]


class FitReport(ctypes.Structure):
    _fields_ = [
        ("clamps", ctypes.c_int64), ("n_q", ctypes.c_int32), ("ridge_lambda", ctypes.c_double),
        ("ms_gram", ctypes.c_double), ("ms_eig", ctypes.c_double), ("ms_project", ctypes.c_double),
        ("ms_basis", ctypes.c_double), ("ms_recon", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("dev_ms_gram", ctypes.c_double), ("dev_ms_project", ctypes.c_double), ("dev_ms_recon", ctypes.c_double),
        ("dev_ms_tridiag", ctypes.c_double), ("dev_ms_logratio", ctypes.c_double),
        ("tridiag_path", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BasisDesc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("k", ctypes.c_int32), ("i_ref", _c_double_p), ("f", _c_double_p),
        ("s", _c_double_p), ("v", _c_double_p), ("b_re", _c_double_p), ("b_im", _c_double_p),
        ("ml_lambda", ctypes.c_double), ("ratio_floor", ctypes.c_double),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch_rows", ctypes.c_int64), ("residual_threshold", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("spectra", ctypes.c_int64), ("launches", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("mean_batch_tiles", ctypes.c_double), ("flagged", ctypes.c_int64),
                ("max_residual", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_LIB = None

SYMBOLS = [
    "fkk_version", "fkk_status_string", "fkk_params_default", "fkk_ctx_create", "fkk_ctx_destroy",
    "fkk_ctx_last_error", "fkk_ctx_workspace_bytes", "fkk_workspace_size", "fkk_fit", "fkk_transform", "fkk_plain", "fkk_plain_f64",
    "fkk_gram",
    "fkk_eigh_topk", "fkk_basis_from_factors", "fkk_project", "fkk_reconstruct", "fkk_basis_residual",
    "fkk_basis_residual_noalloc",
    "fkk_basis_import", "fkk_basis_info", "fkk_basis_export", "fkk_basis_free", "fkk_basis_set_precision",
    "fkk_basis_get_precision", "fkk_server_create", "fkk_server_add_basis",
    "fkk_server_submit", "fkk_server_wait", "fkk_server_drain", "fkk_server_stats_get", "fkk_server_reset_stats",
    "fkk_server_destroy",
]


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fkk_version.restype = ctypes.c_int
    L.fkk_status_string.restype = ctypes.c_char_p
    L.fkk_status_string.argtypes = [ctypes.c_int]
    L.fkk_params_default.argtypes = [ctypes.POINTER(Params)]
    L.fkk_ctx_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.fkk_ctx_destroy.argtypes = [vp]
    L.fkk_ctx_last_error.restype = ctypes.c_char_p
    L.fkk_ctx_last_error.argtypes = [vp]
    L.fkk_ctx_workspace_bytes.restype = ctypes.c_size_t
    L.fkk_ctx_workspace_bytes.argtypes = [vp]
    sz = ctypes.c_size_t
    L.fkk_workspace_size.argtypes = [vp, i32, i64, i32, ctypes.POINTER(Params), ctypes.POINTER(sz)]
    L.fkk_fit.argtypes = [vp, vp, i64, i32, i64, _c_double_p, ctypes.POINTER(Params), ctypes.POINTER(vp), vp, i64,
                          vp, sz, ctypes.POINTER(FitReport)]
    L.fkk_transform.argtypes = [vp, vp, vp, i64, i64, vp, i64, i32, vp, vp, sz]
    L.fkk_plain.argtypes = [vp, vp, i64, i32, i64, _c_double_p, ctypes.POINTER(Params), vp, i64, vp, sz]
    L.fkk_plain_f64.argtypes = [vp, vp, i64, i32, i64, _c_double_p, ctypes.POINTER(Params), vp, i64, vp, sz]
    L.fkk_gram.argtypes = [vp, vp, i64, i32, i64, _c_double_p, dbl, i32, _c_double_p, _c_double_p, _c_int64_p]
    L.fkk_eigh_topk.argtypes = [_c_double_p, i32, i32, _c_double_p, _c_double_p]
    L.fkk_basis_from_factors.argtypes = [vp, i32, i32, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                         _c_double_p, i32, ctypes.POINTER(Params), ctypes.POINTER(vp)]
    L.fkk_project.argtypes = [vp, vp, vp, i64, i64, vp, i64, _c_int64_p, _c_int64_p]
    L.fkk_basis_residual.argtypes = [vp, vp, vp, i64, i64, ctypes.POINTER(ctypes.c_double)]
    L.fkk_basis_residual_noalloc.argtypes = [vp, vp, vp, i64, i64, ctypes.POINTER(ctypes.c_double)]
    L.fkk_reconstruct.argtypes = [vp, vp, vp, i64, i64, vp, i64, i32]
    L.fkk_basis_import.argtypes = [vp, ctypes.POINTER(BasisDesc), ctypes.POINTER(vp)]
    L.fkk_basis_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.fkk_basis_export.argtypes = [vp] + [_c_double_p] * 9 + [_c_int64_p, _c_double_p]
    L.fkk_basis_free.argtypes = [vp]
    L.fkk_basis_set_precision.argtypes = [vp, i32]
    L.fkk_basis_get_precision.argtypes = [vp, ctypes.POINTER(i32)]
    L.fkk_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    L.fkk_server_add_basis.argtypes = [vp, vp, ctypes.POINTER(i32)]
    L.fkk_server_submit.argtypes = [vp, i32, vp, i64, i64, vp, i64, ctypes.POINTER(i64)]
    L.fkk_server_wait.argtypes = [vp, i64, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.fkk_server_drain.argtypes = [vp]
    L.fkk_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.fkk_server_reset_stats.argtypes = [vp]
    L.fkk_server_destroy.argtypes = [vp]
    for name in ("fkk_server_create", "fkk_server_add_basis", "fkk_server_submit", "fkk_server_wait",
                 "fkk_server_drain", "fkk_server_stats_get", "fkk_server_reset_stats"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("fkk_ctx_create", "fkk_workspace_size", "fkk_fit", "fkk_transform", "fkk_plain", "fkk_plain_f64",
                 "fkk_gram", "fkk_basis_free",
                 "fkk_eigh_topk",
                 "fkk_basis_from_factors", "fkk_project", "fkk_reconstruct", "fkk_basis_residual",
                 "fkk_basis_residual_noalloc",
                 "fkk_basis_import", "fkk_basis_info", "fkk_basis_export", "fkk_basis_set_precision",
                 "fkk_basis_get_precision"):
        getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


# Live library objects, closed in dependency order (servers, then
# contexts, then bases) by an exit handler that runs while the interpreter
# and the HIP runtime are still whole.  After it, __del__ does nothing.
_LIVE = {"server": weakref.WeakSet(), "ctx": weakref.WeakSet(), "basis": weakref.WeakSet()}
_SHUTDOWN = False


def close_all():
    """Closes every live server, context and basis (servers first, since
    they hold bases).  Registered to run at interpreter exit."""
    global _SHUTDOWN
    for kind in ("server", "ctx", "basis"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close() if kind != "basis" else obj.free()
            except Exception:
                pass
    _SHUTDOWN = True


atexit.register(close_all)


def workspace_size(op: int, m: int, n: int, p: "Params | None" = None) -> int:
    """Device bytes fkk_fit (OP_FIT), fkk_plain (OP_PLAIN) or fkk_transform
    (OP_TRANSFORM) needs for m spectra of n points."""
    b = ctypes.c_size_t()
    st = lib().fkk_workspace_size(None, int(op), int(m), int(n), ctypes.byref(p) if p is not None else None,
                                  ctypes.byref(b))
    if st != FKK_OK:
        raise FkkError(st, "workspace_size")
    return int(b.value)


def _ws_args(ws):
    """(pointer, bytes) of a caller workspace tensor, or (None, 0)."""
    if ws is None:
        return None, 0
    import torch
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
        raise TypeError("ws must be a contiguous device tensor")
    return ws.data_ptr(), ws.numel() * ws.element_size()


class FkkError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_c_double_p)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def params(**overrides) -> Params:
    """fkk_params_default() with the given fields replaced."""
    p = Params()
    lib().fkk_params_default(ctypes.byref(p))
    q = overrides.pop("q_override", None)
    omega = overrides.pop("rrf_omega", None)
    for key, val in overrides.items():
        if not hasattr(p, key):
            raise AttributeError(key)
        setattr(p, key, val)
    if q is not None:
        q = np.ascontiguousarray(np.asarray(q, dtype=np.int64))
        p._q_keep = q  # keep the buffer alive with the struct
        p.q_override = q.ctypes.data_as(_c_int64_p)
        p.n_q_override = int(q.size)
    if omega is not None:
        omega = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        p._omega_keep = omega
        p.rrf_omega = omega.ctypes.data_as(_c_double_p)
    return p


def _check_tensor(t, name, dtype_name="float32"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"{name} must be {dtype_name}")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride")


def eigh_topk(a, k: int):
    """Top-k eigenpairs of a symmetric matrix (host FP64, library routine)."""
    a = _f64(a)
    n = a.shape[0]
    vals = np.empty(k)
    vecs = np.empty((n, k))
    st = lib().fkk_eigh_topk(_dptr(a), n, k, _dptr(vals), _dptr(vecs))
    if st != FKK_OK:
        raise FkkError(st, "eigh_topk")
    return vals, vecs


class Basis:
    """A fitted or imported basis set (owned by the library)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        if handle:
            _LIVE["basis"].add(self)

    @property
    def handle(self):
        return self._h

    def info(self):
        n, k, nq = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        lib().fkk_basis_info(self._h, ctypes.byref(n), ctypes.byref(k), ctypes.byref(nq))
        return n.value, k.value, nq.value

    @property
    def precision(self) -> int:
        """PREC_FP32, PREC_BF16 or PREC_SPLIT: precision of transforms with this basis."""
        p = ctypes.c_int32()
        st = lib().fkk_basis_get_precision(self._h, ctypes.byref(p))
        if st != FKK_OK:
            raise FkkError(st, "get_precision")
        return p.value

    @precision.setter
    def precision(self, prec: int):
        st = lib().fkk_basis_set_precision(self._h, int(prec))
        if st != FKK_OK:
            raise FkkError(st, "set_precision")

    def export(self) -> dict:
        n, k, nq = self.info()
        out = {"i_ref": np.empty(n), "f": np.empty(n), "s": np.empty(k), "v": np.empty((n, k)),
               "b_re": np.empty((k, n)), "b_im": np.empty((k, n)), "phi_pec_t": np.empty((k, n)),
               "v_sec_t": np.empty((k, n)), "h_v": np.empty((k, n))}
        q = np.empty(max(nq, 1), dtype=np.int64)
        sc = np.empty(3)
        st = lib().fkk_basis_export(self._h, *(_dptr(out[key]) for key in
                                               ("i_ref", "f", "s", "v", "b_re", "b_im", "phi_pec_t", "v_sec_t",
                                                "h_v")), q.ctypes.data_as(_c_int64_p), _dptr(sc))
        if st != FKK_OK:
            raise FkkError(st, "export")
        out["q"] = q[:nq]
        out["ml_lambda"], out["ratio_floor"], out["ridge_lambda"] = float(sc[0]), float(sc[1]), float(sc[2])
        return out

    def free(self):
        """Frees the basis; FkkError (busy) while a server holds it."""
        if self._h and self._h.value:
            st = lib().fkk_basis_free(self._h)
            if st != FKK_OK:
                raise FkkError(st, "basis_free: held by a server")
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        if _SHUTDOWN:
            return
        try:
            self.free()
        except Exception:
            pass


def basis_from_factors(ctx, i_ref, f, s, v, x, p: Params) -> Basis:
    """fKK / fPEC / fSEC on the host from the factors (ctx None: host only)."""
    i_ref, f, s = _f64(i_ref), _f64(f), _f64(s)
    v, x = _f64(v), _f64(x)
    n, k = v.shape
    out = ctypes.c_void_p()
    st = lib().fkk_basis_from_factors(ctx.handle if ctx is not None else None, n, k, _dptr(i_ref), _dptr(f),
                                      _dptr(s), _dptr(v), _dptr(x), x.shape[0], ctypes.byref(p), ctypes.byref(out))
    if st != FKK_OK:
        detail = ctx.last_error() if ctx is not None else ""
        raise FkkError(st, detail)
    return Basis(out.value)


class Context:
    """fkk_ctx bound to a device and the current torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib().fkk_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != FKK_OK:
            raise FkkError(st, "context creation")
        self._h = h
        _LIVE["ctx"].add(self)

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return lib().fkk_ctx_last_error(self._h).decode()

    def workspace_bytes(self) -> int:
        return int(lib().fkk_ctx_workspace_bytes(self._h))

    def _ok(self, st, what):
        if st != FKK_OK:
            raise FkkError(st, f"{what}: {self.last_error()}")

    def close(self):
        if self._h and self._h.value:
            lib().fkk_ctx_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        if _SHUTDOWN:
            return
        try:
            self.close()
        except Exception:
            pass

    # -- whole workflows --------------------------------------------------
    def fit(self, I, i_ref, p: Params, out=None, want_out: bool = True, ws=None, want_basis: bool = True):
        """fKK-EC fit; ws: optional device workspace tensor (workspace_size(OP_FIT))."""
        import torch
        _check_tensor(I, "I")
        m, n = I.shape
        i_ref = _f64(i_ref, (n,))
        if want_out and out is None:
            out = torch.empty((m, n), dtype=torch.float32, device=I.device)
        if out is not None:
            _check_tensor(out, "out")
        wp, wb = _ws_args(ws)
        rep = FitReport()
        b = ctypes.c_void_p()
        st = lib().fkk_fit(self._h, I.data_ptr(), m, n, I.stride(0), _dptr(i_ref), ctypes.byref(p),
                           ctypes.byref(b) if want_basis else None,
                           out.data_ptr() if out is not None else None, out.stride(0) if out is not None else n,
                           wp, wb, ctypes.byref(rep))
        self._ok(st, "fit")
        return (Basis(b.value) if want_basis else None), out, rep.as_dict()

    def transform(self, basis: Basis, I, out=None, plane: int = OUT_IM, norms=None):
        """Stored-basis transform; norms (optional, M x 2 float32 device
        tensor) receives each spectrum's ||A||^2 and ||A V||^2."""
        import torch
        _check_tensor(I, "I")
        m, n = I.shape
        if out is None:
            out = torch.empty((m, n), dtype=torch.float32, device=I.device)
        _check_tensor(out, "out")
        if norms is not None:
            _check_tensor(norms, "norms")
            if tuple(norms.shape) != (m, 2) or not norms.is_contiguous():
                raise ValueError("norms must be a contiguous M x 2 tensor")
        st = lib().fkk_transform(self._h, basis.handle, I.data_ptr(), m, I.stride(0), out.data_ptr(), out.stride(0),
                                 int(plane), norms.data_ptr() if norms is not None else None, None, 0)
        self._ok(st, "transform")
        return out

    def plain(self, I, i_ref, p: Params, out=None, ws=None):
        """Conventional per-spectrum KK / PEC / SEC.  float32 tensors use
        fkk_plain, float64 tensors fkk_plain_f64 (output of the same dtype);
        ws: optional device workspace tensor (workspace_size(OP_PLAIN))."""
        import torch
        f64 = I.dtype == torch.float64
        dt = "float64" if f64 else "float32"
        _check_tensor(I, "I", dt)
        m, n = I.shape
        i_ref = _f64(i_ref, (n,))
        if out is None:
            out = torch.empty((m, n), dtype=I.dtype, device=I.device)
        _check_tensor(out, "out", dt)
        fn = lib().fkk_plain_f64 if f64 else lib().fkk_plain
        wp, wb = _ws_args(ws)
        st = fn(self._h, I.data_ptr(), m, n, I.stride(0), _dptr(i_ref), ctypes.byref(p), out.data_ptr(),
                out.stride(0), wp, wb)
        self._ok(st, "plain")
        return out

    # -- stages -------------------------------------------------------------
    def gram(self, I, i_ref, ratio_floor: float = 1e-6, prec: int = PREC_FP32):
        _check_tensor(I, "I")
        m, n = I.shape
        i_ref = _f64(i_ref, (n,))
        g = np.empty((n, n))
        cs = np.empty(n)
        cl = np.zeros(1, dtype=np.int64)
        st = lib().fkk_gram(self._h, I.data_ptr(), m, n, I.stride(0), _dptr(i_ref), ratio_floor, int(prec), _dptr(g),
                            _dptr(cs), cl.ctypes.data_as(_c_int64_p))
        self._ok(st, "gram")
        return g, cs, int(cl[0])

    def project(self, basis: Basis, I, z=None, want_q: bool = True):
        import torch
        _check_tensor(I, "I")
        m, _ = I.shape
        _, k, _ = basis.info()
        if z is None:
            z = torch.empty((m, k), dtype=torch.float32, device=I.device)
        _check_tensor(z, "z")
        qmax = np.empty(k, dtype=np.int64)
        qmin = np.empty(k, dtype=np.int64)
        st = lib().fkk_project(self._h, basis.handle, I.data_ptr(), m, I.stride(0), z.data_ptr(), z.stride(0),
                               qmax.ctypes.data_as(_c_int64_p) if want_q else None,
                               qmin.ctypes.data_as(_c_int64_p) if want_q else None)
        self._ok(st, "project")
        return (z, qmax, qmin) if want_q else z

    def residual(self, basis: Basis, I) -> float:
        """||A - A V V^T||_F / ||A||_F of the spectra I against the basis."""
        _check_tensor(I, "I")
        m, _ = I.shape
        r = ctypes.c_double()
        st = lib().fkk_basis_residual(self._h, basis.handle, I.data_ptr(), m, I.stride(0), ctypes.byref(r))
        self._ok(st, "basis_residual")
        return r.value

    def residual_noalloc(self, basis: Basis, I) -> float:
        """residual() with the library's fixed scratch array: no allocation."""
        _check_tensor(I, "I")
        m, _ = I.shape
        r = ctypes.c_double()
        st = lib().fkk_basis_residual_noalloc(self._h, basis.handle, I.data_ptr(), m, I.stride(0), ctypes.byref(r))
        self._ok(st, "basis_residual_noalloc")
        return r.value

    def reconstruct(self, basis: Basis, z, plane: int = OUT_IM, out=None):
        import torch
        _check_tensor(z, "z")
        m = z.shape[0]
        n, _, _ = basis.info()
        if out is None:
            out = torch.empty((m, n), dtype=torch.float32, device=z.device)
        _check_tensor(out, "out")
        st = lib().fkk_reconstruct(self._h, basis.handle, z.data_ptr(), m, z.stride(0), out.data_ptr(), out.stride(0),
                                   plane)
        self._ok(st, "reconstruct")
        return out

    def basis_import(self, d: dict) -> Basis:
        arrs = {key: _f64(d[key]) for key in ("i_ref", "f", "s", "v", "b_re", "b_im")}
        n, k = arrs["v"].shape
        desc = BasisDesc(n, k, *(_dptr(arrs[key]) for key in ("i_ref", "f", "s", "v", "b_re", "b_im")),
                         float(d.get("ml_lambda", 0.0)), float(d.get("ratio_floor", 1e-6)))
        out = ctypes.c_void_p()
        st = lib().fkk_basis_import(self._h, ctypes.byref(desc), ctypes.byref(out))
        self._ok(st, "basis_import")
        return Basis(out.value)


class Server:
    """Continuous-batching server of stored-basis transforms (host tiles)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 8 << 30, max_inflight: int = 64,
                 max_batch_rows: int = 1 << 20, residual_threshold: float = 0.0):
        cfg = ServerConfig(hbm_budget_bytes, max_inflight, max_batch_rows, residual_threshold)
        h = ctypes.c_void_p()
        st = lib().fkk_server_create(device, ctypes.byref(cfg), ctypes.byref(h))
        if st != FKK_OK:
            raise FkkError(st, "server creation")
        self._h = h
        self._bases = []
        self._n = []
        self._held = {}  # ticket -> (tile, out): host buffers stay referenced until the tile completes
        _LIVE["server"].add(self)

    def add_basis(self, basis: Basis) -> int:
        bid = ctypes.c_int32()
        st = lib().fkk_server_add_basis(self._h, basis.handle, ctypes.byref(bid))
        if st != FKK_OK:
            raise FkkError(st, "add_basis")
        self._bases.append(basis)  # keep it alive as long as the server
        self._n.append(basis.info()[0])
        return bid.value

    @staticmethod
    def _host_view(a, name):
        """(pointer, rows, cols, row stride in elements) of a host float32
        2-D buffer with unit column stride."""
        if hasattr(a, "data_ptr"):
            if a.is_cuda:
                raise TypeError(f"{name} must be in host memory")
            if str(a.dtype) != "torch.float32" or a.dim() != 2 or a.stride(1) != 1:
                raise TypeError(f"{name} must be a 2-D float32 tensor with unit column stride")
            return a.data_ptr(), a.shape[0], a.shape[1], a.stride(0)
        if not isinstance(a, np.ndarray) or a.dtype != np.float32 or a.ndim != 2 or a.strides[1] != 4 \
                or a.strides[0] % 4:
            raise TypeError(f"{name} must be a 2-D float32 array with unit column stride")
        return a.ctypes.data, a.shape[0], a.shape[1], a.strides[0] // 4

    def submit(self, basis_id: int, tile, out) -> int:
        """tile, out: host (preferably pinned) float32 2-D tensors or arrays;
        out needs at least the tile's rows and both the basis's N columns."""
        if not 0 <= basis_id < len(self._n):
            raise FkkError(-1, f"submit: no basis {basis_id}")
        n = self._n[basis_id]
        tp, trows, tcols, tld = self._host_view(tile, "tile")
        op, orows, ocols, old = self._host_view(out, "out")
        if tcols < n or ocols < n:
            raise FkkError(-1, f"submit: tile and out need {n} columns (got {tcols}, {ocols})")
        if orows < trows:
            raise FkkError(-1, f"submit: out has {orows} rows for a tile of {trows}")
        t = ctypes.c_int64()
        st = lib().fkk_server_submit(self._h, basis_id, tp, trows, tld, op, old, ctypes.byref(t))
        if st != FKK_OK:
            raise FkkError(st, "submit")
        self._held[t.value] = (tile, out)
        return t.value

    def wait(self, ticket: int, timeout_ms: float = -1.0, with_residual: bool = False):
        """Latency (ms) of a completed tile, and with with_residual its
        relative residual against its basis."""
        lat, res = ctypes.c_double(), ctypes.c_double()
        st = lib().fkk_server_wait(self._h, ticket, timeout_ms, ctypes.byref(lat), ctypes.byref(res))
        if st != FKK_OK:
            raise FkkError(st, "wait")
        self._held.pop(ticket, None)
        return (lat.value, res.value) if with_residual else lat.value

    def drain(self):
        st = lib().fkk_server_drain(self._h)
        if st != FKK_OK:
            raise FkkError(st, "drain")
        self._held.clear()

    def stats(self) -> dict:
        s = ServerStats()
        st = lib().fkk_server_stats_get(self._h, ctypes.byref(s))
        if st != FKK_OK:
            raise FkkError(st, "stats")
        return s.as_dict()

    def reset_stats(self):
        lib().fkk_server_reset_stats(self._h)

    def close(self):
        if self._h and self._h.value:
            lib().fkk_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)
            self._held.clear()

    def __del__(self):
        if _SHUTDOWN:
            return
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Server", "Context", "Basis", "Params", "params", "eigh_topk", "basis_from_factors", "lib", "FkkError",
           "workspace_size", "close_all", "OP_FIT", "OP_TRANSFORM", "OP_PLAIN",
           "SYMBOLS", "LIB_PATH", "PREC_FP32", "PREC_BF16",
           "PREC_FP64", "PREC_SPLIT", "SVD_GRAM", "SVD_RANDOMIZED", "SEC_FORM_LOG", "SEC_FORM_RE"]
