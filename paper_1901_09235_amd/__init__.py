"""MI355X (gfx950) convolutional sparse coding: the CSC step of DiCoDiLe.

Python binding of the C ABI in ``include/dicodile.h``.  The functions here only
marshal arguments: every step of the solve runs in the HIP library
``_build/libdicodile_mi355x.so`` (build it with
``python -m paper_1901_09235_amd.build``).  PyTorch provides device memory
and the current stream.  If the library is missing, every call raises.

Problem (arXiv:1901.09235, Sec. 2, eq. csc):
    Z* = argmin_Z 1/2 ||X - Z*D||^2 + lambda ||Z||_1   (optionally Z >= 0)
Shapes: signals X (P, T), D (K, P, L), Z (K, T-L+1);
        images  X (P, T1, T2), D (K, P, L1, L2), Z (K, T1-L1+1, T2-L2+1).
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["DicodileError", "library_path", "load", "dicodile_version", "dicodile_dtd",
           "dicodile_lambda_max", "dicodile_csc", "dicodile_csc_noalloc", "dicodile_objective_kkt",
           "dicodile_dict_stats", "dicodile_copy_probe", "dicodile_corr", "dicodile_csc_batch_autotune", "dicodile_csc_batch", "dicodile_release",
           "dicodile_dict_update", "dicodile_cdl", "Server", "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libdicodile_mi355x.so")
_lib = None

STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP",
          -4: "EDIVERGED", -5: "ETIMEOUT", -6: "ENODEV"}
F32, F64 = 0, 1
CORR_PREC = {"auto": 0, "f64": 1, "bf16": 2, "bf16x3": 3, "direct": 4, "f64_fft": 5}
FP64_METHOD = {"auto": 0, "mfma": 1, "fft": 2}
SELECT = {"lgcd": 0, "greedy": 1, "cyclic": 2, "random": 3}


class DicodileError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("P", ctypes.c_int32), ("K", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("T", ctypes.c_int64 * 2), ("L", ctypes.c_int32 * 2)]


class CscOpts(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("tol", ctypes.c_double),
                ("positive", ctypes.c_int32), ("certify", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("no_soft_lock", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("tile", ctypes.c_int32 * 2),
                ("grid", ctypes.c_int32 * 2), ("warm_start", ctypes.c_int32),
                ("refresh_every", ctypes.c_int32), ("max_polish", ctypes.c_int32),
                ("inner", ctypes.c_int32), ("beta_prec", ctypes.c_int32), ("max_rounds", ctypes.c_int64),
                ("div_guard", ctypes.c_double), ("timeout_s", ctypes.c_double),
                ("kkt_target", ctypes.c_double), ("strategy", ctypes.c_int32),
                ("refresh_limit", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("audit", ctypes.c_void_p), ("audit_rounds", ctypes.c_int32), ("fp64_method", ctypes.c_int32)]


class CscInfo(ctypes.Structure):
    _fields_ = [("n_updates", ctypes.c_int64), ("n_candidates", ctypes.c_int64),
                ("n_softlocked", ctypes.c_int64), ("n_rounds", ctypes.c_int64),
                ("n_sweeps", ctypes.c_int64), ("n_nonzero", ctypes.c_int64),
                ("objective", ctypes.c_double), ("kkt", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("t_total_s", ctypes.c_double),
                ("t_init_s", ctypes.c_double), ("t_cd_s", ctypes.c_double),
                ("t_check_s", ctypes.c_double), ("converged", ctypes.c_int32),
                ("grid", ctypes.c_int32 * 2), ("tile", ctypes.c_int32 * 2),
                ("n_passes", ctypes.c_int32), ("n_fft64", ctypes.c_int32),
                ("n_visits", ctypes.c_int64), ("n_checked", ctypes.c_int64),
                ("n_patched", ctypes.c_int64), ("t_worker_wait_s", ctypes.c_double),
                ("t_worker_select_s", ctypes.c_double), ("t_worker_collect_s", ctypes.c_double),
                ("t_worker_apply_s", ctypes.c_double), ("beta_drift", ctypes.c_double),
                ("t_init_corr_s", ctypes.c_double), ("t_corr64_s", ctypes.c_double),
                ("n_corr64", ctypes.c_int32), ("init_prec", ctypes.c_int32),
                ("t_check_inc_s", ctypes.c_double), ("n_check_inc", ctypes.c_int32), ("n_changed", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_len", ctypes.c_int64),
                ("max_workers", ctypes.c_int32), ("slice_rounds", ctypes.c_int32),
                ("max_active", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("tile", ctypes.c_int32 * 2), ("max_polish", ctypes.c_int32),
                ("admit_workers", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("n_submitted", ctypes.c_int64), ("n_done", ctypes.c_int64),
                ("n_launches", ctypes.c_int64), ("peak_active", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("peak_workers", ctypes.c_int64),
                ("t_rounds_s", ctypes.c_double), ("t_busy_s", ctypes.c_double)]


class DictOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32), ("tol", ctypes.c_double),
                ("c1", ctypes.c_double)]


class DictInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("backtracks", ctypes.c_int32),
                ("cost_initial", ctypes.c_double), ("cost", ctypes.c_double), ("t_s", ctypes.c_double)]


class CdlOpts(ctypes.Structure):
    _fields_ = [("lambda_frac", ctypes.c_double), ("nu", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("no_warm_start", ctypes.c_int32), ("tol_rel", ctypes.c_double), ("csc", CscOpts),
                ("dict", DictOpts)]


class CdlInfo(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32), ("converged", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("objective", ctypes.c_double * 64), ("objective_z", ctypes.c_double * 64),
                ("t_total_s", ctypes.c_double), ("t_csc_s", ctypes.c_double), ("t_stats_s", ctypes.c_double),
                ("t_dict_s", ctypes.c_double), ("n_updates", ctypes.c_int64)]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise DicodileError(-6, f"HIP library not built: {_LIB_PATH} is missing "
                                "(run python -m paper_1901_09235_amd.build)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sp = ctypes.POINTER(Shape)
    lib.dicodile_version.restype = ctypes.c_char_p
    lib.dicodile_last_error.restype = ctypes.c_char_p
    lib.dicodile_release.restype = ctypes.c_int
    lib.dicodile_dtd.argtypes = [sp, i32, vp, vp, vp]
    lib.dicodile_lambda_max.argtypes = [sp, i32, vp, vp, i32, ctypes.POINTER(dbl), vp]
    lib.dicodile_csc.argtypes = [sp, vp, vp, ctypes.POINTER(CscOpts), vp, ctypes.POINTER(CscInfo), vp]
    lib.dicodile_csc_noalloc.argtypes = [sp, vp, vp, ctypes.POINTER(CscOpts), vp, ctypes.POINTER(CscInfo), vp]
    lib.dicodile_objective_kkt.argtypes = [sp, i32, vp, vp, vp, dbl, i32, ctypes.POINTER(dbl),
                                           ctypes.POINTER(dbl), vp]
    lib.dicodile_dict_stats.argtypes = [sp, i32, vp, vp, vp, vp, vp]
    lib.dicodile_corr.argtypes = [sp, i32, vp, vp, vp, i32, vp]
    lib.dicodile_copy_probe.argtypes = [vp, vp, ctypes.c_size_t, i32, ctypes.POINTER(dbl), vp]
    lib.dicodile_csc_batch.argtypes = [i32, ctypes.c_void_p, ctypes.c_void_p, vp, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, vp]
    lib.dicodile_csc_batch_autotune.argtypes = [i32, ctypes.c_void_p, ctypes.c_void_p, vp, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, vp]
    lib.dicodile_dict_update.argtypes = [sp, i32, vp, vp, dbl, vp, ctypes.POINTER(DictOpts),
                                         ctypes.POINTER(DictInfo), vp]
    lib.dicodile_cdl.argtypes = [sp, i32, vp, vp, vp, ctypes.POINTER(CdlOpts), ctypes.POINTER(CdlInfo), vp]
    lib.dicodile_server_create.argtypes = [sp, i32, vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.dicodile_server_submit.argtypes = [vp, sp, vp, ctypes.POINTER(CscOpts), vp,
                                           ctypes.POINTER(ctypes.c_uint64)]
    lib.dicodile_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(CscInfo)]
    lib.dicodile_server_wait.argtypes = [vp, ctypes.c_uint64, dbl, ctypes.POINTER(CscInfo)]
    lib.dicodile_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.dicodile_server_destroy.argtypes = [vp]
    for f in ("dicodile_dtd", "dicodile_lambda_max", "dicodile_csc", "dicodile_csc_noalloc", "dicodile_objective_kkt", "dicodile_corr",
              "dicodile_dict_stats", "dicodile_copy_probe", "dicodile_corr", "dicodile_csc_batch_autotune", "dicodile_csc_batch",
              "dicodile_server_create", "dicodile_server_submit", "dicodile_server_poll",
              "dicodile_server_wait", "dicodile_server_stats", "dicodile_server_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _check(rc: int, allow_not_converged: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_not_converged):
        msg = load().dicodile_last_error().decode(errors="replace")
        raise DicodileError(rc, msg)
    return rc


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise DicodileError(-1, f"unsupported dtype {t.dtype} (float32 or float64)")


def _device_tensor(t, name):
    if not t.is_cuda:
        raise DicodileError(-1, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise DicodileError(-1, f"{name} must be contiguous")
    return t


def _shape(X, D) -> Shape:
    s = Shape()
    if X.dim() == 2 and D.dim() == 3:
        s.ndim, s.P, s.K = 1, X.shape[0], D.shape[0]
        s.T[0], s.L[0] = X.shape[1], D.shape[2]
    elif X.dim() == 3 and D.dim() == 4:
        s.ndim, s.P, s.K = 2, X.shape[0], D.shape[0]
        s.T[0], s.T[1] = X.shape[1], X.shape[2]
        s.L[0], s.L[1] = D.shape[2], D.shape[3]
    else:
        raise DicodileError(-1, f"unsupported shapes X{tuple(X.shape)} D{tuple(D.shape)}")
    if D.shape[1] != X.shape[0]:
        raise DicodileError(-1, "X and D disagree on the channel count P")
    return s


def _zshape(s: Shape):
    if s.ndim == 1:
        return (s.K, s.T[0] - s.L[0] + 1)
    return (s.K, s.T[0] - s.L[0] + 1, s.T[1] - s.L[1] + 1)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def dicodile_version() -> str:
    return load().dicodile_version().decode()


def dicodile_release() -> None:
    _check(load().dicodile_release())


def dicodile_dtd(D, stream=None):
    """DtD (K, K, 2L-1[, 2L2-1]) of a device dictionary D (K, P, L...)."""
    torch = _torch()
    lib = load()
    _device_tensor(D, "D")
    s = Shape()
    if D.dim() == 3:
        s.ndim, s.K, s.P, s.T[0], s.L[0] = 1, D.shape[0], D.shape[1], D.shape[2], D.shape[2]
        out = torch.empty((D.shape[0], D.shape[0], 2 * D.shape[2] - 1), dtype=D.dtype, device=D.device)
    else:
        s.ndim, s.K, s.P = 2, D.shape[0], D.shape[1]
        s.T[0], s.T[1], s.L[0], s.L[1] = D.shape[2], D.shape[3], D.shape[2], D.shape[3]
        out = torch.empty((D.shape[0], D.shape[0], 2 * D.shape[2] - 1, 2 * D.shape[3] - 1),
                          dtype=D.dtype, device=D.device)
    _check(lib.dicodile_dtd(ctypes.byref(s), _dtype_code(D), ctypes.c_void_p(D.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def dicodile_lambda_max(X, D, positive: bool = False, stream=None) -> float:
    lib = load()
    _device_tensor(X, "X")
    _device_tensor(D, "D")
    s = _shape(X, D)
    out = ctypes.c_double(0.0)
    _check(lib.dicodile_lambda_max(ctypes.byref(s), _dtype_code(X), ctypes.c_void_p(X.data_ptr()),
                                   ctypes.c_void_p(D.data_ptr()), int(positive), ctypes.byref(out),
                                   _stream(stream)))
    return out.value


def make_opts(lam: float, tol: float, dtype_code: int, positive=False, certify=True, grid=None,
              tile=None, threads=0, warm_start=False, refresh_every=0, max_polish=0, max_rounds=0,
              div_guard=0.0, timeout_s=0.0, kkt_target=0.0, no_soft_lock=False, inner=0,
              beta_prec=0, strategy=0, seed=0, refresh_limit=0, audit=None, fp64_method=0) -> CscOpts:
    """dcdl_csc_opts from keyword options; audit is an int64 device tensor of
    (rounds, W1 * W2) receiving the round log of the first launch;
    fp64_method is "auto", "mfma" or "fft" (or its code)."""
    o = CscOpts()
    o.lambda_, o.tol = float(lam), float(tol)
    o.positive, o.certify, o.dtype = int(positive), int(certify), int(dtype_code)
    o.no_soft_lock, o.threads = int(no_soft_lock), int(threads)
    if tile is not None:
        t = (tile, 0) if isinstance(tile, int) else tuple(tile)
        o.tile[0], o.tile[1] = int(t[0]), int(t[1])
    if grid is not None:
        g = (grid, 0) if isinstance(grid, int) else tuple(grid)
        o.grid[0], o.grid[1] = int(g[0]), int(g[1])
    o.warm_start, o.refresh_every, o.max_polish = int(warm_start), int(refresh_every), int(max_polish)
    o.refresh_limit = int(refresh_limit)
    o.max_rounds, o.div_guard, o.timeout_s = int(max_rounds), float(div_guard), float(timeout_s)
    o.kkt_target = float(kkt_target)
    o.inner = int(inner)
    o.beta_prec = CORR_PREC[beta_prec] if isinstance(beta_prec, str) else int(beta_prec)
    if isinstance(strategy, str):
        if strategy not in SELECT:
            raise DicodileError(-1, f"unknown selection rule {strategy!r} (one of {sorted(SELECT)})")
        strategy = SELECT[strategy]
    o.strategy, o.seed = int(strategy), int(seed) & (2 ** 64 - 1)
    if isinstance(fp64_method, str):
        if fp64_method not in FP64_METHOD:
            raise DicodileError(-1, f"unknown FP64 method {fp64_method!r} (one of {sorted(FP64_METHOD)})")
        fp64_method = FP64_METHOD[fp64_method]
    o.fp64_method = int(fp64_method)
    if audit is not None:
        torch = _torch()
        _device_tensor(audit, "audit")
        if audit.dtype != torch.int64 or audit.dim() != 2:
            raise DicodileError(-1, "audit must be an int64 device tensor (rounds, workers)")
        o.audit, o.audit_rounds = audit.data_ptr(), int(audit.shape[0])
    return o


def info_dict(info: CscInfo, status: int) -> dict:
    d = {f: getattr(info, f) for f, _ in CscInfo._fields_ if f != "reserved"}
    d["grid"] = (info.grid[0], info.grid[1])
    d["tile"] = (info.tile[0], info.tile[1])
    d["status"] = STATUS.get(status, status)
    return d


def dicodile_csc(X, D, lam: float, tol: float, z_out=None, stream=None, **opts):
    """Solve eq. csc on the device.  Returns (z, info dict).  See _csc_call."""
    return _csc_call("dicodile_csc", X, D, lam, tol, z_out, stream, opts)


def dicodile_csc_noalloc(X, D, lam: float, tol: float, z_out, stream=None, **opts):
    """dicodile_csc with every workspace in the library's fixed device scratch
    (no device allocation in the call; z_out must be given).  Problems needing
    more than that scratch raise DicodileError (EINVAL)."""
    if z_out is None:
        raise DicodileError(-1, "dicodile_csc_noalloc needs z_out")
    return _csc_call("dicodile_csc_noalloc", X, D, lam, tol, z_out, stream, opts)


def _csc_call(fn: str, X, D, lam: float, tol: float, z_out, stream, opts):
    """Solve eq. csc on the device.  Returns (z, info dict).

    Keyword options mirror dcdl_csc_opts: positive, certify, grid, tile,
    threads, warm_start, refresh_every, refresh_limit, max_polish, max_rounds,
    div_guard, timeout_s, kkt_target, no_soft_lock, inner, beta_prec, strategy
    ("lgcd", "greedy", "cyclic", "random" or the dcdl_select code) and seed.  A
    NOT_CONVERGED status is reported in info['status']; errors raise
    DicodileError."""
    torch = _torch()
    lib = load()
    _device_tensor(X, "X")
    _device_tensor(D, "D")
    s = _shape(X, D)
    code = _dtype_code(X)
    if D.dtype != X.dtype:
        raise DicodileError(-1, "X and D must share a dtype")
    if z_out is None:
        if opts.get("warm_start"):
            raise DicodileError(-1, "warm_start needs z_out")
        z_out = torch.empty(_zshape(s), dtype=X.dtype, device=X.device)
    _device_tensor(z_out, "z_out")
    if tuple(z_out.shape) != _zshape(s) or z_out.dtype != X.dtype:
        raise DicodileError(-1, f"z_out must be {_zshape(s)} {X.dtype}")
    o = make_opts(lam, tol, code, **opts)
    info = CscInfo()
    rc = getattr(lib, fn)(ctypes.byref(s), ctypes.c_void_p(X.data_ptr()),
                          ctypes.c_void_p(D.data_ptr()), ctypes.byref(o),
                          ctypes.c_void_p(z_out.data_ptr()), ctypes.byref(info), _stream(stream))
    _check(rc, allow_not_converged=True)
    return z_out, info_dict(info, rc)


def dicodile_corr(X, D, prec="auto", out=None, stream=None):
    """G = corr(X, D) on the valid domain, shape (K, T-L+1 ...), in X's dtype.
    prec: "auto", "f64", "bf16", "bf16x3", "direct" or "f64_fft" (dcdl_corr_prec)."""
    torch = _torch()
    lib = load()
    _device_tensor(X, "X")
    _device_tensor(D, "D")
    s = _shape(X, D)
    if D.dtype != X.dtype:
        raise DicodileError(-1, "X and D must share a dtype")
    if out is None:
        out = torch.empty(_zshape(s), dtype=X.dtype, device=X.device)
    _device_tensor(out, "out")
    if tuple(out.shape) != _zshape(s) or out.dtype != X.dtype:
        raise DicodileError(-1, f"out must be {_zshape(s)} {X.dtype}")
    code = CORR_PREC[prec] if isinstance(prec, str) else int(prec)
    _check(lib.dicodile_corr(ctypes.byref(s), _dtype_code(X), ctypes.c_void_p(X.data_ptr()),
                             ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(out.data_ptr()), code,
                             _stream(stream)))
    return out


def dicodile_objective_kkt(X, D, z, lam: float, positive: bool = False, stream=None):
    """FP64 objective and strict KKT violation (/ lambda) of z."""
    lib = load()
    for t, n in ((X, "X"), (D, "D"), (z, "z")):
        _device_tensor(t, n)
    s = _shape(X, D)
    obj, kkt = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib.dicodile_objective_kkt(ctypes.byref(s), _dtype_code(X), ctypes.c_void_p(X.data_ptr()),
                                      ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                      float(lam), int(positive), ctypes.byref(obj), ctypes.byref(kkt),
                                      _stream(stream)))
    return obj.value, kkt.value


def dicodile_dict_stats(z, X, L, stream=None):
    """(ztz, ztX) of eq. phi: ztz (K, K, 2L-1...), ztX (K, P, L...).  L is the
    atom size: int for signals, (L1, L2) for images."""
    torch = _torch()
    lib = load()
    _device_tensor(z, "z")
    _device_tensor(X, "X")
    s = Shape()
    K, P = z.shape[0], X.shape[0]
    if X.dim() == 2:
        s.ndim, s.P, s.K, s.T[0], s.L[0] = 1, P, K, X.shape[1], int(L)
        ztz = torch.empty((K, K, 2 * int(L) - 1), dtype=X.dtype, device=X.device)
        ztX = torch.empty((K, P, int(L)), dtype=X.dtype, device=X.device)
    else:
        L1, L2 = int(L[0]), int(L[1])
        s.ndim, s.P, s.K = 2, P, K
        s.T[0], s.T[1], s.L[0], s.L[1] = X.shape[1], X.shape[2], L1, L2
        ztz = torch.empty((K, K, 2 * L1 - 1, 2 * L2 - 1), dtype=X.dtype, device=X.device)
        ztX = torch.empty((K, P, L1, L2), dtype=X.dtype, device=X.device)
    if tuple(z.shape) != _zshape(s) or z.dtype != X.dtype:
        raise DicodileError(-1, f"z must be {_zshape(s)} {X.dtype}")
    _check(lib.dicodile_dict_stats(ctypes.byref(s), _dtype_code(X), ctypes.c_void_p(z.data_ptr()),
                                   ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(ztz.data_ptr()),
                                   ctypes.c_void_p(ztX.data_ptr()), _stream(stream)))
    return ztz, ztX


def _dict_shape(D) -> Shape:
    s = Shape()
    if D.dim() == 3:
        s.ndim, s.P, s.K, s.L[0], s.T[0] = 1, D.shape[1], D.shape[0], D.shape[2], D.shape[2]
    elif D.dim() == 4:
        s.ndim, s.P, s.K = 2, D.shape[1], D.shape[0]
        s.L[0], s.L[1], s.T[0], s.T[1] = D.shape[2], D.shape[3], D.shape[2], D.shape[3]
    else:
        raise DicodileError(-1, f"unsupported dictionary shape {tuple(D.shape)}")
    return s


def dicodile_dict_update(ztz, ztX, x_sq: float, D, max_iter: int = 0, tol: float = 0.0, c1: float = 0.0,
                         stream=None) -> dict:
    """Dictionary update of eq. dict_update from the statistics (ztz, ztX);
    D is updated in place.  Returns the info dict."""
    lib = load()
    for t, n in ((ztz, "ztz"), (ztX, "ztX"), (D, "D")):
        _device_tensor(t, n)
        if t.dtype != D.dtype:
            raise DicodileError(-1, "ztz, ztX and D must share a dtype")
    o = DictOpts()
    o.max_iter, o.tol, o.c1 = int(max_iter), float(tol), float(c1)
    info = DictInfo()
    _check(lib.dicodile_dict_update(ctypes.byref(_dict_shape(D)), _dtype_code(D), ctypes.c_void_p(ztz.data_ptr()),
                                    ctypes.c_void_p(ztX.data_ptr()), float(x_sq), ctypes.c_void_p(D.data_ptr()),
                                    ctypes.byref(o), ctypes.byref(info), _stream(stream)))
    return {f: getattr(info, f) for f, _ in DictInfo._fields_}


def dicodile_cdl(X, D, lambda_frac: float = 0.1, nu: float = 1e-4, max_outer: int = 0, tol_rel: float = 0.0,
                 warm_start: bool = True, z_out=None, dict_max_iter: int = 0, dict_tol: float = 0.0, stream=None,
                 **csc_opts):
    """Alg. 2 (convolutional dictionary learning): D is updated in place.
    Returns (z, info dict with the objective after each outer iteration)."""
    torch = _torch()
    lib = load()
    _device_tensor(X, "X")
    _device_tensor(D, "D")
    if X.dtype != D.dtype:
        raise DicodileError(-1, "X and D must share a dtype")
    s = _shape(X, D)
    if z_out is None:
        z_out = torch.empty(_zshape(s), dtype=X.dtype, device=X.device)
    _device_tensor(z_out, "z_out")
    o = CdlOpts()
    o.lambda_frac, o.nu, o.max_outer, o.tol_rel = float(lambda_frac), float(nu), int(max_outer), float(tol_rel)
    o.no_warm_start = int(not warm_start)
    o.csc = make_opts(1.0, 0.0, _dtype_code(X), **csc_opts)
    o.dict.max_iter, o.dict.tol = int(dict_max_iter), float(dict_tol)
    info = CdlInfo()
    rc = lib.dicodile_cdl(ctypes.byref(s), _dtype_code(X), ctypes.c_void_p(X.data_ptr()),
                          ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(z_out.data_ptr()), ctypes.byref(o),
                          ctypes.byref(info), _stream(stream))
    _check(rc, allow_not_converged=True)
    n = info.outer
    d = {"outer": n, "converged": info.converged, "lambda": info.lambda_,
         "objective": list(info.objective[:n]), "objective_z": list(info.objective_z[:n]),
         "t_total_s": info.t_total_s, "t_csc_s": info.t_csc_s, "t_stats_s": info.t_stats_s,
         "t_dict_s": info.t_dict_s, "n_updates": info.n_updates, "status": STATUS.get(rc, rc)}
    return z_out, d


def dicodile_copy_probe(dst, src, repeats: int = 10, stream=None) -> float:
    """Average seconds of one streaming copy dst <- src (device tensors of equal byte size)."""
    lib = load()
    _device_tensor(dst, "dst")
    _device_tensor(src, "src")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise DicodileError(-1, "copy probe buffers differ in size")
    out = ctypes.c_double(0.0)
    _check(lib.dicodile_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                   ctypes.c_size_t(nbytes), int(repeats), ctypes.byref(out),
                                   _stream(stream)))
    return out.value


class BatchOpts(ctypes.Structure):
    _fields_ = [("no_graph", ctypes.c_int32), ("workers", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("tile", ctypes.c_int32 * 2),
                ("max_polish", ctypes.c_int32), ("inner", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("t_total_s", ctypes.c_double), ("t_setup_s", ctypes.c_double),
                ("t_rounds_s", ctypes.c_double), ("t_check_s", ctypes.c_double),
                ("n_updates", ctypes.c_int64), ("workers", ctypes.c_int64),
                ("n_converged", ctypes.c_int32), ("n_passes", ctypes.c_int32),
                ("used_graph", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("n_trials", ctypes.c_int32), ("n_sample", ctypes.c_int32), ("t_tune_s", ctypes.c_double),
                ("trial_budget_s", ctypes.c_double), ("obj_default", ctypes.c_double),
                ("obj_best", ctypes.c_double), ("cached", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("obj_spread", ctypes.c_double)]


def _batch_args(Xs, D, lams, tols, opts):
    n = len(Xs)
    _device_tensor(D, "D")
    code = _dtype_code(D)
    shapes = (Shape * n)()
    xp = (ctypes.c_void_p * n)()
    ol = (CscOpts * n)()
    for i, X in enumerate(Xs):
        _device_tensor(X, f"X[{i}]")
        if X.dtype != D.dtype:
            raise DicodileError(-1, "every X must share D's dtype")
        shapes[i] = _shape(X, D)
        xp[i] = X.data_ptr()
        ol[i] = make_opts(lams[i], tols[i], code, **opts)
    return shapes, xp, ol


def dicodile_csc_batch_autotune(Xs, D, lams, tols, stream=None, **opts):
    """Tile, threads and worker budget for dicodile_csc_batch, timed on a
    sample of the batch.  Returns (dict of batch keyword options, info dict)."""
    lib = load()
    n = len(Xs)
    shapes, xp, ol = _batch_args(Xs, D, lams, tols, opts)
    best = BatchOpts()
    ti = TuneInfo()
    rc = lib.dicodile_csc_batch_autotune(ctypes.c_int32(n), ctypes.cast(shapes, ctypes.c_void_p),
                                         ctypes.cast(xp, ctypes.c_void_p), ctypes.c_void_p(D.data_ptr()),
                                         ctypes.cast(ol, ctypes.c_void_p), None,
                                         ctypes.cast(ctypes.byref(best), ctypes.c_void_p),
                                         ctypes.cast(ctypes.byref(ti), ctypes.c_void_p), _stream(stream))
    _check(rc)
    kw = {"workers": best.workers, "threads": best.threads, "tile": (best.tile[0], best.tile[1])}
    return kw, {f: getattr(ti, f) for f, _ in TuneInfo._fields_ if f != "reserved"}


def dicodile_csc_batch(Xs, D, lams, tols, z_outs=None, stream=None, graph=True, workers=0,
                       threads=0, tile=None, max_polish=0, inner=0, **opts):
    """Solve len(Xs) instances sharing D in one persistent launch.

    Xs: list of device tensors (P, T...) with the same P and ndim; lams, tols:
    per-instance floats.  Per-instance keyword options (positive, certify,
    kkt_target, no_soft_lock, div_guard) apply to every instance.  Returns
    (z list, per-instance info list, batch info dict)."""
    torch = _torch()
    lib = load()
    n = len(Xs)
    if n == 0:
        return [], [], {}
    _device_tensor(D, "D")
    code = _dtype_code(D)
    shapes = (Shape * n)()
    xp = (ctypes.c_void_p * n)()
    zp = (ctypes.c_void_p * n)()
    ol = (CscOpts * n)()
    if z_outs is None:
        z_outs = [None] * n
    outs = []
    for i, X in enumerate(Xs):
        _device_tensor(X, f"X[{i}]")
        if X.dtype != D.dtype:
            raise DicodileError(-1, "every X must share D's dtype")
        s = _shape(X, D)
        shapes[i] = s
        z = z_outs[i]
        if z is None:
            z = torch.empty(_zshape(s), dtype=X.dtype, device=X.device)
        _device_tensor(z, f"z_out[{i}]")
        if tuple(z.shape) != _zshape(s):
            raise DicodileError(-1, f"z_out[{i}] must be {_zshape(s)}")
        outs.append(z)
        xp[i] = X.data_ptr()
        zp[i] = z.data_ptr()
        ol[i] = make_opts(lams[i], tols[i], code, **opts)
    bo = BatchOpts()
    bo.no_graph, bo.workers, bo.threads, bo.max_polish = int(not graph), int(workers), int(threads), int(max_polish)
    bo.inner = int(inner)
    if tile is not None:
        t = (tile, 0) if isinstance(tile, int) else tuple(tile)
        bo.tile[0], bo.tile[1] = int(t[0]), int(t[1])
    infos = (CscInfo * n)()
    bi = BatchInfo()
    rc = lib.dicodile_csc_batch(ctypes.c_int32(n), ctypes.cast(shapes, ctypes.c_void_p),
                                ctypes.cast(xp, ctypes.c_void_p), ctypes.c_void_p(D.data_ptr()),
                                ctypes.cast(ol, ctypes.c_void_p), ctypes.cast(zp, ctypes.c_void_p),
                                ctypes.cast(infos, ctypes.c_void_p), ctypes.cast(ctypes.byref(bo), ctypes.c_void_p),
                                ctypes.cast(ctypes.byref(bi), ctypes.c_void_p), _stream(stream))
    _check(rc, allow_not_converged=True)
    il = [info_dict(infos[i], 0 if infos[i].converged else 1) for i in range(n)]
    bd = {f: getattr(bi, f) for f, _ in BatchInfo._fields_ if f != "reserved"}
    bd["status"] = STATUS.get(rc, rc)
    return outs, il, bd


_live_servers = set()


def _close_live_servers():
    for srv in list(_live_servers):
        srv.close()


class Server:
    """Continuous-batching CSC server over one dictionary (dicodile_server_*).

    ``submit`` queues a request and returns a ticket; ``wait``/``poll`` return
    (z, info dict) once it has finished.  X and z stay referenced here until
    then.  Use as a context manager or call ``close``; servers still open at
    interpreter exit are closed then."""

    def __init__(self, D, hbm_budget_bytes=0, max_len=0, max_workers=0, slice_rounds=0,
                 max_active=0, threads=0, tile=None, max_polish=0, admit_workers=0):
        lib = load()
        _device_tensor(D, "D")
        self.dtype_code = _dtype_code(D)
        self.D = D
        s = Shape()
        if D.dim() == 3:
            s.ndim, s.P, s.K, s.L[0] = 1, D.shape[1], D.shape[0], D.shape[2]
            s.T[0] = D.shape[2]
        elif D.dim() == 4:
            s.ndim, s.P, s.K = 2, D.shape[1], D.shape[0]
            s.L[0], s.L[1] = D.shape[2], D.shape[3]
            s.T[0], s.T[1] = D.shape[2], D.shape[3]
        else:
            raise DicodileError(-1, f"unsupported dictionary shape {tuple(D.shape)}")
        o = ServerOpts()
        o.hbm_budget_bytes, o.max_len = int(hbm_budget_bytes), int(max_len)
        o.max_workers, o.slice_rounds, o.max_active = int(max_workers), int(slice_rounds), int(max_active)
        o.threads, o.max_polish, o.admit_workers = int(threads), int(max_polish), int(admit_workers)
        if tile is not None:
            t = (tile, 0) if isinstance(tile, int) else tuple(tile)
            o.tile[0], o.tile[1] = int(t[0]), int(t[1])
        h = ctypes.c_void_p()
        _check(lib.dicodile_server_create(ctypes.byref(s), self.dtype_code, ctypes.c_void_p(D.data_ptr()),
                                          ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}
        _live_servers.add(self)

    def submit(self, X, lam: float, tol: float, z_out=None, **opts) -> int:
        """Queue one request; X must be complete on the device (synchronised)."""
        torch = _torch()
        lib = load()
        _device_tensor(X, "X")
        if X.dtype != self.D.dtype:
            raise DicodileError(-1, "X must share the dictionary's dtype")
        s = _shape(X, self.D)
        if z_out is None:
            z_out = torch.empty(_zshape(s), dtype=X.dtype, device=X.device)
        _device_tensor(z_out, "z_out")
        if tuple(z_out.shape) != _zshape(s) or z_out.dtype != X.dtype:
            raise DicodileError(-1, f"z_out must be {_zshape(s)} {X.dtype}")
        o = make_opts(lam, tol, self.dtype_code, **opts)
        t = ctypes.c_uint64()
        _check(lib.dicodile_server_submit(self._h, ctypes.byref(s), ctypes.c_void_p(X.data_ptr()),
                                          ctypes.byref(o), ctypes.c_void_p(z_out.data_ptr()),
                                          ctypes.byref(t)))
        self._keep[t.value] = (X, z_out)
        return t.value

    def _finish(self, ticket, rc, info):
        if rc == 2:
            return None
        X, z = self._keep.pop(ticket, (None, None))
        _check(rc, allow_not_converged=True)
        return z, info_dict(info, rc)

    def poll(self, ticket: int):
        """(z, info) if finished, else None."""
        info = CscInfo()
        rc = load().dicodile_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(info))
        return self._finish(ticket, rc, info)

    def wait(self, ticket: int, timeout_s: float = 0.0):
        """Block until the request finishes: (z, info); None on timeout."""
        info = CscInfo()
        rc = load().dicodile_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s), ctypes.byref(info))
        return self._finish(ticket, rc, info)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().dicodile_server_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _live_servers.discard(self)
            rc = load().dicodile_server_destroy(h)
            self._keep.clear()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _release_at_exit():
    """Hands the library's device workspaces and its stream back before the
    interpreter exits, while the HIP runtime is still whole (the runtime's own
    teardown runs later, from C-level exit handlers).  Nothing is done when the
    library was never loaded or no device was ever initialised."""
    if _lib is None:
        return
    import sys
    torch = sys.modules.get("torch")
    if torch is None or not torch.cuda.is_initialized():
        return
    torch.cuda.synchronize()
    _lib.dicodile_release()


import atexit as _atexit  # noqa: E402

# atexit runs handlers last-registered first: servers close, then the release
_atexit.register(_release_at_exit)
_atexit.register(_close_live_servers)
