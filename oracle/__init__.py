"""FP64 CPU oracle for the DiCoDiLe CSC step (arXiv:1901.09235).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
(``paper_1901_09235_amd``) never imports it and shares no code with it.

The arithmetic lives in ``csc_oracle.c`` (plain sequential C, double
precision); this module compiles it with gcc and wraps it with ctypes over
numpy arrays.  ``brute.py`` holds an independent brute-force Lasso solver for
tiny problems, used to pin the C code.

Array conventions (1-D inputs are promoted to the 2-D form with T1 = L1 = 1):
  X (P, T1, T2) or (P, T);  D (K, P, L1, L2) or (K, P, L);
  Z (K, T1-L1+1, T2-L2+1) or (K, T-L+1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libcsc_oracle.so")
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


class LgcdInfo(ctypes.Structure):
    _fields_ = [("n_updates", ctypes.c_int64), ("n_sweeps", ctypes.c_int64),
                ("converged", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("cost_decrease", ctypes.c_double), ("max_drift", ctypes.c_double),
                ("t_solve_s", ctypes.c_double), ("t_kkt_s", ctypes.c_double),
                ("sweeps_kkt", ctypes.c_int64)]


class DzInfo(ctypes.Structure):
    _fields_ = [("n_rounds", ctypes.c_int64), ("n_sweeps", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64), ("n_updates", ctypes.c_int64),
                ("n_softlocked", ctypes.c_int64), ("n_interfering", ctypes.c_int64),
                ("converged", ctypes.c_int32), ("diverged", ctypes.c_int32)]


def build(force: bool = True) -> str:
    """Compile csc_oracle.c into a shared library with gcc (no fast-math)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    shp = [ctypes.c_int, _i64, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_atom_norms.argtypes = [ctypes.c_int] * 4 + [_dp, _dp]
    lib.orc_dtd.argtypes = [ctypes.c_int] * 4 + [_dp, _dp]
    lib.orc_corr.argtypes = shp + [_dp, _dp, _dp]
    lib.orc_reconstruct.argtypes = shp + [_dp, _dp, _dp]
    lib.orc_lambda_max.argtypes = shp + [_dp, _dp, ctypes.c_int]
    lib.orc_lambda_max.restype = ctypes.c_double
    lib.orc_objective.argtypes = shp + [_dp, _dp, _dp, ctypes.c_double]
    lib.orc_objective.restype = ctypes.c_double
    lib.orc_kkt.argtypes = shp + [_dp, _dp, _dp, ctypes.c_double, ctypes.c_int]
    lib.orc_kkt.restype = ctypes.c_double
    lib.orc_beta.argtypes = shp + [_dp, _dp, _dp, _dp]
    lib.orc_lgcd.argtypes = shp + [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp,
                                   ctypes.POINTER(LgcdInfo)]
    lib.orc_lgcd.restype = ctypes.c_int
    lib.orc_dicodile_z.argtypes = shp + [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_double, _i64, _dp,
                                         ctypes.POINTER(DzInfo), ctypes.POINTER(ctypes.c_int64),
                                         _i64]
    lib.orc_dicodile_z.restype = ctypes.c_int
    lib.orc_dict_stats.argtypes = shp + [_dp, _dp, _dp, _dp]
    lib.orc_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.orc_draw.restype = ctypes.c_uint64
    lib.orc_rcd.argtypes = shp + [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  ctypes.c_uint64, _i64, ctypes.c_int, _dp, ctypes.POINTER(LgcdInfo)]
    lib.orc_rcd.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _as2d(X, D):
    """Promote 1-D signals to the 2-D form. Returns (X3, D4, is_1d)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    if X.ndim == 2 and D.ndim == 3:
        return X[:, None, :].copy(), D[:, :, None, :].copy(), True
    if X.ndim == 3 and D.ndim == 4:
        return X, D, False
    raise ValueError(f"unsupported shapes X{X.shape} D{D.shape}")


def _shape(X3, D4):
    P, T1, T2 = X3.shape
    K, P2, L1, L2 = D4.shape
    if P2 != P:
        raise ValueError("channel mismatch between X and D")
    return P, T1, T2, K, L1, L2


def _zshape(P, T1, T2, K, L1, L2):
    return (K, T1 - L1 + 1, T2 - L2 + 1)


def _out_z(Z3, is_1d):
    return Z3[:, 0, :].copy() if is_1d else Z3


def _in_z(Z, shape3, is_1d):
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if is_1d and Z.ndim == 2:
        Z = Z[:, None, :]
    return np.ascontiguousarray(Z.reshape(shape3))


def atom_norms(D) -> np.ndarray:
    """n_k = ||D_k||^2."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    D4 = D[:, :, None, :] if D.ndim == 3 else D
    D4 = np.ascontiguousarray(D4)
    K, P, L1, L2 = D4.shape
    n = np.zeros(K)
    _load().orc_atom_norms(K, P, L1, L2, _p(D4), _p(n))
    return n


def dtd(D) -> np.ndarray:
    """C[k0, k, tau + L - 1] = sum_p sum_t D[k0,p,t] D[k,p,t+tau]."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    is_1d = D.ndim == 3
    D4 = np.ascontiguousarray(D[:, :, None, :]) if is_1d else D
    K, P, L1, L2 = D4.shape
    C = np.zeros((K, K, 2 * L1 - 1, 2 * L2 - 1))
    _load().orc_dtd(K, P, L1, L2, _p(D4), _p(C))
    return C[:, :, 0, :].copy() if is_1d else C


def corr(R, D) -> np.ndarray:
    """G[k, w] = sum_p sum_t D[k,p,t] R[p, w+t] on the valid domain."""
    R3, D4, is_1d = _as2d(R, D)
    s = _shape(R3, D4)
    G = np.zeros(_zshape(*s))
    _load().orc_corr(*s, _p(R3), _p(D4), _p(G))
    return _out_z(G, is_1d)


def reconstruct(Z, D, T) -> np.ndarray:
    """Z*D on the full domain of size T (int or (T1, T2))."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    is_1d = D.ndim == 3
    D4 = np.ascontiguousarray(D[:, :, None, :]) if is_1d else D
    K, P, L1, L2 = D4.shape
    T1, T2 = (1, int(T)) if is_1d else (int(T[0]), int(T[1]))
    Z3 = _in_z(Z, (K, T1 - L1 + 1, T2 - L2 + 1), is_1d)
    out = np.zeros((P, T1, T2))
    _load().orc_reconstruct(P, T1, T2, K, L1, L2, _p(Z3), _p(D4), _p(out))
    return out[:, 0, :].copy() if is_1d else out


def lambda_max(X, D, positive: bool = False) -> float:
    X3, D4, _ = _as2d(X, D)
    return float(_load().orc_lambda_max(*_shape(X3, D4), _p(X3), _p(D4), int(positive)))


def objective(X, D, Z, lam: float) -> float:
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    Z3 = _in_z(Z, _zshape(*s), is_1d)
    return float(_load().orc_objective(*s, _p(X3), _p(D4), _p(Z3), float(lam)))


def kkt(X, D, Z, lam: float, positive: bool = False) -> float:
    """Strict KKT violation max over coordinates, divided by lambda."""
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    Z3 = _in_z(Z, _zshape(*s), is_1d)
    return float(_load().orc_kkt(*s, _p(X3), _p(D4), _p(Z3), float(lam), int(positive)))


def beta(X, D, Z) -> np.ndarray:
    """beta = corr(X - Z*D, D) + n (.) Z."""
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    Z3 = _in_z(Z, _zshape(*s), is_1d)
    out = np.zeros(_zshape(*s))
    _load().orc_beta(*s, _p(X3), _p(D4), _p(Z3), _p(out))
    return _out_z(out, is_1d)


def _default_tile(L1, L2, is_1d):
    return (1, 2 * L2) if is_1d else (2 * L1, 2 * L2)


def lgcd(X, D, lam: float, tol: float, positive: bool = False, tile=None,
         max_sweeps: int = 10 ** 9, z0=None, certify: bool = True, check_every: int = 0,
         kkt_every: int = 0, kkt_target: float = 1e-4, beta0=None):
    """Sequential LGCD (Alg. 1).  Returns (Z, info dict).

    certify=True makes support- and sign-changing moves score at least tol
    (the certifying stop rule); certify=False is the plain |Delta Z| rule.
    z0 warm-starts the sweeps; beta0 (with z0) is beta of z0 computed by the
    caller (e.g. ``beta_fft``), used instead of the direct FP64 loops."""
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    P, T1, T2, K, L1, L2 = s
    if tile is None:
        tile = _default_tile(L1, L2, is_1d)
    elif np.isscalar(tile):
        tile = (1, int(tile)) if is_1d else (int(tile), int(tile))
    Z = np.zeros(_zshape(*s)) if z0 is None else _in_z(z0, _zshape(*s), is_1d).copy()
    if beta0 is not None and z0 is None:
        raise ValueError("beta0 needs the iterate z0 it belongs to")
    b0 = None if beta0 is None else _in_z(beta0, _zshape(*s), is_1d)
    info = LgcdInfo()
    rc = _load().orc_lgcd(*s, _p(X3), _p(D4), float(lam), float(tol), int(positive),
                          int(tile[0]), int(tile[1]), int(max_sweeps), int(z0 is not None),
                          int(certify), int(check_every), int(kkt_every), float(kkt_target),
                          None if b0 is None else _p(b0), _p(Z), ctypes.byref(info))
    if rc != 0:
        raise ValueError("orc_lgcd rejected its arguments")
    d = {f: getattr(info, f) for f, _ in LgcdInfo._fields_ if f != "pad"}
    return _out_z(Z, is_1d), d


def draw(seed: int, stream: int, n: int) -> int:
    """The n-th value of stream `stream` of the randomized rule's generator
    (SplitMix64 of `seed`, counter n + stream * 2^40)."""
    return int(_load().orc_draw(int(seed) & (2 ** 64 - 1), int(stream), int(n)))


def rcd(X, D, lam: float, tol: float, seed: int = 0, positive: bool = False, certify: bool = True,
        max_epochs: int = 10 ** 6):
    """Sequential randomized coordinate descent (Sec. 3's random selection
    rule; the RCD of Sec. 5's comparison).  Coordinates are drawn uniformly
    with `draw(seed, 0, n)`; the run stops after an epoch (H W draws) whose
    final scan finds no move scoring >= tol.  Returns (Z, info dict) with
    n_sweeps = epochs."""
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    Z = np.zeros(_zshape(*s))
    info = LgcdInfo()
    rc = _load().orc_rcd(*s, _p(X3), _p(D4), float(lam), float(tol), int(positive),
                         int(seed) & (2 ** 64 - 1), int(max_epochs), int(certify), _p(Z),
                         ctypes.byref(info))
    if rc != 0:
        raise ValueError("orc_rcd rejected its arguments")
    d = {f: getattr(info, f) for f, _ in LgcdInfo._fields_ if f != "pad"}
    return _out_z(Z, is_1d), d


def dicodile_z(X, D, lam: float, tol: float, grid, positive: bool = False, tile=None,
               certify: bool = True, soft_lock: bool = True, div_guard: float = 0.0, max_rounds: int = 10 ** 9,
               log_rounds: int = 0):
    """Bulk-synchronous execution of Alg. 3 on one core.

    Returns (Z, info dict, log) where log has shape (log_rounds, W, 4) with
    (k0, w0_1, w0_2, accepted) per worker, k0 = -1 for no candidate."""
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    P, T1, T2, K, L1, L2 = s
    if tile is None:
        tile = _default_tile(L1, L2, is_1d)
    elif is_1d and np.isscalar(tile):
        tile = (1, int(tile))
    if is_1d and np.isscalar(grid):
        grid = (1, int(grid))
    W1, W2 = int(grid[0]), int(grid[1])
    Z = np.zeros(_zshape(*s))
    info = DzInfo()
    log = np.zeros((max(int(log_rounds), 0), W1 * W2, 4), dtype=np.int64)
    logp = log.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if log_rounds > 0 else None
    rc = _load().orc_dicodile_z(*s, _p(X3), _p(D4), float(lam), float(tol), int(positive),
                                int(certify), W1, W2, int(tile[0]), int(tile[1]), int(soft_lock), float(div_guard),
                                int(max_rounds), _p(Z), ctypes.byref(info), logp,
                                int(log_rounds))
    if rc != 0:
        raise ValueError("orc_dicodile_z rejected its arguments")
    d = {f: getattr(info, f) for f, _ in DzInfo._fields_}
    return _out_z(Z, is_1d), d, log


def dict_stats(Z, X, L):
    """phi (K, K, 2L1-1, 2L2-1) and psi (K, P, L1, L2) of eq. phi.

    L is the atom size: int for 1-D signals, (L1, L2) for images."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    is_1d = X.ndim == 2
    X3 = np.ascontiguousarray(X[:, None, :]) if is_1d else X
    P, T1, T2 = X3.shape
    L1, L2 = (1, int(L)) if is_1d else (int(L[0]), int(L[1]))
    K = int(np.asarray(Z).shape[0])
    Z3 = _in_z(Z, (K, T1 - L1 + 1, T2 - L2 + 1), is_1d)
    phi = np.zeros((K, K, 2 * L1 - 1, 2 * L2 - 1))
    psi = np.zeros((K, P, L1, L2))
    _load().orc_dict_stats(P, T1, T2, K, L1, L2, _p(Z3), _p(X3), _p(phi), _p(psi))
    if is_1d:
        return phi[:, :, 0, :].copy(), psi[:, :, 0, :].copy()
    return phi, psi
