"""Seeded synthetic CSC problems shaped like the paper's workloads.

Inputs follow the convolutional linear model X = Z*D + xi (Sec. 2, eq. model)
and the recipe of the paper's simulations (Sec. 5: Gaussian atoms normalised
to unit norm, Bernoulli sparse activations, white Gaussian noise).  The two
real images the paper uses (Mandrill, Hubble) are not available; the image
problems here are synthetic stand-ins with the same atom counts and sizes.

This module only draws random inputs and forms X by direct accumulation of
the shifted atoms.  It computes nothing the solver computes (no lambda_max,
no correlation, no coordinate update); the regularisation is returned as a
fraction of lambda_max for the caller to resolve.

Draw order for every problem: dictionary, shapes, activation support,
activation amplitudes, noise; all from numpy's PCG64 with the stated seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    X: np.ndarray            # (P, T) or (P, T1, T2), float64
    D: np.ndarray            # (K, P, L) or (K, P, L1, L2), float64, unit-norm atoms
    z_index: np.ndarray      # flat indices of the non-zero activations in zshape
    z_value: np.ndarray      # their values
    zshape: tuple            # (K, T-L+1) or (K, T1-L1+1, T2-L2+1)
    lambda_frac: float       # lambda = lambda_frac * lambda_max
    dtype: str               # "f64" or "f32": the working precision of the solve
    tol_rel: float           # epsilon as a multiple of lambda (f32), or absolute (f64)
    tol_abs: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def is_1d(self) -> bool:
        return self.X.ndim == 2

    @property
    def Z_true(self) -> np.ndarray:
        """The generating activations as a dense array (built on each access)."""
        Z = np.zeros(int(np.prod(self.zshape)))
        Z[self.z_index] = self.z_value
        return Z.reshape(self.zshape)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_dictionary(rng, K: int, P: int, L) -> np.ndarray:
    """K atoms with i.i.d. N(0,1) entries, each scaled to unit l2 norm."""
    shape = (K, P) + (tuple(L) if isinstance(L, (tuple, list)) else (int(L),))
    D = rng.standard_normal(shape)
    norms = np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1))
    return D / norms.reshape((K,) + (1,) * (D.ndim - 1))


def smooth_dictionary(rng, K: int, P: int, L) -> np.ndarray:
    """K smooth 2-D atoms of shape L = (L1, L2): an oriented anisotropic
    Gaussian envelope (widths U(1.5, 5) pixels, angle U(0, pi)) times a
    low-frequency cosine along its long axis (U(0, 0.6) rad/pixel), the same
    on every channel up to a N(0,1) channel weight, scaled to unit l2 norm.
    Shifted copies of such atoms overlap strongly, like the patch-like atoms
    learnt on natural images; the i.i.d. Gaussian atoms of
    gaussian_dictionary barely do."""
    L1, L2 = (int(v) for v in L)
    yy, xx = np.mgrid[0:L1, 0:L2]
    yy = yy - (L1 - 1) / 2.0
    xx = xx - (L2 - 1) / 2.0
    D = np.empty((K, P, L1, L2))
    for k in range(K):
        sx, sy = rng.uniform(1.5, 5.0, size=2)
        th = rng.uniform(0.0, np.pi)
        f = rng.uniform(0.0, 0.6)
        u = np.cos(th) * xx + np.sin(th) * yy
        v = -np.sin(th) * xx + np.cos(th) * yy
        atom = np.exp(-0.5 * ((u / sx) ** 2 + (v / sy) ** 2)) * np.cos(f * u)
        w = rng.standard_normal(P) if P > 1 else np.ones(1)
        D[k] = w[:, None, None] * atom[None]
        D[k] /= np.sqrt((D[k] ** 2).sum())
    return D


def bernoulli_support(rng, n: int, rho: float) -> np.ndarray:
    """Indices of a Bernoulli(rho) process on [0, n[, drawn as geometric gaps."""
    if rho <= 0.0 or n == 0:
        return np.zeros(0, dtype=np.int64)
    out = []
    pos = -1
    chunk = max(16, int(n * rho * 1.2) + 16)
    while True:
        gaps = rng.geometric(rho, size=chunk)
        idx = pos + np.cumsum(gaps)
        keep = idx[idx < n]
        out.append(keep)
        if keep.size < idx.size:
            break
        pos = int(idx[-1])
    return np.concatenate(out).astype(np.int64)


def _amplitudes(rng, kind: str, n: int) -> np.ndarray:
    if kind == "uniform":      # U(0.5, 1.5)
        return rng.uniform(0.5, 1.5, size=n)
    if kind == "exp":          # Exp(1)
        return rng.exponential(1.0, size=n)
    if kind == "gauss10":      # N(0, 10^2), the paper's 1-D recipe
        return rng.normal(0.0, 10.0, size=n)
    raise ValueError(kind)


def shifted_atom_sum(D: np.ndarray, index: np.ndarray, value: np.ndarray, zshape, T) -> np.ndarray:
    """sum over the non-zero activations (flat `index` into zshape, `value`) of
    a copy of the activation's atom at its position: X = Z*D of eq. model,
    accumulated with one histogram per channel."""
    if D.ndim == 3:
        X = shifted_atom_sum(D[:, :, None, :], index, value, (zshape[0], 1, zshape[1]), (1, int(T)))
        return X[:, 0, :]
    K, P, L1, L2 = D.shape
    T1, T2 = T
    H, W = zshape[1], zshape[2]
    X = np.zeros((P, T1 * T2))
    t1, t2 = np.meshgrid(np.arange(L1), np.arange(L2), indexing="ij")
    tap = (t1 * T2 + t2).ravel()                       # flattened tap offsets
    k_of = index // (H * W)
    r = index - k_of * (H * W)
    base_all = (r // W) * T2 + (r % W)                 # top-left corner in X
    chunk = max(1, 4_000_000 // (L1 * L2))
    for k in range(K):
        sel = k_of == k
        if not sel.any():
            continue
        base, v = base_all[sel], value[sel]
        Dk = D[k].reshape(P, L1 * L2)
        for c in range(0, base.size, chunk):
            idx = (base[c:c + chunk, None] + tap[None, :]).ravel()
            for p in range(P):
                w = (v[c:c + chunk, None] * Dk[p][None, :]).ravel()
                X[p] += np.bincount(idx, weights=w, minlength=T1 * T2)
    return X.reshape(P, T1, T2)


def make_problem(name: str, seed: int, P: int, T, K: int, L, rho: float, amp: str,
                 sigma: float, lambda_frac: float = 0.1, dtype: str = "f32",
                 tol_rel: float = 1e-5, tol_abs: bool = False, D: np.ndarray | None = None,
                 rng=None) -> Problem:
    """Generic problem: T and L are ints (1-D) or pairs (2-D)."""
    rng = _rng(seed) if rng is None else rng
    if D is None:
        D = gaussian_dictionary(rng, K, P, L)
    is_1d = not isinstance(T, (tuple, list))
    if is_1d:
        zshape = (K, int(T) - int(L) + 1)
    else:
        zshape = (K, int(T[0]) - int(L[0]) + 1, int(T[1]) - int(L[1]) + 1)
    n = int(np.prod(zshape))
    idx = bernoulli_support(rng, n, rho)
    val = _amplitudes(rng, amp, idx.size)
    X = shifted_atom_sum(D, idx, val, zshape, T)
    X = X + sigma * rng.standard_normal(X.shape)
    return Problem(name, X, D, idx, val, zshape, lambda_frac, dtype, tol_rel, tol_abs,
                   meta=dict(seed=seed, rho=rho, amp=amp, sigma=sigma))


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the paper's experiments: the 1-D
# simulation (Sec. 5, K=25 atoms of length 250 over P=7 channels), the image
# experiments (K=25 atoms of 16x16; Hubble: K=25 atoms of 32x32) and two
# deployment patterns (a batch of uneven images and a stream of requests).
# ---------------------------------------------------------------------------

def signal_1d(seed: int = 1000) -> Problem:
    """1-D, P=1, T=5000, K=5 atoms of length 64, Bernoulli(0.007) x U(0.5,1.5),
    noise N(0, 0.1^2), lambda = 0.1 lambda_max, double precision, tol 1e-8."""
    return make_problem("signal_1d_T5000_K5_L64", seed, P=1, T=5000, K=5, L=64, rho=0.007,
                        amp="uniform", sigma=0.1, lambda_frac=0.1, dtype="f64",
                        tol_rel=1e-8, tol_abs=True)


def image_1024(seed: int = 2000, size: int = 1024) -> Problem:
    """2-D, P=1, size x size pixels, K=25 atoms 16x16, Bernoulli(0.001) x
    U(0.5,1.5), sigma=0.1, lambda = 0.1 lambda_max, single precision."""
    return make_problem(f"image_{size}_K25_L16", seed, P=1, T=(size, size), K=25, L=(16, 16),
                        rho=0.001, amp="uniform", sigma=0.1, lambda_frac=0.1, dtype="f32")


def image_4096_rgb(seed: int = 3000, size: int = 4096) -> Problem:
    """2-D, P=3, size x size pixels, K=25 atoms 3x32x32, Bernoulli(5e-4) x
    Exp(1), sigma=0.05, lambda = 0.1 lambda_max, single precision."""
    return make_problem(f"image_rgb_{size}_K25_L32", seed, P=3, T=(size, size), K=25,
                        L=(32, 32), rho=5e-4, amp="exp", sigma=0.05, lambda_frac=0.1,
                        dtype="f32")


def batch_images(n: int = 256, seed: int = 4000, lo: int = 128, hi: int = 1024):
    """n single-channel images with sides uniform in [lo, hi] (independent
    height and width), shared K=16 atoms 12x12, Bernoulli(0.002) x
    U(0.5,1.5), sigma=0.1, lambda = 0.1 lambda_max each.  Image i uses seed
    seed+1+i; the dictionary uses seed."""
    D = gaussian_dictionary(_rng(seed), 16, 1, (12, 12))
    out = []
    for i in range(n):
        rng = _rng(seed + 1 + i)
        h, w = (int(v) for v in rng.integers(lo, hi + 1, size=2))
        out.append(make_problem(f"batch_{i}_{h}x{w}", seed + 1 + i, P=1, T=(h, w), K=16,
                                L=(12, 12), rho=0.002, amp="uniform", sigma=0.1,
                                lambda_frac=0.1, dtype="f32", D=D, rng=rng))
    return D, out


def serving_dictionary(seed: int = 5000) -> np.ndarray:
    """K=40 atoms, P=32 channels, length 128, unit norm."""
    return gaussian_dictionary(_rng(seed), 40, 32, 128)


def serving_arrivals(n: int, rate_hz: float = 200.0, seed: int = 5001) -> np.ndarray:
    """Poisson arrival times (seconds) at rate_hz."""
    return np.cumsum(_rng(seed).exponential(1.0 / rate_hz, size=n))


def serving_request(j: int, D: np.ndarray, seed0: int = 6000, t_lo: float = 1e4,
                    t_hi: float = 5e5) -> Problem:
    """Request j: T log-uniform in [t_lo, t_hi], Bernoulli(0.001) x Exp(1),
    sigma=0.1, lambda = 0.2 lambda_max, single precision."""
    rng = _rng(seed0 + j)
    T = int(round(float(np.exp(rng.uniform(np.log(t_lo), np.log(t_hi))))))
    return make_problem(f"request_{j}_T{T}", seed0 + j, P=32, T=T, K=40, L=128, rho=0.001,
                        amp="exp", sigma=0.1, lambda_frac=0.2, dtype="f32", D=D, rng=rng)


def paper_signal_1d(seed: int = 7000, T: int = 37500) -> Problem:
    """The paper's 1-D simulation: P=7, K=25, L=250, Bernoulli(0.007) x
    N(0, 10^2), noise N(0,1), lambda = 0.1 lambda_max."""
    return make_problem("paper_1d_P7_K25_L250", seed, P=7, T=T, K=25, L=250, rho=0.007,
                        amp="gauss10", sigma=1.0, lambda_frac=0.1, dtype="f32")
