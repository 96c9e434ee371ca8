"""FP64 oracle tools for parity at the workloads' full sizes (arXiv:1901.09235).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The direct loops of
``csc_oracle.c`` cost 2 K P |Theta| flops per position for beta, which is
teraflops for the largest workloads; here the one dense step of beta, the
correlation corr(R, D), is taken by FFT (scipy.fft, a library primitive,
FP64), and everything else stays in the C oracle:

  corr_fft(R, D)        G_k[w] = sum_p sum_t D_{k,p}[t] R_p[w + t] on the valid
                        domain (the paper's R * D~_k, Sec. 2), as a circular
                        convolution with the flipped atom: no wrap-around reaches
                        the valid outputs when the transform length is >= T.
  beta_fft(X, D, Z)     beta = corr(X - Z*D, D) + n (.) Z (definition of beta,
                        Sec. 3), with Z*D from the C oracle (non-zeros only).
  kkt_from_g(...)       the strict KKT violation of eq. csc from g.
  dual_gap(X, D, Z, lam)
                        P(Z) - Dual(nu) for the dual point nu = s R, s = min(1,
                        lam / max|corr(R, D)|) (max of corr for Z >= 0): weak
                        duality makes it an upper bound of F(Z) - F*.
  polish(X, D, Z0, lam) warm-started sequential LGCD (Alg. 1) from Z0 with
                        beta from beta_fft, by default with one-position
                        sub-domains (the cyclic rule Sec. 3 obtains from size-1
                        sub-domains), in chunks of sweeps each started from a
                        fresh beta: its summed Prop. A.1 decrease is
                        F(Z0) - F(Z_pol) exactly (to rounding), and with the
                        dual gap of Z_pol it bounds F(Z0) - F*.

Pinned in ``tests/test_oracle_large.py`` against the direct C loops, the
brute-force Lasso and scipy.
"""
from __future__ import annotations

import numpy as np
from scipy import fft as sfft

from . import _as2d, _in_z, _out_z, _shape, _zshape, atom_norms, lgcd, objective, reconstruct


def corr_fft(R, D, workers: int = -1) -> np.ndarray:
    """corr(R, D) on the valid domain by FFT, FP64.  R (P, T[, T2]), D (K, P, L[, L2])."""
    R3, D4, is_1d = _as2d(R, D)
    P, T1, T2, K, L1, L2 = _shape(R3, D4)
    n1 = sfft.next_fast_len(T1, real=True) if T1 > 1 else 1
    n2 = sfft.next_fast_len(T2, real=True)
    FR = sfft.rfftn(R3, s=(n1, n2), axes=(1, 2), workers=workers)
    G = np.empty(_zshape(P, T1, T2, K, L1, L2))
    for k in range(K):
        FD = sfft.rfftn(D4[k, :, ::-1, ::-1], s=(n1, n2), axes=(1, 2), workers=workers)
        FD *= FR
        full = sfft.irfftn(FD.sum(axis=0), s=(n1, n2), axes=(0, 1), workers=workers)
        G[k] = full[L1 - 1:T1, L2 - 1:T2]
    return _out_z(G, is_1d)


def beta_fft(X, D, Z, workers: int = -1) -> np.ndarray:
    """beta = corr(X - Z*D, D) + n (.) Z, FP64, with the correlation by FFT."""
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    Z3 = _in_z(Z, _zshape(*s), is_1d)
    T = X3.shape[2] if is_1d else X3.shape[1:]
    R = X3 - (reconstruct(Z3[:, 0, :], D4[:, :, 0, :], T)[:, None, :] if is_1d else reconstruct(Z3, D4, T))
    G = corr_fft(R, D4, workers=workers)
    n = atom_norms(D4)
    G += n.reshape(-1, 1, 1) * Z3
    return _out_z(G, is_1d)


def kkt_from_g(g, Z, lam: float, positive: bool = False) -> float:
    """Strict KKT violation of eq. csc divided by lam, for the negative
    gradient g = corr(X - Z*D, D): on zeros max(|g| - lam, 0) (max(g - lam, 0)
    when Z >= 0), on the support |g - lam sign Z|."""
    g = np.asarray(g, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    zero = Z == 0
    if positive:
        v_zero = np.maximum(g - lam, 0.0)
    else:
        v_zero = np.maximum(np.abs(g) - lam, 0.0)
    v_supp = np.abs(g - lam * np.sign(Z))
    return float(np.where(zero, v_zero, v_supp).max()) / lam


def dual_gap(X, D, Z, lam: float, positive: bool = False, workers: int = -1) -> dict:
    """Primal F(Z), the dual value of nu = s R and their gap (an upper bound of
    F(Z) - F*), with the strict KKT of Z from the same correlation."""
    X3, D4, is_1d = _as2d(X, D)
    s = _shape(X3, D4)
    Z3 = _in_z(Z, _zshape(*s), is_1d)
    T = X3.shape[2] if is_1d else X3.shape[1:]
    R = X3 - (reconstruct(Z3[:, 0, :], D4[:, :, 0, :], T)[:, None, :] if is_1d else reconstruct(Z3, D4, T))
    g = corr_fft(R, D4, workers=workers)
    gmax = float(g.max()) if positive else float(np.abs(g).max())
    sc = 1.0 if gmax <= lam else lam / gmax
    primal = 0.5 * float((R * R).sum()) + lam * float(np.abs(Z3).sum())
    dual = 0.5 * float((X3 * X3).sum()) - 0.5 * float(((X3 - sc * R) ** 2).sum())
    return {"primal": primal, "dual": dual, "gap": primal - dual, "kkt": kkt_from_g(g, Z3, lam, positive)}


def polish(X, D, Z0, lam: float, tol_rel: float = 1e-8, positive: bool = False, tile=(1, 1),
           sweeps_per_chunk: int = 4, max_chunks: int = 200, workers: int = -1, progress=None) -> dict:
    """Warm-started FP64 LGCD from Z0 to tol = tol_rel * lam (certifying stop).

    Runs chunks of `sweeps_per_chunk` sweeps, each from beta recomputed by
    beta_fft at the chunk's starting iterate, until a chunk stops on the
    certificate.  Returns F(Z0), the summed Prop. A.1 decrease, F of the
    polished point, its dual gap and strict KKT, and bound = decrease + gap
    >= F(Z0) - F*, with rel_bound = bound / F(Z0).  `progress(msg)` is called
    after every chunk."""
    Z = np.asarray(Z0, dtype=np.float64)
    f0 = objective(X, D, Z, lam)
    decrease, updates, sweeps, converged = 0.0, 0, 0, 0
    for chunk in range(max_chunks):
        b = beta_fft(X, D, Z, workers=workers)
        Z, info = lgcd(X, D, lam, tol_rel * lam, positive=positive, tile=tile, z0=Z, beta0=b,
                       max_sweeps=sweeps_per_chunk)
        decrease += info["cost_decrease"]
        updates += info["n_updates"]
        sweeps += info["n_sweeps"]
        if progress:
            progress(f"polish chunk {chunk}: {info['n_updates']} updates in {info['n_sweeps']} sweeps, "
                     f"decrease {info['cost_decrease']:.3e}")
        if info["converged"]:
            converged = 1
            break
    dg = dual_gap(X, D, Z, lam, positive=positive, workers=workers)
    bound = decrease + max(dg["gap"], 0.0)
    return {"f0": f0, "decrease": decrease, "f_polished": dg["primal"], "dual_gap": dg["gap"],
            "kkt_polished": dg["kkt"], "bound": bound, "rel_bound": bound / abs(f0), "updates": updates,
            "sweeps": sweeps, "converged": converged, "Z": Z}
