"""Brute-force Lasso for tiny CSC problems (eq. csc of arXiv:1901.09235).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Independent of the C
oracle: it builds the Toeplitz design matrix of the convolution explicitly,
one column per coordinate (k, w), and enumerates every sign pattern in
{-1, 0, +1}^n.  For a support S with signs s the stationarity condition of
the Lasso reads A_S^T (y - A_S z_S) = lambda s, so
z_S = (A_S^T A_S)^{-1} (A_S^T y - lambda s); a pattern is admissible when
sign(z_S) = s.  The Lasso minimiser is admissible for its own pattern, and
every admissible z_S is a feasible point, so the least objective over the
admissible patterns is the optimum.
"""
from __future__ import annotations

import itertools

import numpy as np


def design_matrix(D: np.ndarray, T) -> np.ndarray:
    """Columns are the flattened shifted atoms e_w * D_k (valid-domain shifts).

    D: (K, P, L) with T an int, or (K, P, L1, L2) with T = (T1, T2).
    Column order: k major, then the shift in raster order."""
    D = np.asarray(D, dtype=np.float64)
    if D.ndim == 3:
        D = D[:, :, None, :]
        T1, T2 = 1, int(T)
    else:
        T1, T2 = int(T[0]), int(T[1])
    K, P, L1, L2 = D.shape
    H, W = T1 - L1 + 1, T2 - L2 + 1
    cols = []
    for k in range(K):
        for w1 in range(H):
            for w2 in range(W):
                img = np.zeros((P, T1, T2))
                img[:, w1:w1 + L1, w2:w2 + L2] = D[k]
                cols.append(img.ravel())
    return np.stack(cols, axis=1)


def lasso_objective(A: np.ndarray, y: np.ndarray, z: np.ndarray, lam: float) -> float:
    r = y - A @ z
    return 0.5 * float(r @ r) + lam * float(np.abs(z).sum())


def brute_force_lasso(A: np.ndarray, y: np.ndarray, lam: float, positive: bool = False):
    """Exact Lasso minimiser by enumeration.  Only for n <= 12 columns."""
    n = A.shape[1]
    if n > 12:
        raise ValueError("brute force is limited to 12 coordinates")
    G = A.T @ A
    c = A.T @ y
    best_z = np.zeros(n)
    best_f = lasso_objective(A, y, best_z, lam)
    signs = (0, 1) if positive else (-1, 0, 1)
    for pattern in itertools.product(signs, repeat=n):
        s = np.array(pattern, dtype=np.float64)
        S = np.flatnonzero(s)
        if S.size == 0:
            continue
        GS = G[np.ix_(S, S)]
        if np.linalg.matrix_rank(GS) < S.size:
            continue
        zS = np.linalg.solve(GS, c[S] - lam * s[S])
        if np.any(np.sign(zS) != s[S]):
            continue
        z = np.zeros(n)
        z[S] = zS
        f = lasso_objective(A, y, z, lam)
        if f < best_f:
            best_f, best_z = f, z
    return best_z, best_f
