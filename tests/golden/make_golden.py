"""Writes tiny CSC problems and their exact Lasso minimisers to brute_force_cases.json.

The expected values come from the brute-force enumerator in ``oracle/brute.py``
(sign-pattern enumeration over the explicit Toeplitz design), not from the
coordinate-descent code they are used to check.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import brute  # noqa: E402

CASES = [
    # name, seed, K, P, L, T, lambda fraction of max|A^T y|, positive
    ("1d_K2_L3_T7", 11, 2, 1, 3, 7, 0.3, False),
    ("1d_K2_L3_T7_pos", 12, 2, 1, 3, 7, 0.2, True),
    ("1d_K1_P2_L4_T13", 13, 1, 2, 4, 13, 0.25, False),
    ("2d_K1_P2_L2x2_T4x4", 14, 1, 2, (2, 2), (4, 4), 0.3, False),
    ("2d_K2_P1_L3x2_T4x3", 15, 2, 1, (3, 2), (4, 3), 0.15, False),
    ("2d_K6_P2_L3x3_T3x3_dense", 16, 6, 2, (3, 3), (3, 3), 0.2, False),
]


def main():
    out = []
    for name, seed, K, P, L, T, frac, positive in CASES:
        rng = np.random.Generator(np.random.PCG64(seed))
        dshape = (K, P) + (tuple(L) if isinstance(L, tuple) else (L,))
        D = rng.standard_normal(dshape)
        D /= np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1)).reshape((K,) + (1,) * (D.ndim - 1))
        xshape = (P,) + (tuple(T) if isinstance(T, tuple) else (T,))
        X = rng.standard_normal(xshape)
        A = brute.design_matrix(D, T)
        y = X.ravel()
        lam = frac * float(np.abs(A.T @ y).max())
        z, f = brute.brute_force_lasso(A, y, lam, positive=positive)
        out.append(dict(name=name, source="oracle/brute.py sign-pattern enumeration",
                        D=D.tolist(), X=X.tolist(), T=T, lam=lam, positive=positive,
                        z=z.tolist(), objective=f))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "brute_force_cases.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
