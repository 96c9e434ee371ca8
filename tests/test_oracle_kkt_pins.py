"""Two-sided pins of the oracle's strict-KKT grader and of the non-negative
lambda_max (Sec. 2: optimality of eq. csc and the lambda_max paragraph).

The grader of every GPU parity test is ``oracle.kkt``.  Here it is evaluated
at deliberately NON-optimal points and must equal, to rounding, the distance
of the negative gradient g = A^T (y - A z) to lambda times the subdifferential
of |z| (signed) or of |z| + the indicator of z >= 0 (non-negative).  g comes
from ``oracle/brute.py``'s explicit Toeplitz design, a numpy matrix product
that shares nothing with the C oracle's correlation and residual loops.  The
points mix zeros whose |g| is above and below lambda with support
coordinates whose g has the same and the opposite sign as z, so dropping the
support branch or replacing |g - lambda sign z| by |g| - lambda changes the
value; ``test_kkt_pins_reject_planted_mistakes`` compiles such mutants of the
C source and checks that they fail.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest
from scipy import signal

import oracle
from oracle import brute


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _dict(rng, K, P, L):
    shape = (K, P) + (tuple(L) if isinstance(L, tuple) else (L,))
    D = rng.standard_normal(shape)
    return D / np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1)).reshape((K,) + (1,) * (D.ndim - 1))


def _problem(seed, oned, P=2, K=3):
    rng = _rng(seed)
    if oned:
        D = _dict(rng, K, P, 4)
        T = 17
        X = rng.standard_normal((P, T))
        zshape = (K, T - 3)
    else:
        D = _dict(rng, K, P, (3, 2))
        T = (7, 8)
        X = rng.standard_normal((P,) + T)
        zshape = (K, 5, 7)
    return rng, D, T, X, zshape


def _subgradient_distance(A, y, z, lam, positive):
    """max_i dist(g_i, lam * subdifferential_i) / lam with g = A^T (y - A z).

    Signed: the subdifferential of |z_i| is {sign z_i} off zero and [-1, 1]
    at zero.  Non-negative: that of |z_i| + indicator(z_i >= 0) is {1} for
    z_i > 0 and (-inf, 1] at zero."""
    g = A.T @ (y - A @ z)
    lo = np.where(z != 0, lam * np.sign(z), -np.inf if positive else -lam)
    hi = np.where(z != 0, lam * np.sign(z), lam)
    proj = np.clip(g, lo, hi)
    return float(np.abs(g - proj).max()) / lam, g


def _mixed_point(rng, zshape, positive):
    """A point whose zeros and support exercise every branch: z is drawn with
    about half of the coordinates non-zero; signs are random for the signed
    case, positive otherwise."""
    z = rng.standard_normal(zshape) * (rng.random(zshape) < 0.5)
    if positive:
        z = np.abs(z)
    return z


@pytest.mark.parametrize("oned", [True, False])
@pytest.mark.parametrize("positive", [False, True])
def test_kkt_equals_subgradient_distance_at_non_optimal_points(oned, positive):
    rng, D, T, X, zshape = _problem(100 + 2 * oned + positive, oned)
    A = brute.design_matrix(D, T)
    y = X.ravel()
    g0 = A.T @ y
    for trial in range(6):
        lam = float(np.quantile(np.abs(g0), 0.3 + 0.1 * trial))
        z = _mixed_point(rng, zshape, positive)
        want, g = _subgradient_distance(A, y, z.ravel(), lam, positive)
        gz = g.reshape(zshape)
        zero = z == 0
        # the point really exercises every branch
        assert (zero & (np.abs(gz) > lam)).any() and (zero & (np.abs(gz) < lam)).any()
        supp = ~zero
        assert (supp & (np.sign(gz) == np.sign(z))).any() and (supp & (np.sign(gz) != np.sign(z))).any()
        got = oracle.kkt(X, D, z, lam, positive=positive)
        assert got == pytest.approx(want, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("positive", [False, True])
def test_kkt_is_zero_exactly_at_the_brute_force_optimum(positive):
    """At the enumerated exact minimiser the grader reads 0 (to rounding); a
    sign flip of one support coordinate makes it read that coordinate's
    distance, |g - lambda sign(-z)|, which is at least 2 when z is small."""
    rng, D, T, X, zshape = _problem(120 + positive, True, P=1, K=2)
    T = 8
    X = X[:, :T]
    zshape = (2, T - 3)
    A = brute.design_matrix(D, T)
    y = X.ravel()
    lam = 0.3 * float(np.abs(A.T @ y).max())
    zs, _ = brute.brute_force_lasso(A, y, lam, positive=positive)
    assert np.count_nonzero(zs) >= 1
    assert oracle.kkt(X, D, zs.reshape(zshape), lam, positive=positive) < 1e-10
    if not positive:
        i = int(np.flatnonzero(zs)[0])
        zf = zs.copy()
        zf[i] = -zf[i]
        want, _ = _subgradient_distance(A, y, zf, lam, False)
        assert want > 1.0
        assert oracle.kkt(X, D, zf.reshape(zshape), lam) == pytest.approx(want, rel=1e-12)


def _mutant(tmp_path, name, pattern, replacement):
    src_path = os.path.join(os.path.dirname(oracle.__file__), "csc_oracle.c")
    with open(src_path) as fh:
        src = fh.read()
    new, n = re.subn(pattern, replacement, src, count=1)
    assert n == 1, f"mutation {name} did not apply"
    c = tmp_path / f"{name}.c"
    c.write_text(new)
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.orc_kkt.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int]
    lib.orc_kkt.restype = ctypes.c_double
    return lib


@pytest.mark.parametrize("name,pattern,replacement", [
    # the support branch dropped: every coordinate graded as a zero
    ("no_support_branch", r"if \(z == 0\.0\)\n(\s*)v = (positive \? [^;]*;)\n\s*else\n\s*v = [^;]*;",
     r"v = \2"),
    # |g| - lambda on the support instead of |g - lambda sign z|
    ("abs_minus_lambda", r"v = fabs\(g - lambda \* \(z > 0\.0 \? 1\.0 : -1\.0\)\);",
     "v = fabs(fabs(g) - lambda);"),
    # the sign of z ignored on the support
    ("no_sign", r"v = fabs\(g - lambda \* \(z > 0\.0 \? 1\.0 : -1\.0\)\);", "v = fabs(g - lambda);"),
])
def test_kkt_pins_reject_planted_mistakes(tmp_path, name, pattern, replacement):
    """Plausible mistakes planted in a copy of the C oracle's grader are caught
    by the explicit-design pin above."""
    lib = _mutant(tmp_path, name, pattern, replacement)
    rng, D, T, X, zshape = _problem(130, False)
    A = brute.design_matrix(D, T)
    y = X.ravel()
    lam = float(np.quantile(np.abs(A.T @ y), 0.5))
    z = _mixed_point(rng, zshape, False)
    want, _ = _subgradient_distance(A, y, z.ravel(), lam, False)
    X3 = np.ascontiguousarray(X, dtype=np.float64)
    D4 = np.ascontiguousarray(D, dtype=np.float64)
    Z3 = np.ascontiguousarray(z, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    got = lib.orc_kkt(2, 7, 8, 3, 3, 2, X3.ctypes.data_as(dp), D4.ctypes.data_as(dp), Z3.ctypes.data_as(dp),
                      lam, 0)
    assert abs(got - want) > 1e-6 * max(1.0, want), f"mutant {name} was not caught"
    assert oracle.kkt(X, D, z, lam) == pytest.approx(want, rel=1e-12)


# ------------------------------------------------------ non-negative lambda_max

def _negative_dominated_signal(seed):
    """A 1-D signal whose largest |corr(X, D)| is a NEGATIVE correlation, so
    the signed and the non-negative lambda_max differ."""
    rng = _rng(seed)
    K, P, L, T = 3, 2, 6, 60
    D = _dict(rng, K, P, L)
    X = 0.05 * rng.standard_normal((P, T))
    X[:, 20:20 + L] -= 3.0 * D[1]
    X[:, 40:40 + L] += 1.0 * D[2]
    corr = np.stack([sum(signal.correlate(X[p], D[k, p], "valid") for p in range(P)) for k in range(K)])
    return X, D, corr


def test_positive_lambda_max_is_the_largest_correlation():
    X, D, corr = _negative_dominated_signal(140)
    assert -corr.min() > corr.max() > 0
    assert oracle.lambda_max(X, D, positive=True) == pytest.approx(corr.max(), rel=1e-13)
    assert oracle.lambda_max(X, D) == pytest.approx(np.abs(corr).max(), rel=1e-13)
    # all correlations negative: no positive coordinate can ever move
    assert oracle.lambda_max(-np.abs(X), np.abs(D), positive=True) == 0.0


def test_positive_zero_solution_at_and_above_positive_lambda_max():
    """For lambda >= lambda_max+ the non-negative problem has Z = 0; the signed
    one at the same lambda does not (its lambda_max is larger)."""
    X, D, corr = _negative_dominated_signal(141)
    lmp = oracle.lambda_max(X, D, positive=True)
    for lam in (lmp, 1.2 * lmp):
        Z, info = oracle.lgcd(X, D, lam, 0.0, positive=True)
        assert info["n_updates"] == 0 and not Z.any()
    Zs, info = oracle.lgcd(X, D, lmp, 0.0)
    assert info["n_updates"] > 0 and (Zs < 0).any()


def test_positive_first_activation_just_below_positive_lambda_max():
    """Just below lambda_max+ the only non-zero of the non-negative solution is
    the argmax of corr(X, D) (not of |corr|), positive, with value
    (lambda_max+ - lambda) / ||D_k||^2."""
    X, D, corr = _negative_dominated_signal(142)
    D = D.copy()
    D[2] *= 0.8  # the winning atom has a non-unit norm
    corr = np.stack([sum(signal.correlate(X[p], D[k, p], "valid") for p in range(2)) for k in range(3)])
    lmp = oracle.lambda_max(X, D, positive=True)
    lam = lmp * (1 - 1e-9)
    Z, _ = oracle.lgcd(X, D, lam, 0.0, positive=True)
    nz = np.argwhere(Z != 0)
    assert nz.shape[0] == 1
    k, w = nz[0]
    assert (k, w) == np.unravel_index(np.argmax(corr), corr.shape)
    nk = float((D[k] ** 2).sum())
    assert Z[k, w] > 0
    assert Z[k, w] == pytest.approx((lmp - lam) / nk, rel=1e-6)
