"""Pins of the FP64 oracle against facts fixed outside it.

Each test compares the oracle (``oracle/``) with a library routine
(scipy.signal, sklearn), an exact enumeration (``oracle/brute.py`` and the
fixtures it wrote), a closed form, or an identity the paper proves.  None of
them re-types the oracle's own formula.
"""
import json
import os

import numpy as np
import pytest
from scipy import signal

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "brute_force_cases.json")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _dict(rng, K, P, L):
    shape = (K, P) + (tuple(L) if isinstance(L, tuple) else (L,))
    D = rng.standard_normal(shape)
    return D / np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1)).reshape((K,) + (1,) * (D.ndim - 1))


# --------------------------------------------------------------------- operators

@pytest.mark.parametrize("L", [(3, 4), (1, 5), (2, 2)])
def test_dtd_equals_scipy_correlate(L):
    """DtD (the kernel of eq. beta_update) from scipy's full cross-correlation."""
    rng = _rng(1)
    D = _dict(rng, 3, 2, L)
    C = oracle.dtd(D)
    for k0 in range(3):
        for k in range(3):
            ref = sum(signal.correlate(D[k, p], D[k0, p], mode="full") for p in range(2))
            np.testing.assert_allclose(C[k0, k], ref, rtol=0, atol=1e-14)


def test_dtd_symmetries():
    """C[k, k', tau] = C[k', k, -tau] and C[k, k, 0] = ||D_k||^2."""
    D = _dict(_rng(2), 4, 3, (3, 5))
    C = oracle.dtd(D)
    np.testing.assert_allclose(C, np.transpose(C, (1, 0, 2, 3))[:, :, ::-1, ::-1], atol=1e-14)
    np.testing.assert_allclose(C[np.arange(4), np.arange(4), 2, 4], 1.0, atol=1e-14)


@pytest.mark.parametrize("oned", [True, False])
def test_corr_equals_scipy_valid_correlation(oned):
    rng = _rng(3)
    if oned:
        D = _dict(rng, 3, 2, 5)
        R = rng.standard_normal((2, 23))
    else:
        D = _dict(rng, 3, 2, (3, 4))
        R = rng.standard_normal((2, 9, 11))
    G = oracle.corr(R, D)
    for k in range(3):
        ref = sum(signal.correlate(R[p], D[k, p], mode="valid") for p in range(2))
        np.testing.assert_allclose(G[k], ref, atol=1e-13)


@pytest.mark.parametrize("oned", [True, False])
def test_reconstruct_equals_scipy_full_convolution(oned):
    rng = _rng(4)
    if oned:
        D = _dict(rng, 3, 2, 5)
        T = 23
        Z = rng.standard_normal((3, T - 4)) * (rng.random((3, T - 4)) < 0.3)
    else:
        D = _dict(rng, 3, 2, (3, 4))
        T = (9, 11)
        Z = rng.standard_normal((3, 7, 8)) * (rng.random((3, 7, 8)) < 0.3)
    out = oracle.reconstruct(Z, D, T)
    for p in range(2):
        ref = sum(signal.convolve(Z[k], D[k, p], mode="full") for k in range(3))
        np.testing.assert_allclose(out[p], ref, atol=1e-13)


# --------------------------------------------------------------- lambda_max pins

def test_zero_solution_at_and_above_lambda_max():
    """For lambda >= lambda_max, Z = 0 is optimal (Sec. 2): no update at all."""
    rng = _rng(5)
    D = _dict(rng, 3, 1, (4, 4))
    X = rng.standard_normal((1, 20, 18))
    lm = oracle.lambda_max(X, D)
    for lam in (lm, lm * 1.5):
        Z, info = oracle.lgcd(X, D, lam, 0.0)
        assert info["n_updates"] == 0 and info["converged"] == 1
        assert not Z.any()


def test_first_activation_just_below_lambda_max():
    """Just below lambda_max the only non-zero is the argmax of |corr(X, D)|,
    with value (lambda_max - lambda) sign / ||D_k||^2."""
    rng = _rng(6)
    D = _dict(rng, 3, 2, 6)
    D[1] *= 0.7  # a non-unit atom, so the 1/||D_k||^2 factor is exercised
    X = rng.standard_normal((2, 60))
    G = signal.correlate(X[0], D[0, 0], "valid")  # only used to check shapes
    assert G.shape == (55,)
    lm = oracle.lambda_max(X, D)
    lam = lm * (1 - 1e-9)
    Z, info = oracle.lgcd(X, D, lam, 0.0)
    nz = np.argwhere(Z != 0)
    assert nz.shape[0] == 1
    k, w = nz[0]
    corr = sum(signal.correlate(X[p], D[k, p], "valid") for p in range(2))
    assert abs(abs(corr[w]) - lm) < 1e-12
    nk = float((D[k] ** 2).sum())
    assert Z[k, w] == pytest.approx(np.sign(corr[w]) * (lm - lam) / nk, rel=1e-6)


# ------------------------------------------------------------- whole-solver pins

def _golden_cases():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_lgcd_matches_brute_force_fixtures(case):
    """The oracle's minimiser equals the enumerated exact Lasso solution."""
    D = np.array(case["D"])
    X = np.array(case["X"])
    lam = case["lam"]
    Z, info = oracle.lgcd(X, D, lam, 1e-14, positive=case["positive"], tile=None)
    assert info["converged"] == 1
    f = oracle.objective(X, D, Z, lam)
    assert f == pytest.approx(case["objective"], rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(Z.ravel(), np.array(case["z"]), atol=1e-9)


@pytest.mark.parametrize("positive", [False, True])
def test_lgcd_matches_brute_force_random(positive):
    for seed in range(20, 26):
        rng = _rng(seed)
        D = _dict(rng, 2, 1, 3)
        X = rng.standard_normal((1, 7))
        A = brute.design_matrix(D, 7)
        lam = 0.2 * float(np.abs(A.T @ X.ravel()).max())
        _, fstar = brute.brute_force_lasso(A, X.ravel(), lam, positive=positive)
        Z, _ = oracle.lgcd(X, D, lam, 1e-14, positive=positive, tile=2)
        assert oracle.objective(X, D, Z, lam) == pytest.approx(fstar, rel=1e-12)


@pytest.mark.parametrize("positive", [False, True])
@pytest.mark.parametrize("oned", [True, False])
def test_lgcd_matches_sklearn_lasso(oned, positive):
    """Cross-check on a few hundred coordinates against sklearn's Lasso run on
    the explicit Toeplitz design (sklearn scales the data term by 1/n)."""
    from sklearn.linear_model import Lasso
    rng = _rng(30 + oned)
    if oned:
        D, T = _dict(rng, 3, 2, 8), 64
        X = rng.standard_normal((2, T))
    else:
        D, T = _dict(rng, 2, 1, (3, 3)), (12, 12)
        X = rng.standard_normal((1,) + T)
    A = brute.design_matrix(D, T)
    y = X.ravel()
    lam = 0.1 * oracle.lambda_max(X, D, positive=positive)
    model = Lasso(alpha=lam / y.size, fit_intercept=False, tol=1e-14, max_iter=200000,
                  positive=positive)
    model.fit(A, y)
    f_sk = brute.lasso_objective(A, y, model.coef_, lam)
    Z, info = oracle.lgcd(X, D, lam, 1e-12 * lam, positive=positive)
    f_or = oracle.objective(X, D, Z, lam)
    assert f_or <= f_sk * (1 + 1e-10)
    assert f_or == pytest.approx(f_sk, rel=1e-9)
    if positive:
        assert (Z >= 0).all()


def test_closed_form_for_single_tap_atoms():
    """K = P = 1 and a 1x1 atom make the design diagonal:
    Z = ST(d X, lambda) / d^2 elementwise."""
    rng = _rng(40)
    d = 0.8
    D = np.full((1, 1, 1, 1), d)
    X = rng.standard_normal((1, 5, 6))
    lam = 0.3
    Z, _ = oracle.lgcd(X, D, lam, 0.0)
    u = d * X[0]
    ref = np.sign(u) * np.maximum(np.abs(u) - lam, 0) / d ** 2
    np.testing.assert_allclose(Z[0], ref, atol=1e-15)


# ----------------------------------------------------- invariants from the paper

def _image_problem(seed, size=24, K=3, L=(4, 4), P=1):
    rng = _rng(seed)
    D = _dict(rng, K, P, L)
    Zt = (rng.random((K, size - L[0] + 1, size - L[1] + 1)) < 0.02) * rng.uniform(0.5, 1.5, (K, size - L[0] + 1, size - L[1] + 1))
    X = sum(np.stack([signal.convolve(Zt[k], D[k, p]) for p in range(P)]) for k in range(K))
    X = X + 0.1 * rng.standard_normal(X.shape)
    return X, D


def test_cost_decrease_prop_a1_sums_to_objective_change():
    """Summing Prop. A.1's Delta E over every update gives F(0) - F(Z)."""
    X, D = _image_problem(50)
    lam = 0.1 * oracle.lambda_max(X, D)
    Z, info = oracle.lgcd(X, D, lam, 1e-10 * lam)
    f0 = oracle.objective(X, D, np.zeros_like(Z), lam)
    f1 = oracle.objective(X, D, Z, lam)
    assert info["cost_decrease"] > 0
    assert f0 - f1 == pytest.approx(info["cost_decrease"], rel=1e-10)


def test_objective_is_monotone_over_sweeps():
    X, D = _image_problem(51)
    lam = 0.1 * oracle.lambda_max(X, D)
    prev = oracle.objective(X, D, np.zeros((3, 21, 21)), lam)
    for s in range(1, 12):
        Z, _ = oracle.lgcd(X, D, lam, 0.0, max_sweeps=s)
        f = oracle.objective(X, D, Z, lam)
        assert f <= prev + 1e-12
        prev = f


def test_incremental_beta_equals_definition():
    """eq. beta_update keeps beta equal to its definition (no drift in FP64)."""
    X, D = _image_problem(52)
    lam = 0.1 * oracle.lambda_max(X, D)
    _, info = oracle.lgcd(X, D, lam, 1e-9 * lam, check_every=1)
    assert info["max_drift"] < 1e-12


def test_certifying_stop_bounds_strict_kkt():
    """With the certifying rule, exit implies strict KKT <= max_k n_k tol / lambda."""
    X, D = _image_problem(53)
    D[0] *= 1.3
    lam = 0.1 * oracle.lambda_max(X, D)
    tol = 1e-4 * lam
    nmax = max(float((D[k] ** 2).sum()) for k in range(3))
    Z, info = oracle.lgcd(X, D, lam, tol, certify=True)
    assert info["converged"] == 1
    assert oracle.kkt(X, D, Z, lam) <= nmax * tol / lam * (1 + 1e-9)
    Zp, _ = oracle.lgcd(X, D, lam, tol, positive=True, certify=True)
    assert (Zp >= 0).all()
    assert oracle.kkt(X, D, Zp, lam, positive=True) <= nmax * tol / lam * (1 + 1e-9)


def test_interference_formula_prop_a2():
    """Simultaneous updates change F by sum of the single-update decreases minus
    C[k_w, k_w', w_w - w_w'] dZ_w dZ_w' summed over unordered pairs."""
    rng = _rng(54)
    X, D = _image_problem(54, size=14, K=2, L=(3, 3))
    lam = 0.05
    H = W = 12
    Z = (rng.random((2, H, W)) < 0.2) * rng.standard_normal((2, H, W))
    beta = oracle.beta(X, D, Z)
    C = oracle.dtd(D)
    n = oracle.atom_norms(D)
    ups = [(0, 5, 5, 0.7), (1, 6, 4, -0.4), (0, 4, 6, 0.3), (1, 9, 9, 0.2)]  # last one far
    f0 = oracle.objective(X, D, Z, lam)
    single = 0.0
    for k, a, b, dz in ups:
        z, zn = Z[k, a, b], Z[k, a, b] + dz
        single += 0.5 * n[k] * (z * z - zn * zn) - beta[k, a, b] * (z - zn) + lam * (abs(z) - abs(zn))
        # Prop. A.1 itself, against a direct evaluation
        Z1 = Z.copy()
        Z1[k, a, b] = zn
        de = 0.5 * n[k] * (z * z - zn * zn) - beta[k, a, b] * (z - zn) + lam * (abs(z) - abs(zn))
        assert f0 - oracle.objective(X, D, Z1, lam) == pytest.approx(de, rel=1e-11, abs=1e-12)
    def lag(ki, kj, u, v):  # C is zero outside Phi = [-L+1, L-1]^2
        return C[ki, kj, u + 2, v + 2] if abs(u) <= 2 and abs(v) <= 2 else 0.0

    inter = 0.0
    for i in range(len(ups)):
        for j in range(i + 1, len(ups)):
            ki, ai, bi, di = ups[i]
            kj, aj, bj, dj = ups[j]
            inter += lag(ki, kj, ai - aj, bi - bj) * di * dj
    assert inter != 0.0
    Zall = Z.copy()
    for k, a, b, dz in ups:
        Zall[k, a, b] += dz
    assert f0 - oracle.objective(X, D, Zall, lam) == pytest.approx(single - inter, rel=1e-11)


def test_softlock_round_simulator_has_no_interference_and_matches_lgcd():
    X, D = _image_problem(55, size=48, K=3, L=(4, 4))
    lam = 0.1 * oracle.lambda_max(X, D)
    tol = 1e-9 * lam
    Zs, _ = oracle.lgcd(X, D, lam, tol)
    Zd, info, log = oracle.dicodile_z(X, D, lam, tol, grid=(5, 5), log_rounds=20)
    assert info["converged"] == 1 and info["n_interfering"] == 0
    assert info["n_softlocked"] > 0  # the test was exercised
    fs, fd = oracle.objective(X, D, Zs, lam), oracle.objective(X, D, Zd, lam)
    assert fd == pytest.approx(fs, rel=1e-10)
    # every logged accepted candidate lies in its worker's sub-domain
    assert log.shape == (20, 25, 4)


def test_without_softlock_updates_interfere():
    """The ablation of Sec. 5: with many workers and no soft-lock, accepted
    updates fall inside each other's neighbourhood."""
    X, D = _image_problem(56, size=48, K=3, L=(4, 4))
    lam = 0.1 * oracle.lambda_max(X, D)
    _, info, _ = oracle.dicodile_z(X, D, lam, 1e-9 * lam, grid=(9, 9), tile=(5, 5),
                                   soft_lock=False, max_rounds=2000, div_guard=1e6)
    assert info["n_interfering"] > 0


def test_one_dimensional_worker_split_matches_lgcd():
    rng = _rng(57)
    D = _dict(rng, 3, 2, 8)
    X = rng.standard_normal((2, 300))
    lam = 0.1 * oracle.lambda_max(X, D)
    Zs, _ = oracle.lgcd(X, D, lam, 1e-10 * lam)
    Zd, info, _ = oracle.dicodile_z(X, D, lam, 1e-10 * lam, grid=6)
    assert info["n_interfering"] == 0 and info["converged"] == 1
    assert oracle.objective(X, D, Zd, lam) == pytest.approx(oracle.objective(X, D, Zs, lam), rel=1e-10)


# ------------------------------------------------------------- dictionary stats

def test_dict_stats_equal_scipy_correlations():
    rng = _rng(60)
    K, P, L, T = 3, 2, (3, 4), (10, 12)
    Z = rng.standard_normal((K, 8, 9)) * (rng.random((K, 8, 9)) < 0.3)
    X = rng.standard_normal((P,) + T)
    phi, psi = oracle.dict_stats(Z, X, L)
    for k in range(K):
        for kk in range(K):
            full = signal.correlate(Z[kk], Z[k], mode="full")  # lag 0 at (7, 8)
            np.testing.assert_allclose(phi[k, kk], full[7 - 2:7 + 3, 8 - 3:8 + 4], atol=1e-13)
        for p in range(P):
            np.testing.assert_allclose(psi[k, p], signal.correlate(X[p], Z[k], mode="valid"),
                                       atol=1e-13)
    np.testing.assert_allclose(phi[np.arange(K), np.arange(K), 2, 3], (Z ** 2).sum(axis=(1, 2)))


def test_dict_gradient_and_cost_from_stats():
    """Sec. 4.2: phi and psi are sufficient for F(D) and its gradient.
    grad = -psi + phi*D, F = 1/2||X||^2 - <D, psi> + 1/2 sum D phi D,
    checked against a direct scipy evaluation and central differences."""
    rng = _rng(61)
    K, P, L, T = 2, 2, (3, 3), (9, 10)
    D = _dict(rng, K, P, L)
    Z = rng.standard_normal((K, 7, 8)) * (rng.random((K, 7, 8)) < 0.4)
    X = rng.standard_normal((P,) + T)
    phi, psi = oracle.dict_stats(Z, X, L)

    def direct_F(Dm):
        R = X - np.stack([sum(signal.convolve(Z[k], Dm[k, p]) for k in range(K)) for p in range(P)])
        return 0.5 * float((R ** 2).sum())

    grad = -psi.copy()
    quad = 0.0
    for k in range(K):
        for kk in range(K):
            for p in range(P):
                for t1 in range(3):
                    for t2 in range(3):
                        for s1 in range(3):
                            for s2 in range(3):
                                c = phi[k, kk, t1 - s1 + 2, t2 - s2 + 2] * D[kk, p, s1, s2]
                                grad[k, p, t1, t2] += c
                                quad += D[k, p, t1, t2] * c
    F = 0.5 * float((X ** 2).sum()) - float((D * psi).sum()) + 0.5 * quad
    assert F == pytest.approx(direct_F(D), rel=1e-12)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 1, 2, 1), (0, 1, 1, 2)]:
        Dp, Dm = D.copy(), D.copy()
        Dp[idx] += h
        Dm[idx] -= h
        fd = (direct_F(Dp) - direct_F(Dm)) / (2 * h)
        assert grad[idx] == pytest.approx(fd, rel=1e-6, abs=1e-8)
