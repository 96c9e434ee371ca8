"""Pins of the oracle's full-size tools (``oracle/large.py``): the FFT
correlation and beta against the direct FP64 loops (themselves pinned to
scipy.signal), the KKT from g against the C grader (pinned two-sided), the
duality gap against the brute-force Lasso optimum, and the warm-started
polish against the objective and a cold solve."""
import numpy as np
import pytest
from scipy import signal

import oracle
from oracle import brute, large


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _dict(rng, K, P, L):
    shape = (K, P) + (tuple(L) if isinstance(L, tuple) else (L,))
    D = rng.standard_normal(shape)
    return D / np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1)).reshape((K,) + (1,) * (D.ndim - 1))


CASES = {
    "1d_short": (2, 3, 5, 23),
    "1d_long": (3, 4, 64, 1000),
    "2d": (2, 3, (3, 4), (9, 11)),
    "2d_ragged": (3, 2, (5, 7), (31, 17)),
}


def _case(name, seed):
    P, K, L, T = CASES[name]
    rng = _rng(seed)
    D = _dict(rng, K, P, L)
    X = rng.standard_normal((P,) + (T if isinstance(T, tuple) else (T,)))
    zs = (K,) + tuple(t - l + 1 for t, l in zip(T if isinstance(T, tuple) else (T,),
                                                 L if isinstance(L, tuple) else (L,)))
    Z = rng.standard_normal(zs) * (rng.random(zs) < 0.2)
    return X, D, Z


@pytest.mark.parametrize("name", sorted(CASES))
def test_corr_fft_equals_direct_loops(name):
    X, D, _ = _case(name, 200)
    G = oracle.corr(X, D)
    Gf = large.corr_fft(X, D)
    assert Gf.shape == G.shape
    np.testing.assert_allclose(Gf, G, rtol=0, atol=1e-12 * np.abs(G).max())


def test_corr_fft_equals_scipy_on_one_channel():
    rng = _rng(201)
    D = _dict(rng, 1, 1, (6, 5))
    R = rng.standard_normal((1, 40, 33))
    ref = signal.correlate(R[0], D[0, 0], mode="valid")
    np.testing.assert_allclose(large.corr_fft(R, D)[0], ref, atol=1e-12)


@pytest.mark.parametrize("name", sorted(CASES))
def test_beta_fft_equals_definition(name):
    X, D, Z = _case(name, 202)
    b = oracle.beta(X, D, Z)
    np.testing.assert_allclose(large.beta_fft(X, D, Z), b, rtol=0, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("positive", [False, True])
@pytest.mark.parametrize("name", ["1d_short", "2d_ragged"])
def test_kkt_from_g_equals_the_c_grader(name, positive):
    X, D, Z = _case(name, 203)
    if positive:
        Z = np.abs(Z)
    b = large.beta_fft(X, D, Z)
    g = b - oracle.atom_norms(D).reshape((-1,) + (1,) * (Z.ndim - 1)) * Z
    for lam in (0.05, 0.3, 1.0):
        assert large.kkt_from_g(g, Z, lam, positive) == pytest.approx(oracle.kkt(X, D, Z, lam, positive),
                                                                      rel=1e-10, abs=1e-12)
        assert large.dual_gap(X, D, Z, lam, positive)["kkt"] == pytest.approx(
            oracle.kkt(X, D, Z, lam, positive), rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("positive", [False, True])
def test_dual_gap_bounds_the_brute_force_suboptimality(positive):
    """Weak duality: gap(Z) >= F(Z) - F* >= 0 at any Z, and gap = 0 (to
    rounding) at the exact minimiser from enumeration."""
    rng = _rng(204)
    D = _dict(rng, 2, 1, 3)
    T = 7
    X = rng.standard_normal((1, T))
    A = brute.design_matrix(D, T)
    lam = 0.25 * float(np.abs(A.T @ X.ravel()).max())
    zs, fstar = brute.brute_force_lasso(A, X.ravel(), lam, positive=positive)
    d0 = large.dual_gap(X, D, zs.reshape(2, 5), lam, positive)
    assert d0["primal"] == pytest.approx(fstar, rel=1e-12)
    assert abs(d0["gap"]) <= 1e-10 * fstar
    for _ in range(20):
        Z = rng.standard_normal((2, 5)) * (rng.random((2, 5)) < 0.5)
        if positive:
            Z = np.abs(Z)
        d = large.dual_gap(X, D, Z, lam, positive)
        f = oracle.objective(X, D, Z, lam)
        assert d["primal"] == pytest.approx(f, rel=1e-12)
        assert d["gap"] >= f - fstar - 1e-12 * fstar


def test_polish_decrease_and_bound():
    """From a perturbed minimiser, the polish's summed Prop. A.1 decrease is
    F(Z0) - F(Z_pol); Z_pol meets a cold oracle solve; bound >= F(Z0) - F*;
    beta from beta_fft gives the same run as the direct loops."""
    rng = _rng(205)
    D = _dict(rng, 3, 2, (4, 4))
    Zt = (rng.random((3, 29, 27)) < 0.02) * rng.uniform(0.5, 1.5, (3, 29, 27))
    X = np.stack([sum(signal.convolve(Zt[k], D[k, p]) for k in range(3)) for p in range(2)])
    X += 0.1 * rng.standard_normal(X.shape)
    lam = 0.1 * oracle.lambda_max(X, D)
    Zc, _ = oracle.lgcd(X, D, lam, 1e-12 * lam)
    fstar = oracle.objective(X, D, Zc, lam)
    Z0 = Zc * (1 + 0.01 * rng.standard_normal(Zc.shape))
    Z0[0, 3, 4] += 0.05  # a spurious non-zero
    f0 = oracle.objective(X, D, Z0, lam)
    res = large.polish(X, D, Z0, lam, tol_rel=1e-10, tile=None, sweeps_per_chunk=3)
    assert res["converged"] == 1
    # one-position sub-domains (the default) reach the same minimiser
    res1 = large.polish(X, D, Z0, lam, tol_rel=1e-10)
    assert res1["f_polished"] == pytest.approx(fstar, rel=1e-11)
    assert res1["decrease"] == pytest.approx(f0 - res1["f_polished"], rel=1e-9)
    assert res["f0"] == pytest.approx(f0, rel=1e-14)
    assert res["decrease"] == pytest.approx(f0 - oracle.objective(X, D, res["Z"], lam), rel=1e-9)
    assert res["f_polished"] == pytest.approx(fstar, rel=1e-11)
    assert res["bound"] >= f0 - fstar - 1e-10 * fstar
    assert res["rel_bound"] == pytest.approx((f0 - fstar) / f0, rel=1e-3)
    Zd, _ = oracle.lgcd(X, D, lam, 1e-10 * lam, z0=Z0)
    np.testing.assert_allclose(res["Z"], Zd, atol=1e-9)
