"""Pins of the dictionary-update oracle (Sec. 4.2, eq. dict_update) and of the
alternation of Alg. 2, against quantities fixed independently of it: a direct
evaluation of 1/2||X - Z*D||^2 by scipy convolutions, central differences,
least squares on the explicit convolution design, an independent constrained
solver (scipy SLSQP), and the optimality conditions of the constrained
problem."""
import numpy as np
import pytest
from scipy import optimize, signal

import oracle
from oracle import cdl


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _setup(seed, K, P, L, T, density=0.3, xscale=1.0):
    rng = _rng(seed)
    D = rng.standard_normal((K, P) + L)
    D /= np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1)).reshape((K,) + (1,) * (D.ndim - 1))
    zs = (K,) + tuple(t - l + 1 for t, l in zip(T, L))
    Z = rng.standard_normal(zs) * (rng.random(zs) < density)
    X = xscale * rng.standard_normal((P,) + T)
    return D, Z, X


def _direct_F(X, Z, D):
    K, P = D.shape[:2]
    R = X - np.stack([sum(signal.convolve(Z[k], D[k, p]) for k in range(K)) for p in range(P)])
    return 0.5 * float((R ** 2).sum())


def _design(Z, T, L):
    """Columns: the signal produced by a unit tap (k, t) of one channel."""
    K = Z.shape[0]
    cols = []
    for k in range(K):
        for t in np.ndindex(*L):
            e = np.zeros(L)
            e[t] = 1.0
            cols.append(signal.convolve(Z[k], e).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("dims", ["1d", "2d"])
def test_cost_and_gradient_from_statistics(dims):
    if dims == "1d":
        D, Z, X = _setup(1, 3, 2, (7,), (40,))
    else:
        D, Z, X = _setup(2, 2, 3, (3, 4), (11, 12))
    L = D.shape[2] if D.ndim == 3 else D.shape[2:]
    phi, psi = oracle.dict_stats(Z, X, L)
    x_sq = float((X ** 2).sum())
    assert cdl.dict_cost(D, phi, psi, x_sq) == pytest.approx(_direct_F(X, Z, D), rel=1e-12)
    g = cdl.dict_grad(D, phi, psi)
    h = 1e-6
    rng = _rng(3)
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in D.shape)
        Dp, Dm = D.copy(), D.copy()
        Dp[idx] += h
        Dm[idx] -= h
        fd = (_direct_F(X, Z, Dp) - _direct_F(X, Z, Dm)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_phi_matrix_is_symmetric():
    D, Z, X = _setup(4, 3, 1, (3, 5), (9, 12))
    phi, _ = oracle.dict_stats(Z, X, D.shape[2:])
    M = cdl.phi_matrix(phi, D)
    assert np.allclose(M, M.T, atol=1e-12)


def test_unconstrained_minimiser_is_least_squares():
    """With a small X the least-squares atoms have norms below 1, so the
    constraint is inactive and the update must reach the lstsq solution of the
    explicit convolution design (channel by channel)."""
    D, Z, X = _setup(5, 2, 2, (5,), (60,), density=0.5, xscale=0.05)
    phi, psi = oracle.dict_stats(Z, X, 5)
    A = _design(Z, (60,), (5,))
    sol = np.stack([np.linalg.lstsq(A, X[p], rcond=None)[0] for p in range(2)], axis=1)  # (K*L, P)
    Dls = sol.reshape(2, 5, 2).transpose(0, 2, 1)
    assert np.all(np.sqrt((Dls.reshape(2, -1) ** 2).sum(axis=1)) < 0.9)
    Dn, info = cdl.dict_update(0.5 * D, phi, psi, float((X ** 2).sum()), max_iter=5000, tol=1e-16)
    assert np.allclose(Dn, Dls, atol=1e-7), np.abs(Dn - Dls).max()


def test_constrained_minimiser_matches_slsqp_and_kkt():
    """Active constraints: the update reaches the optimum of an independent
    constrained solver, and satisfies the optimality conditions of
    min F s.t. ||D_k|| <= 1: grad_k = 0 on inactive atoms, and
    grad_k = -mu_k D_k with mu_k >= 0 on atoms at norm 1."""
    D, Z, X = _setup(6, 2, 2, (2, 3), (7, 8), density=0.4, xscale=2.0)
    phi, psi = oracle.dict_stats(Z, X, (2, 3))
    x_sq = float((X ** 2).sum())
    Dn, info = cdl.dict_update(D, phi, psi, x_sq, max_iter=20000, tol=1e-16)
    K = D.shape[0]
    norms = np.sqrt((Dn.reshape(K, -1) ** 2).sum(axis=1))
    assert np.all(norms <= 1 + 1e-12)
    g = cdl.dict_grad(Dn, phi, psi)
    for k in range(K):
        gk, dk = g[k].ravel(), Dn[k].ravel()
        if norms[k] < 1 - 1e-6:
            assert np.linalg.norm(gk) <= 1e-6 * max(1.0, np.abs(psi).max())
        else:
            mu = -float(gk @ dk)
            assert mu >= -1e-9
            assert np.linalg.norm(gk + mu * dk) <= 1e-5 * max(1.0, np.linalg.norm(gk))

    shape = D.shape

    def f(v):
        return _direct_F(X, Z, v.reshape(shape))

    cons = [{"type": "ineq", "fun": (lambda v, k=k: 1.0 - float((v.reshape(shape)[k] ** 2).sum()))}
            for k in range(K)]
    ref = optimize.minimize(f, cdl.project(D).ravel(), method="SLSQP", constraints=cons,
                            options={"ftol": 1e-14, "maxiter": 2000})
    assert ref.success
    assert info["trace"][-1] == pytest.approx(ref.fun, rel=1e-7)


def test_armijo_steps_and_monotone_trace():
    D, Z, X = _setup(7, 3, 2, (6,), (50,), density=0.3)
    phi, psi = oracle.dict_stats(Z, X, 6)
    _, info = cdl.dict_update(D, phi, psi, float((X ** 2).sum()), max_iter=200)
    tr = np.asarray(info["trace"])
    assert np.all(np.diff(tr) <= 1e-12 * np.abs(tr[:-1]))
    assert info["iterations"] >= 1 and len(info["steps"]) == len(tr) - 1


def test_projection():
    rng = _rng(8)
    D = rng.standard_normal((4, 2, 3)) * np.array([0.1, 1.0, 3.0, 10.0]).reshape(4, 1, 1)
    Pd = cdl.project(D)
    n0 = np.sqrt((D.reshape(4, -1) ** 2).sum(axis=1))
    n1 = np.sqrt((Pd.reshape(4, -1) ** 2).sum(axis=1))
    for k in range(4):
        if n0[k] <= 1:
            assert np.array_equal(Pd[k], D[k])
        else:
            assert n1[k] == pytest.approx(1.0, rel=1e-14)
            assert np.allclose(Pd[k] * n0[k], D[k])


def test_alternation_decreases_and_stops():
    """Alg. 2: every block step decreases the objective (the CSC step solves
    for Z at fixed D, the update decreases F at fixed Z), atoms stay feasible
    and the loop stops once the relative decrease falls below nu."""
    rng = _rng(9)
    from paper_1901_09235_amd import synth
    D0 = synth.gaussian_dictionary(rng, 3, 1, 16)
    pb = synth.make_problem("cdl", 910, P=1, T=600, K=3, L=16, rho=0.01, amp="uniform", sigma=0.1, D=D0)
    Dstart = synth.gaussian_dictionary(_rng(11), 3, 1, 16)
    D, Z, info = cdl.cdl(pb.X, Dstart, 0.1, nu=1e-3, max_outer=30)
    costs, zc = info["costs"], info["z_costs"]
    assert len(costs) >= 2
    for q in range(len(costs)):
        assert costs[q] <= zc[q] * (1 + 1e-12)
        if q > 0:
            assert zc[q] <= costs[q - 1] * (1 + 1e-9)
    n = np.sqrt((D.reshape(3, -1) ** 2).sum(axis=1))
    assert np.all(n <= 1 + 1e-12)
    assert info["outer"] == 30 or (costs[-2] - costs[-1]) <= 1e-3 * costs[-2]
