"""FP64 CPU oracle for the dictionary update of DiCoDiLe (Sec. 4.2,
eq. dict_update) and the alternation of Alg. 2.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  The GPU library
never imports it and shares no code with it.

Problem (eq. dict_update):  D* = argmin_{||D_k||_2 <= 1} 1/2 ||X - Z*D||^2.

Sufficient statistics (eq. phi), computed by ``oracle.dict_stats``:
  phi[k, k', tau] = sum_w Z_k[w] Z_k'[w + tau],  tau in Phi = [-L+1, L-1]^d
  psi[k, p, t]    = sum_w Z_k[w] X_p[w + t],      t in Theta
They give the cost and the gradient independently of the signal size
(Sec. 4.2, with the gradient's sign read as in R14):
  F(D)      = 1/2 ||X||^2 - <D, psi> + 1/2 sum_p D_p^T Phi D_p
  grad F(D) = -psi + Phi D,   (Phi D)_{k,p}[t] = sum_{k'} sum_{t'} phi[k, k', t - t'] D_{k',p}[t']
where Phi is the symmetric (K |Theta|) x (K |Theta|) matrix of the quadratic
form, built here explicitly (small problems only).

The update is projected gradient descent with an Armijo backtracking line
search along the projection arc (the paper cites Wright & Nocedal): from
D, try D(a) = Proj(D - a grad F(D)) for a = a0, a0/2, a0/4, ... and accept
the first with F(D(a)) <= F(D) + c1 <grad F(D), D(a) - D>.  Proj scales
every atom with norm above 1 back to the unit sphere.  Reading (R21): c1 =
1e-4; a0 is twice the last accepted step (the first a0 is 1 / the Gershgorin
bound of Phi's largest eigenvalue); stop when an iteration decreases F by
less than tol * max(1, F) or after max_iter iterations.

Alg. 2 alternates the CSC step (here the sequential LGCD of Alg. 1, which
reaches the same minimiser as DiCoDiLe-Z) and the dictionary update, and stops
when the relative decrease of the objective 1/2||X - Z*D||^2 + lambda ||Z||_1
over one outer iteration is below nu.  Reading (R22): lambda is fixed at
lambda_frac * lambda_max(X, D^(0)) for the whole run.
"""
from __future__ import annotations

import numpy as np

import oracle


def _theta(D):
    """Atom tap shape (L1, L2) of D (K, P, L) or (K, P, L1, L2)."""
    return (1, D.shape[2]) if D.ndim == 3 else (D.shape[2], D.shape[3])


def _phi4(phi, D):
    """phi as (K, K, 2L1-1, 2L2-1) whatever the dimension."""
    return phi[:, :, None, :] if D.ndim == 3 else phi


def phi_matrix(phi, D):
    """The matrix Phi[(k, t), (k', t')] = phi[k, k', t - t'] over flattened taps: the
    coefficient of D_{k,p}[t] D_{k',p}[t'] in ||sum_k Z_k * D_{k,p}||^2, since
    sum_x Z_k[x - t] Z_k'[x - t'] = phi[k, k', t - t']."""
    K = D.shape[0]
    L1, L2 = _theta(D)
    ph = _phi4(np.asarray(phi, dtype=np.float64), D)
    t1, t2 = np.meshgrid(np.arange(L1), np.arange(L2), indexing="ij")
    t1, t2 = t1.ravel(), t2.ravel()
    d1 = t1[:, None] - t1[None, :] + L1 - 1  # t - t' (row t, column t'), offset into Phi
    d2 = t2[:, None] - t2[None, :] + L2 - 1
    n = L1 * L2
    M = np.zeros((K * n, K * n))
    for k in range(K):
        for kk in range(K):
            M[k * n:(k + 1) * n, kk * n:(kk + 1) * n] = ph[k, kk][d1, d2]
    return M


def _as_cols(D):
    """D (K, P, taps...) -> (K |Theta|, P): one column per channel."""
    K, P = D.shape[:2]
    return np.ascontiguousarray(D.reshape(K, P, -1).transpose(0, 2, 1).reshape(-1, P))


def _from_cols(C, D):
    K, P = D.shape[:2]
    n = int(np.prod(D.shape[2:]))
    return np.ascontiguousarray(C.reshape(K, n, P).transpose(0, 2, 1).reshape(D.shape))


def dict_cost(D, phi, psi, x_sq, M=None):
    """F(D) from the statistics (Sec. 4.2); x_sq = ||X||^2."""
    M = phi_matrix(phi, D) if M is None else M
    C = _as_cols(D)
    return 0.5 * x_sq - float(np.sum(D * psi)) + 0.5 * float(np.sum(C * (M @ C)))


def dict_grad(D, phi, psi, M=None):
    """grad F(D) = -psi + Phi D (Sec. 4.2, sign as in R14)."""
    M = phi_matrix(phi, D) if M is None else M
    return -np.asarray(psi, dtype=np.float64) + _from_cols(M @ _as_cols(D), D)


def project(D):
    """Every atom with ||D_k||_2 > 1 scaled back to norm 1 (the feasible set of eq. dict_update)."""
    K = D.shape[0]
    n = np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1))
    s = np.where(n > 1.0, 1.0 / np.where(n > 0, n, 1.0), 1.0)
    return D * s.reshape((K,) + (1,) * (D.ndim - 1))


def dict_update(D0, phi, psi, x_sq, max_iter=500, tol=1e-12, c1=1e-4, shrink=0.5):
    """PGD with Armijo backtracking along the projection arc from D0.

    Returns (D, info) with info: iterations, objective trace, accepted steps,
    backtracks."""
    M = phi_matrix(phi, D0)
    D = project(np.asarray(D0, dtype=np.float64))
    f = dict_cost(D, phi, psi, x_sq, M)
    gersh = float(np.max(np.sum(np.abs(M), axis=1)))
    step = 0.5 / gersh if gersh > 0 else 1.0  # doubled before the first trial
    trace, steps, backtracks = [f], [], 0
    for it in range(max_iter):
        g = dict_grad(D, phi, psi, M)
        step *= 2.0
        while True:
            Dn = project(D - step * g)
            fn = dict_cost(Dn, phi, psi, x_sq, M)
            if fn <= f + c1 * float(np.sum(g * (Dn - D))):
                break
            step *= shrink
            backtracks += 1
            if step < 1e-300:
                return D, dict(iterations=it, trace=trace, steps=steps, backtracks=backtracks)
        dec = f - fn
        D, f = Dn, fn
        trace.append(f)
        steps.append(step)
        if dec <= tol * max(1.0, abs(f)):
            return D, dict(iterations=it + 1, trace=trace, steps=steps, backtracks=backtracks)
    return D, dict(iterations=max_iter, trace=trace, steps=steps, backtracks=backtracks)


def cdl(X, D0, lambda_frac, nu=1e-4, max_outer=20, tol_rel=1e-8, dict_max_iter=500):
    """Alg. 2 on one core: CSC step (Alg. 1) then dictionary update, until the
    relative decrease of the objective over an outer iteration is below nu.

    Returns (D, Z, info) with the objective after each outer iteration."""
    X = np.asarray(X, dtype=np.float64)
    D = project(np.asarray(D0, dtype=np.float64))
    lam = lambda_frac * oracle.lambda_max(X, D)
    L = D.shape[2] if D.ndim == 3 else (D.shape[2], D.shape[3])
    x_sq = float(np.sum(X * X))
    costs, z_costs = [], []
    Z = None
    for q in range(max_outer):
        Z, _ = oracle.lgcd(X, D, lam, tol_rel * lam)
        z_costs.append(oracle.objective(X, D, Z, lam))
        phi, psi = oracle.dict_stats(Z, X, L)
        D, _ = dict_update(D, phi, psi, x_sq, max_iter=dict_max_iter)
        costs.append(oracle.objective(X, D, Z, lam))
        if q > 0 and (costs[-2] - costs[-1]) <= nu * abs(costs[-2]):
            break
    return D, Z, dict(lam=lam, costs=costs, z_costs=z_costs, outer=len(costs))
