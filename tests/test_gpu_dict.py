"""The dictionary update (eq. dict_update) and the alternation of Alg. 2 on the
GPU against the FP64 oracle of the same steps (oracle/cdl.py)."""
import numpy as np
import pytest

import oracle
from oracle import cdl
from paper_1901_09235_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_09235_amd as dl
    dl.load()
    return dl


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _stats_case(seed, K, P, L, T, density=0.3, xscale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    D = rng.standard_normal((K, P) + L)
    D /= np.sqrt((D.reshape(K, -1) ** 2).sum(axis=1)).reshape((K,) + (1,) * (D.ndim - 1))
    zs = (K,) + tuple(t - l + 1 for t, l in zip(T, L))
    Z = rng.standard_normal(zs) * (rng.random(zs) < density)
    X = xscale * rng.standard_normal((P,) + T)
    Lp = L[0] if len(L) == 1 else L
    phi, psi = oracle.dict_stats(Z, X, Lp)
    return D, phi, psi, float((X ** 2).sum())


@pytest.mark.parametrize("case", ["1d", "2d", "1d_inactive"])
def test_dict_update_matches_oracle(lib, case):
    """From the same FP64 statistics and start, the GPU update reaches the
    oracle's constrained optimum: the same cost (1e-9 relative) and the
    constrained optimality conditions evaluated by the oracle's gradient."""
    if case == "1d":
        D, phi, psi, x_sq = _stats_case(21, 4, 3, (9,), (80,))
    elif case == "2d":
        D, phi, psi, x_sq = _stats_case(22, 3, 2, (4, 5), (14, 15))
    else:
        D, phi, psi, x_sq = _stats_case(23, 2, 2, (5,), (60,), density=0.5, xscale=0.05)
    Do, io = cdl.dict_update(D, phi, psi, x_sq, max_iter=20000, tol=1e-15)
    Dg = dev(D, torch.float64)
    info = lib.dicodile_dict_update(dev(phi, torch.float64), dev(psi, torch.float64), x_sq, Dg,
                                    max_iter=20000, tol=1e-15)
    assert info["cost_initial"] == pytest.approx(io["trace"][0], rel=1e-12)
    assert info["cost"] == pytest.approx(io["trace"][-1], rel=1e-9)
    Dn = Dg.cpu().numpy()
    assert cdl.dict_cost(Dn, phi, psi, x_sq) == pytest.approx(info["cost"], rel=1e-12)
    K = D.shape[0]
    norms = np.sqrt((Dn.reshape(K, -1) ** 2).sum(axis=1))
    assert np.all(norms <= 1 + 1e-12)
    g = cdl.dict_grad(Dn, phi, psi)
    for k in range(K):
        gk, dk = g[k].ravel(), Dn[k].ravel()
        if norms[k] < 1 - 1e-6:
            assert np.linalg.norm(gk) <= 1e-5 * max(1.0, np.abs(psi).max())
        else:
            mu = -float(gk @ dk)
            assert mu >= -1e-7
            assert np.linalg.norm(gk + mu * dk) <= 1e-4 * max(1.0, np.linalg.norm(gk))


def test_dict_update_fp32_statistics(lib):
    D, phi, psi, x_sq = _stats_case(24, 3, 2, (7,), (70,))
    phi32, psi32 = phi.astype(np.float32).astype(np.float64), psi.astype(np.float32).astype(np.float64)
    _, io = cdl.dict_update(D.astype(np.float32).astype(np.float64), phi32, psi32, x_sq, max_iter=20000, tol=1e-15)
    Dg = dev(D, torch.float32)
    info = lib.dicodile_dict_update(dev(phi32, torch.float32), dev(psi32, torch.float32), x_sq, Dg,
                                    max_iter=20000, tol=1e-15)
    assert info["cost"] == pytest.approx(io["trace"][-1], rel=1e-7)


def test_cdl_alternation_matches_oracle(lib):
    """Alg. 2 on a small multichannel signal: the GPU alternation (FP64)
    follows the oracle's: the same lambda, and per outer iteration the same
    objective after the CSC step and after the dictionary update."""
    D0 = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(31)), 3, 2, 16)
    pb = synth.make_problem("cdl", 3100, P=2, T=700, K=3, L=16, rho=0.01, amp="uniform", sigma=0.1, D=D0)
    Dstart = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(32)), 3, 2, 16)
    Do, Zo, io = cdl.cdl(pb.X, Dstart, 0.1, nu=1e-3, max_outer=8, tol_rel=1e-10)
    Dg = dev(Dstart, torch.float64)
    z, info = lib.dicodile_cdl(dev(pb.X, torch.float64), Dg, lambda_frac=0.1, nu=1e-3, max_outer=8,
                               tol_rel=1e-10, dict_max_iter=500, dict_tol=1e-12, timeout_s=60)
    assert info["lambda"] == pytest.approx(io["lam"], rel=1e-12)
    n = min(info["outer"], io["outer"])
    assert n >= 2
    for q in range(n):
        assert info["objective_z"][q] == pytest.approx(io["z_costs"][q], rel=1e-6), q
        assert info["objective"][q] == pytest.approx(io["costs"][q], rel=1e-6), q
    # the objective never increases across block steps
    for q in range(info["outer"]):
        assert info["objective"][q] <= info["objective_z"][q] * (1 + 1e-12)
        if q:
            assert info["objective_z"][q] <= info["objective"][q - 1] * (1 + 1e-9)
    Dn = Dg.cpu().numpy()
    assert np.all(np.sqrt((Dn.reshape(3, -1) ** 2).sum(axis=1)) <= 1 + 1e-12)


def test_cdl_fp32_image(lib):
    """FP32 alternation on a small image: finite, feasible, non-increasing."""
    D0 = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(33)), 4, 1, (6, 6))
    pb = synth.make_problem("cdl2", 3300, P=1, T=(60, 64), K=4, L=(6, 6), rho=0.01, amp="uniform", sigma=0.1, D=D0)
    Dstart = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(34)), 4, 1, (6, 6))
    Dg = dev(Dstart, torch.float32)
    z, info = lib.dicodile_cdl(dev(pb.X, torch.float32), Dg, lambda_frac=0.1, nu=1e-3, max_outer=6, timeout_s=60)
    assert info["outer"] >= 2
    obj = np.asarray(info["objective"])
    assert np.all(np.isfinite(obj)) and np.all(np.diff(obj) <= 1e-5 * obj[:-1])
    Dn = Dg.double().cpu().numpy()
    assert np.all(np.sqrt((Dn.reshape(4, -1) ** 2).sum(axis=1)) <= 1 + 1e-6)
