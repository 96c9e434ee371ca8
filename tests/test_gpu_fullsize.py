"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses, on outputs the oracle can compute one by one.

The oracle cannot solve these problems in test time, so each GPU solution Z
is checked through quantities that certify it at any size:
  * the FP64 objective 1/2||X - Z*D||^2 + lambda ||Z||_1 recomputed by the
    oracle's reconstruction (Z*D over the whole image or signal);
  * the gradient g = corr(X - Z*D, D) at sampled coordinates (random ones and
    random non-zeros), each from its own window of the oracle's residual, and
    the strict KKT conditions there (|g| <= lambda on zeros, g = lambda sign z
    on the support, to 1e-4 lambda);
  * the GPU's own FP64 report of both, which must agree with the oracle's.
lambda is 0.1 x the oracle's lambda_max of a 256-wide crop (the full-size
lambda_max is a dense correlation the oracle cannot afford here), so it never
comes from the GPU path."""
import numpy as np
import pytest

import oracle
from paper_1901_09235_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

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


def _crop_lambda(X, D, frac=0.1, side=256):
    if X.ndim == 2:
        return frac * oracle.lambda_max(X[:, :max(side * 8, D.shape[2])], D)
    return frac * oracle.lambda_max(X[:, :side, :side], D)


def _sampled_check(X, D, Z, lam, info, rng, n_rand=3000, n_nz=3000):
    """Oracle objective and sampled strict KKT of a GPU solution Z (FP64)."""
    is_1d = X.ndim == 2
    T = X.shape[1] if is_1d else X.shape[1:]
    R = X - oracle.reconstruct(Z, D, T)
    obj = 0.5 * float(np.sum(R * R)) + lam * float(np.abs(Z).sum())
    assert info["objective"] == pytest.approx(obj, rel=1e-9)
    X3 = R[:, None, :] if is_1d else R
    D4 = D[:, :, None, :] if is_1d else D
    Z3 = Z[:, None, :] if is_1d else Z
    K, P, L1, L2 = D4.shape
    H, W = Z3.shape[1:]
    ks = rng.integers(0, K, n_rand)
    hs = rng.integers(0, H, n_rand)
    ws = rng.integers(0, W, n_rand)
    nz = np.flatnonzero(Z3)
    if nz.size:
        pick = rng.choice(nz, size=min(n_nz, nz.size), replace=False)
        k2, r2 = np.divmod(pick, H * W)
        h2, w2 = np.divmod(r2, W)
        ks, hs, ws = np.concatenate([ks, k2]), np.concatenate([hs, h2]), np.concatenate([ws, w2])
    t1 = np.arange(L1)[None, :, None]
    t2 = np.arange(L2)[None, None, :]
    worst = 0.0
    for s in range(0, ks.size, 1000):
        sl = slice(s, s + 1000)
        win = X3[:, hs[sl, None, None] + t1, ws[sl, None, None] + t2]  # (P, S, L1, L2)
        g = np.einsum("pstu,sptu->s", win, D4[ks[sl]])
        z = Z3[ks[sl], hs[sl], ws[sl]]
        viol = np.where(z == 0, np.maximum(np.abs(g) - lam, 0.0), np.abs(g - lam * np.sign(z)))
        worst = max(worst, float(viol.max()) / lam)
    assert worst <= 1e-4, worst
    assert worst <= info["kkt"] * (1 + 1e-6) + 1e-12
    return worst


def test_image_1024_full_size(lib):
    pb = synth.image_1024()
    X = pb.X.astype(np.float32).astype(np.float64)
    D = pb.D.astype(np.float32).astype(np.float64)
    lam = _crop_lambda(X, D)
    z, info = lib.dicodile_csc(dev(X, torch.float32), dev(D, torch.float32), lam, 1e-5 * lam,
                               max_rounds=50_000_000, timeout_s=120.0)
    assert info["status"] == "OK", info
    assert info["kkt"] <= 1e-4
    _sampled_check(X, D, z.double().cpu().numpy(), lam, info, np.random.default_rng(1))


def test_image_rgb_4096_full_size(lib):
    pb = synth.image_4096_rgb()
    X = pb.X.astype(np.float32).astype(np.float64)
    D = pb.D.astype(np.float32).astype(np.float64)
    lam = _crop_lambda(X, D)
    z, info = lib.dicodile_csc(dev(X, torch.float32), dev(D, torch.float32), lam, 1e-5 * lam,
                               max_rounds=50_000_000, timeout_s=120.0)
    assert info["status"] == "OK", info
    Z = z.double().cpu().numpy()
    del z
    _sampled_check(X, D, Z, lam, info, np.random.default_rng(2))


def test_signal_1d_full_size_matches_oracle_solution(lib):
    """The 1-D workload is small enough for the oracle's own solve: the GPU
    (FP64, the benchmark's grid) reaches its objective to 1e-12."""
    pb = synth.signal_1d()
    lam = pb.lambda_frac * oracle.lambda_max(pb.X, pb.D)
    z, info = lib.dicodile_csc(dev(pb.X, torch.float64), dev(pb.D, torch.float64), lam, pb.tol_rel,
                               max_rounds=50_000_000, timeout_s=60.0)
    assert info["status"] == "OK"
    Zo, _ = oracle.lgcd(pb.X, pb.D, lam, pb.tol_rel)
    fo = oracle.objective(pb.X, pb.D, Zo, lam)
    assert info["objective"] == pytest.approx(fo, rel=1e-12)


def test_serving_requests_full_length(lib):
    """Requests of the serving recipe at their full lengths (the longest of the
    first 48 and two others), through the server."""
    D = synth.serving_dictionary()
    pbs = [synth.serving_request(j, D) for j in (14, 3, 20)]  # T = 491641, 21594, 24569
    Dd = dev(D, torch.float32)
    D32 = D.astype(np.float32).astype(np.float64)
    with lib.Server(Dd, max_len=max(pb.X.shape[1] for pb in pbs)) as srv:
        items = []
        for pb in pbs:
            X = pb.X.astype(np.float32).astype(np.float64)
            lam = _crop_lambda(X, D32, frac=0.2)
            Xd = dev(X, torch.float32)
            torch.cuda.synchronize()
            items.append((X, lam, Xd, srv.submit(Xd, lam, 1e-5 * lam, timeout_s=60)))
        for X, lam, Xd, t in items:
            z, info = srv.wait(t, timeout_s=120)
            assert info["status"] == "OK", info
            _sampled_check(X, D32, z.double().cpu().numpy(), lam, info, np.random.default_rng(3))


def test_batch_images_full_size_sampled(lib):
    """The full 256-image batch in one launch (the benchmark's call), with the
    sampled certificate on four instances spread over the sizes."""
    D, pbs = synth.batch_images()
    Dd = dev(D, torch.float32)
    D32 = D.astype(np.float32).astype(np.float64)
    Xs, lams = [], []
    for pb in pbs:
        X = pb.X.astype(np.float32).astype(np.float64)
        Xs.append(X)
        lams.append(_crop_lambda(X, D32, side=128))
    zs, infos, binfo = lib.dicodile_csc_batch([dev(X, torch.float32) for X in Xs], Dd, lams,
                                              [1e-5 * l for l in lams])
    assert binfo["n_converged"] == len(pbs), binfo
    order = np.argsort([X.shape[1] * X.shape[2] for X in Xs])
    for i in order[[0, 85, 170, 255]]:
        _sampled_check(Xs[i], D32, zs[i].double().cpu().numpy(), lams[i], infos[i],
                       np.random.default_rng(10 + int(i)), n_rand=1000, n_nz=1000)
