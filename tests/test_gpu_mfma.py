"""The matrix-core correlation G = corr(X, D) in each precision against the
FP64 oracle, element by element, within error bounds derived from the
arithmetic of each path (absC = corr(|X|, |D|), n = P L1 L2 terms):

  F64     products and sums in FP64:           |err| <= 2 n 2^-53 absC
  BF16    operands rounded to BF16 (2^-9 each), FP32 sums:
                                               |err| <= (2^-8 + n 2^-23) absC
  BF16X3  hi/lo splits, hi*hi + hi*lo + lo*hi: each product off by at most
          |xl dl| + the split remainders (<= 3 2^-17 relative), FP32 sums:
                                               |err| <= (3 2^-17 + 3 n 2^-23) absC
  DIRECT  FP32 (or FP64) FMA chain:            |err| <= n 2^-23 absC (2^-52)

Shapes span several workgroup tiles with ragged tails, atom counts above 64
(two atom groups), channel counts that are padded (P = 3, 5) and taps that
are padded (L = 250, 12)."""
import numpy as np
import pytest

import oracle
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


CASES = {
    # name: (P, T, K, L)
    "serving_like": (32, 1000, 40, 128),
    "signal_p1": (1, 3000, 5, 64),
    "paper_1d": (7, 1400, 25, 250),
    "atoms70": (2, 700, 70, 20),
    "image_p1": (1, (70, 83), 25, (16, 16)),
    "rgb": (3, (75, 90), 25, (32, 32)),
    "image_p5_L12": (5, (41, 150), 16, (12, 12)),
}


def _case(name, seed=5):
    P, T, K, L = CASES[name]
    rng = np.random.Generator(np.random.PCG64(seed))
    D = synth.gaussian_dictionary(rng, K, P, L)
    shape = (P, T) if isinstance(T, int) else (P,) + tuple(T)
    X = rng.standard_normal(shape)
    return X, D


def _bound(prec, n, absC):
    u = 2.0 ** -53
    if prec == "f64":
        return 2 * n * u * absC + 1e-300
    if prec == "bf16":
        return (2.0 ** -8 + n * 2.0 ** -23) * absC
    if prec == "bf16x3":
        return (3 * 2.0 ** -17 + 3 * n * 2.0 ** -23) * absC
    return n * 2.0 ** -23 * absC


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "bf16", "bf16x3", "direct"])
def test_corr_fp32_data_within_bound(lib, name, prec):
    X, D = _case(name)
    X32, D32 = X.astype(np.float32).astype(np.float64), D.astype(np.float32).astype(np.float64)
    G = lib.dicodile_corr(dev(X32, torch.float32), dev(D32, torch.float32), prec=prec).double().cpu().numpy()
    ref = oracle.corr(X32, D32)
    absC = oracle.corr(np.abs(X32), np.abs(D32))
    n = D.size // D.shape[0]
    # the FP32 output rounding adds 2^-24 |G|
    bound = _bound(prec, n, absC) + 2.0 ** -24 * np.abs(ref)
    err = np.abs(G - ref)
    assert G.shape == ref.shape
    assert np.all(err <= bound), (name, prec, float(np.max(err / np.maximum(absC, 1e-300))))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "direct"])
def test_corr_fp64_data_within_bound(lib, name, prec):
    X, D = _case(name, seed=6)
    G = lib.dicodile_corr(dev(X, torch.float64), dev(D, torch.float64), prec=prec).cpu().numpy()
    ref = oracle.corr(X, D)
    absC = oracle.corr(np.abs(X), np.abs(D))
    n = D.size // D.shape[0]
    err = np.abs(G - ref)
    assert np.all(err <= 2 * n * 2.0 ** -53 * absC + 1e-300), (name, prec)


def test_bf16_is_rejected_for_fp64_data(lib):
    X, D = _case("signal_p1")
    with pytest.raises(lib.DicodileError):
        lib.dicodile_corr(dev(X, torch.float64), dev(D, torch.float64), prec="bf16")


@pytest.mark.parametrize("beta_prec", ["f64", "bf16", "bf16x3", "direct"])
def test_solve_reaches_oracle_with_each_init_precision(lib, beta_prec):
    """Whatever contraction initialises beta, the FP32 solve ends at the
    oracle's minimiser: a BF16 start is corrected by the FP64 drift pass."""
    D = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(9)), 8, 4, 32)
    pb = synth.make_problem("p", 901, P=4, T=4000, K=8, L=32, rho=0.004, amp="exp", sigma=0.1, D=D)
    X = pb.X.astype(np.float32).astype(np.float64)
    Dd = D.astype(np.float32).astype(np.float64)
    lam = 0.1 * oracle.lambda_max(X, Dd)
    z, info = lib.dicodile_csc(dev(X, torch.float32), dev(Dd, torch.float32), lam, 1e-5 * lam,
                               beta_prec=beta_prec, max_polish=4, timeout_s=60)
    assert info["status"] == "OK", info
    Zo, _ = oracle.lgcd(X, Dd, lam, 1e-10 * lam)
    fo = oracle.objective(X, Dd, Zo, lam)
    fg = oracle.objective(X, Dd, z.double().cpu().numpy(), lam)
    assert (fg - fo) / fo <= 1e-6
    assert oracle.kkt(X, Dd, z.double().cpu().numpy(), lam) <= 1e-4


def test_beta_drift_is_reported_and_orders_by_precision(lib):
    """info['beta_drift'] is the distance, in units of lambda, between the beta
    kept by the rounds and its FP64 definition at the first check: finite for
    every initialisation, and larger for a BF16 start than for FP64 or split
    BF16 starts."""
    D = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(10)), 8, 4, 32)
    pb = synth.make_problem("p", 902, P=4, T=6000, K=8, L=32, rho=0.004, amp="exp", sigma=0.1, D=D)
    X = dev(pb.X, torch.float32)
    Dd = dev(D, torch.float32)
    lam = 0.1 * oracle.lambda_max(pb.X.astype(np.float32).astype(np.float64), D.astype(np.float32).astype(np.float64))
    drift = {}
    for prec in ("f64", "bf16x3", "bf16"):
        _, info = lib.dicodile_csc(X, Dd, lam, 1e-5 * lam, beta_prec=prec, max_polish=4, timeout_s=60)
        assert info["status"] == "OK"
        drift[prec] = info["beta_drift"]
    assert all(np.isfinite(v) and v >= 0 for v in drift.values()), drift
    assert drift["bf16"] > drift["bf16x3"] and drift["bf16"] > drift["f64"], drift
    assert drift["f64"] < 1e-3 and drift["bf16x3"] < 1e-2, drift


@pytest.mark.parametrize("beta_prec", ["bf16", "f64"])
def test_periodic_refresh_reaches_oracle(lib, beta_prec):
    """refresh_every rebuilds beta from its FP64 definition between chunks of
    rounds (whatever contraction initialised it); the solve still certifies
    and meets the oracle's objective."""
    D = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(11)), 6, 2, 24)
    pb = synth.make_problem("p", 903, P=2, T=5000, K=6, L=24, rho=0.005, amp="uniform", sigma=0.1, D=D)
    X = pb.X.astype(np.float32).astype(np.float64)
    Dd = D.astype(np.float32).astype(np.float64)
    lam = 0.1 * oracle.lambda_max(X, Dd)
    z, info = lib.dicodile_csc(dev(X, torch.float32), dev(Dd, torch.float32), lam, 1e-5 * lam,
                               beta_prec=beta_prec, refresh_every=2, grid=4, max_polish=4, timeout_s=60)
    assert info["status"] == "OK", info
    Zo, _ = oracle.lgcd(X, Dd, lam, 1e-10 * lam)
    fo = oracle.objective(X, Dd, Zo, lam)
    fg = oracle.objective(X, Dd, z.double().cpu().numpy(), lam)
    assert (fg - fo) / fo <= 1e-6


def test_single_drift_correction_after_bf16_start(lib):
    """The precision pattern of the large image: a BF16 matrix-core start,
    one FP64 drift correction after two sweeps (refresh_limit = 1), the FP64
    check.  The correction and every check are FP64 contractions (counted and
    timed in info); the result meets the oracle's objective and strict KKT."""
    D = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(12)), 6, 3, (8, 8))
    pb = synth.make_problem("p", 904, P=3, T=(72, 80), K=6, L=(8, 8), rho=0.004, amp="exp", sigma=0.05, D=D)
    X = pb.X.astype(np.float32).astype(np.float64)
    Dd = D.astype(np.float32).astype(np.float64)
    lam = 0.1 * oracle.lambda_max(X, Dd)
    z, info = lib.dicodile_csc(dev(X, torch.float32), dev(Dd, torch.float32), lam, 1e-5 * lam,
                               beta_prec="bf16", refresh_every=2, refresh_limit=1, grid=(3, 3), timeout_s=60,
                               fp64_method="mfma")
    assert info["status"] == "OK", info
    assert info["init_prec"] == 2 and info["t_init_corr_s"] > 0 and info["n_fft64"] == 0
    # the one correction (a dense FP64 contraction), then one check per pass
    # after it, each carried forward from the correction's FP64 gradient
    assert info["n_corr64"] == 1 and info["n_check_inc"] == info["n_passes"] - 1, info
    assert info["t_corr64_s"] > 0
    Zo, _ = oracle.lgcd(X, Dd, lam, 1e-10 * lam)
    fo = oracle.objective(X, Dd, Zo, lam)
    Zg = z.double().cpu().numpy()
    assert (oracle.objective(X, Dd, Zg, lam) - fo) / fo <= 1e-6
    assert oracle.kkt(X, Dd, Zg, lam) <= 1e-4


def test_failed_check_rebuilds_beta_in_the_same_contraction(lib):
    """A check that fails (here: a BF16 start and no earlier correction, so
    the first pass converges on a perturbed beta) rebuilds beta from the FP64
    contraction it has just run, and the polish pass's check is carried
    forward from it: one FP64 contraction for the whole solve, and the
    polished result meets the oracle."""
    D = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(13)), 5, 2, 40)
    pb = synth.make_problem("p", 905, P=2, T=8000, K=5, L=40, rho=0.005, amp="exp", sigma=0.1, D=D)
    X = pb.X.astype(np.float32).astype(np.float64)
    Dd = D.astype(np.float32).astype(np.float64)
    lam = 0.1 * oracle.lambda_max(X, Dd)
    z, info = lib.dicodile_csc(dev(X, torch.float32), dev(Dd, torch.float32), lam, 1e-5 * lam,
                               beta_prec="bf16", grid=6, max_polish=4, timeout_s=60)
    assert info["status"] == "OK", info
    # the first (dense) check fails and is the FP64 reference of the polish
    # pass's check, which carries its gradient forward
    assert info["n_passes"] >= 2 and info["n_corr64"] == 1, info
    assert info["n_check_inc"] == info["n_passes"] - 1, info
    Zo, _ = oracle.lgcd(X, Dd, lam, 1e-10 * lam)
    fo = oracle.objective(X, Dd, Zo, lam)
    Zg = z.double().cpu().numpy()
    assert (oracle.objective(X, Dd, Zg, lam) - fo) / fo <= 1e-6
    assert oracle.kkt(X, Dd, Zg, lam) <= 1e-4


@pytest.mark.parametrize("positive", [False, True])
def test_incremental_check_equals_the_dense_check(lib, positive):
    """After the one drift correction (on the matrix cores: the incremental
    check follows the matrix-core contraction only), the final check carries
    that FP64 contraction's gradient and residual forward over the
    coordinates changed since (info n_check_inc); its objective and strict
    KKT equal a dense FP64 check of the returned z (dicodile_objective_kkt)
    and the oracle's."""
    D = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(14)), 7, 2, (9, 7))
    pb = synth.make_problem("p", 906, P=2, T=(90, 77), K=7, L=(9, 7), rho=0.004, amp="exp", sigma=0.05, D=D)
    X = pb.X.astype(np.float32).astype(np.float64)
    Dd = D.astype(np.float32).astype(np.float64)
    lam = 0.1 * oracle.lambda_max(X, Dd, positive=positive)
    Xt, Dt = dev(X, torch.float32), dev(Dd, torch.float32)
    z, info = lib.dicodile_csc(Xt, Dt, lam, 1e-5 * lam, positive=positive, beta_prec="bf16", refresh_every=2,
                               refresh_limit=1, grid=(3, 3), timeout_s=60, fp64_method="mfma")
    assert info["status"] == "OK", info
    assert info["n_check_inc"] >= 1 and info["t_check_inc_s"] > 0, info
    assert info["n_corr64"] == 1, info  # the drift correction only
    f_dense, k_dense = lib.dicodile_objective_kkt(Xt, Dt, z, lam, positive=positive)
    assert info["objective"] == pytest.approx(f_dense, rel=1e-10)
    assert info["kkt"] == pytest.approx(k_dense, rel=1e-6, abs=1e-10)
    Zg = z.double().cpu().numpy()
    assert oracle.objective(X, Dd, Zg, lam) == pytest.approx(info["objective"], rel=1e-9)
    assert oracle.kkt(X, Dd, Zg, lam, positive=positive) == pytest.approx(info["kkt"], rel=1e-6, abs=1e-10)
    Zo, _ = oracle.lgcd(X, Dd, lam, 1e-10 * lam, positive=positive)
    fo = oracle.objective(X, Dd, Zo, lam)
    assert (info["objective"] - fo) / fo <= 1e-6
