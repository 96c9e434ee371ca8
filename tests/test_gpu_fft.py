"""The FP64 contraction by FFT (``dcdl_fft.h``) against the FP64 oracle and
the FP64 matrix-core contraction.

FP64 transforms of N = N1 N2 points carry a relative error of order
log2(N) 2^-53 of the largest magnitudes involved, so G is compared with
|err| <= 1e-12 max|G| (the shapes here have N <= 2^21).  The shapes cover one
and two column passes (N1 <= 128 and 256 ... 8192 rows), ragged sizes padded to
the next power of two, atoms taller than one row block (the dense atom
spectra), several channels and K beyond one chunk of the epilogue (K = 40)."""
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
    # name: (P, (T1, T2), K, (L1, L2))
    "one_pass": (1, (70, 83), 5, (16, 16)),
    "two_pass_ragged": (3, (300, 130), 4, (32, 32)),
    "tall_atoms": (2, (200, 90), 3, (70, 5)),
    "wide_k40": (2, (129, 257), 40, (8, 12)),
    "p8": (8, (64, 64), 3, (3, 3)),
}


def _case(name, seed=11):
    P, T, K, L = CASES[name]
    rng = np.random.Generator(np.random.PCG64(seed))
    D = synth.gaussian_dictionary(rng, K, P, L)
    X = rng.standard_normal((P,) + T)
    return X, D


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", sorted(CASES))
def test_fft_corr_matches_oracle(lib, name, dtype):
    X, D = _case(name)
    if dtype == torch.float32:
        X, D = X.astype(np.float32).astype(np.float64), D.astype(np.float32).astype(np.float64)
    ref = oracle.corr(X, D)
    G = lib.dicodile_corr(dev(X, dtype), dev(D, dtype), prec="f64_fft").double().cpu().numpy()
    # FP32 data (compared with the oracle on the same rounded inputs): the
    # FP64 result is rounded once to FP32
    rtol = 0.0 if dtype == torch.float64 else 2.0 ** -24
    np.testing.assert_allclose(G, ref, rtol=rtol, atol=1e-12 * np.abs(ref).max())


def test_fft_corr_equals_matrix_cores_on_the_image_workload(lib):
    """1024 x 1024, 25 atoms of 16 x 16 (two column passes of 16 x 64): the
    FFT and the FP64 matrix-core contraction agree to FP64 rounding."""
    rng = np.random.Generator(np.random.PCG64(12))
    X = torch.from_numpy(rng.standard_normal((1, 1024, 1024))).cuda()
    D = torch.from_numpy(synth.gaussian_dictionary(rng, 25, 1, (16, 16))).cuda()
    Gf = lib.dicodile_corr(X, D, prec="f64_fft")
    Gm = lib.dicodile_corr(X, D, prec="f64")
    err = float((Gf - Gm).abs().max() / Gm.abs().max())
    assert err <= 1e-13, err


def test_lambda_max_and_objective_by_fft_match_oracle(lib):
    """On 3 x 200 x 200 with 32 x 32 atoms the estimate picks the FFT for
    lambda_max and the objective/KKT check (auto); both match the oracle."""
    rng = np.random.Generator(np.random.PCG64(13))
    D = synth.gaussian_dictionary(rng, 6, 3, (32, 32))
    X = rng.standard_normal((3, 200, 200))
    for positive in (False, True):
        lm = lib.dicodile_lambda_max(dev(X, torch.float64), dev(D, torch.float64), positive)
        assert lm == pytest.approx(oracle.lambda_max(X, D, positive), rel=1e-12)
    Z = (rng.random((6, 169, 169)) < 0.01) * rng.standard_normal((6, 169, 169))
    lam = 0.2 * oracle.lambda_max(X, D)
    obj, kkt = lib.dicodile_objective_kkt(dev(X, torch.float64), dev(D, torch.float64), dev(Z, torch.float64), lam)
    assert obj == pytest.approx(oracle.objective(X, D, Z, lam), rel=1e-12)
    assert kkt == pytest.approx(oracle.kkt(X, D, Z, lam), rel=1e-10)


@pytest.mark.parametrize("method", ["fft", "mfma"])
def test_solve_with_fp64_method_matches_oracle(lib, method):
    """A BF16-started solve whose FP64 drift correction and checks run by FFT
    (or on the matrix cores) meets the target against the oracle's optimum."""
    pb = synth.make_problem("t", 14, P=3, T=(150, 140), K=5, L=(12, 12), rho=0.01, amp="uniform", sigma=0.1)
    X32, D32 = pb.X.astype(np.float32), pb.D.astype(np.float32)
    X64, D64 = X32.astype(np.float64), D32.astype(np.float64)
    lam = 0.1 * oracle.lambda_max(X64, D64)
    z, info = lib.dicodile_csc(dev(X32, torch.float32), dev(D32, torch.float32), lam, 1e-5 * lam,
                               beta_prec="bf16", refresh_every=2, refresh_limit=1, fp64_method=method)
    assert info["converged"] == 1
    assert (info["n_fft64"] > 0) == (method == "fft")
    # the incremental check follows the matrix-core contraction only
    assert info["n_check_inc"] == 0 or method == "mfma"
    zo, _ = oracle.lgcd(X64, D64, lam, 1e-9 * lam)
    f_opt = oracle.objective(X64, D64, zo, lam)
    f = oracle.objective(X64, D64, z.double().cpu().numpy(), lam)
    assert (f - f_opt) / f_opt <= 1e-6
    assert oracle.kkt(X64, D64, z.double().cpu().numpy(), lam) <= 1e-4
    assert info["kkt"] == pytest.approx(oracle.kkt(X64, D64, z.double().cpu().numpy(), lam), rel=1e-6, abs=1e-9)


def test_solve_initialised_by_fft(lib):
    """beta_prec = f64_fft initialises beta in FP64 by FFT: no drift at the
    first check beyond the rounds' own FP32 rounding, and the same optimum."""
    pb = synth.make_problem("t", 15, P=1, T=(256, 200), K=4, L=(8, 8), rho=0.01, amp="uniform", sigma=0.1)
    X, D = pb.X, pb.D
    lam = 0.1 * oracle.lambda_max(X, D)
    z, info = lib.dicodile_csc(dev(X, torch.float64), dev(D, torch.float64), lam, 1e-6 * lam, beta_prec="f64_fft")
    assert info["converged"] == 1 and info["init_prec"] == 5 and info["n_fft64"] >= 1
    zo, _ = oracle.lgcd(X, D, lam, 1e-10 * lam)
    f_opt = oracle.objective(X, D, zo, lam)
    assert (oracle.objective(X, D, z.cpu().numpy(), lam) - f_opt) / f_opt <= 1e-6
    assert info["beta_drift"] <= 1e-9
