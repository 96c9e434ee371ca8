"""Edge cases of the solve on the GPU against the oracle: the largest atom
count the library takes, 1x1 atoms (a diagonal problem with a closed form), a
domain one position wide, atoms longer than the patch size the union pass
takes, many channels, and a warm start from a perturbed iterate."""
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


def _compare(lib, pb, dtype, lam_frac=0.1, obj_tol=1e-6, **opts):
    X, D = pb.X, pb.D
    if dtype == torch.float32:
        X, D = X.astype(np.float32).astype(np.float64), D.astype(np.float32).astype(np.float64)
    lam = lam_frac * oracle.lambda_max(X, D)
    rel = 1e-10 if dtype == torch.float64 else 1e-5
    z, info = lib.dicodile_csc(dev(X, dtype), dev(D, dtype), lam, rel * lam, max_rounds=20_000_000,
                               timeout_s=60, **opts)
    assert info["status"] == "OK", info
    Zo, _ = oracle.lgcd(X, D, lam, 1e-11 * lam)
    fo = oracle.objective(X, D, Zo, lam)
    Zg = z.double().cpu().numpy()
    assert (oracle.objective(X, D, Zg, lam) - fo) / abs(fo) <= obj_tol
    assert oracle.kkt(X, D, Zg, lam) <= 1e-4
    return Zg, info


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_largest_atom_count(lib, dtype):
    """K = 1024, the most the library takes (one 16-byte vector group per
    four or two atoms, 256 or 512 groups per position).  1024 atoms of four
    samples are highly coherent; at lambda = 0.3 lambda_max the problem stays
    well enough conditioned for FP32 (at 0.1 lambda_max the FP32 solve needs
    over a million updates and its incremental beta drifts past the KKT
    target)."""
    D = synth.gaussian_dictionary(np.random.Generator(np.random.PCG64(201)), 1024, 1, 4)
    pb = synth.make_problem("k1024", 202, P=1, T=60, K=1024, L=4, rho=0.002, amp="uniform", sigma=0.1, D=D)
    _compare(lib, pb, dtype, lam_frac=0.3, grid=2)


def test_atom_count_above_the_limit_is_rejected(lib):
    X = torch.zeros((1, 40), dtype=torch.float32, device="cuda")
    D = torch.zeros((1025, 1, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.DicodileError):
        lib.dicodile_csc(X, D, 1.0, 1e-5)


def test_one_by_one_atoms_closed_form(lib):
    """K = P = 1 and a 1x1 atom: the design is diagonal, so the minimiser is
    Z = ST(d X, lambda) / d^2 elementwise, on any worker grid."""
    rng = np.random.Generator(np.random.PCG64(203))
    d = 0.7
    X = rng.standard_normal((1, 45, 38))
    D = np.full((1, 1, 1, 1), d)
    lam = 0.4
    for grid in ((1, 1), (5, 3)):
        z, info = lib.dicodile_csc(dev(X, torch.float64), dev(D, torch.float64), lam, 0.0, grid=grid,
                                   max_rounds=20_000_000, timeout_s=60)
        assert info["status"] == "OK" and info["grid"] == grid
        u = d * X[0]
        ref = np.sign(u) * np.maximum(np.abs(u) - lam, 0) / d ** 2
        np.testing.assert_allclose(z.cpu().numpy()[0], ref, rtol=0, atol=1e-14)


def test_domain_one_position_wide(lib):
    """2-D atoms as wide as the image: the valid domain is a single column."""
    pb = synth.make_problem("col", 204, P=2, T=(300, 9), K=3, L=(5, 9), rho=0.02, amp="uniform", sigma=0.1)
    _, info = _compare(lib, pb, torch.float64, grid=(4, 1))
    assert info["grid"] == (4, 1)


def test_long_atoms_take_the_update_by_update_path(lib):
    """1-D atoms of 600 samples patch 1199 positions, beyond what the union
    pass takes: neighbouring workers' updates are applied one by one."""
    pb = synth.make_problem("long", 205, P=2, T=2400, K=2, L=600, rho=0.002, amp="uniform", sigma=0.1)
    _compare(lib, pb, torch.float64, grid=3)
    _compare(lib, pb, torch.float32, grid=3)


def test_many_channels(lib):
    pb = synth.make_problem("chan", 206, P=16, T=800, K=4, L=20, rho=0.005, amp="exp", sigma=0.1)
    _compare(lib, pb, torch.float32, grid=4)


def test_warm_start_from_a_perturbed_iterate(lib):
    """A warm start away from the solution (perturbed support and values)
    still reaches the oracle's minimiser."""
    pb = synth.make_problem("warm", 207, P=1, T=(48, 52), K=3, L=(6, 6), rho=0.01, amp="uniform", sigma=0.1)
    lam = 0.1 * oracle.lambda_max(pb.X, pb.D)
    Zo, _ = oracle.lgcd(pb.X, pb.D, lam, 1e-11 * lam)
    rng = np.random.Generator(np.random.PCG64(208))
    Z0 = Zo * (1 + 0.3 * rng.standard_normal(Zo.shape)) + 0.05 * (rng.random(Zo.shape) < 0.01)
    z = dev(Z0, torch.float64)
    z, info = lib.dicodile_csc(dev(pb.X, torch.float64), dev(pb.D, torch.float64), lam, 1e-10 * lam, z_out=z,
                               warm_start=True, grid=(2, 2), max_rounds=20_000_000, timeout_s=60)
    assert info["status"] == "OK" and info["n_updates"] > 0
    fo = oracle.objective(pb.X, pb.D, Zo, lam)
    assert (oracle.objective(pb.X, pb.D, z.cpu().numpy(), lam) - fo) / fo <= 1e-9
