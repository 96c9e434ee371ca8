"""GPU interference audit of the soft-lock (Alg. 3, eq. soft_lock; Prop. A.2).

The round kernel logs every worker's published candidate of each round
(dcdl_csc_opts.audit).  Two updates of one round interfere exactly when each
lies in the other's V: the cross term of Prop. A.2 for the pair is
C[k, k', w - w'] dZ dZ', and DtD vanishes outside Phi = (-L, L) per axis.
With the soft-lock on, no two accepted candidates of a round may lie within
(L1, L2) of each other on a 2-D worker grid, so the interference term of every
round is exactly zero; with it off, such pairs occur.  The log is also checked
for consistency with the solve's counters."""
import numpy as np
import pytest

from paper_1901_09235_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1901_09235_amd as dl
    dl.load()
    return dl


def _decode(rec, W):
    has = (rec >> 63) & 1
    acc = (rec >> 62) & 1
    k = (rec >> 32) & 0xFFFF
    pos = rec & 0xFFFFFFFF
    return has.astype(bool), acc.astype(bool), k, pos // W, pos % W


def _interacting_pairs(acc, h, w, L1, L2):
    """Pairs of accepted candidates of one round within each other's V."""
    idx = np.flatnonzero(acc)
    if idx.size < 2:
        return 0
    dh = np.abs(h[idx, None] - h[None, idx])
    dw = np.abs(w[idx, None] - w[None, idx])
    close = (dh < L1) & (dw < L2)
    np.fill_diagonal(close, False)
    return int(close.sum() // 2)


def _run(dl, pb, grid, rounds, **kw):
    X = torch.from_numpy(pb.X).to("cuda", dtype=torch.float32).contiguous()
    D = torch.from_numpy(pb.D).to("cuda", dtype=torch.float32).contiguous()
    lam = 0.1 * dl.dicodile_lambda_max(X, D)
    nW = grid[0] * grid[1]
    audit = torch.full((rounds, nW), -1, dtype=torch.int64, device="cuda")
    try:
        _, info = dl.dicodile_csc(X, D, lam, 1e-5 * lam, grid=grid, audit=audit, max_polish=4, timeout_s=60,
                                  div_guard=1e3, **kw)
    except dl.DicodileError as e:  # the divergence guard stopped the solve; the log stands
        info = {"status": str(e)}
    torch.cuda.synchronize()
    return audit.cpu().numpy().astype(np.uint64), info


@pytest.mark.parametrize("atoms", ["gaussian", "smooth"])
def test_accepted_candidates_never_interact_with_soft_lock(dl, atoms):
    if atoms == "smooth":
        D = synth.smooth_dictionary(np.random.Generator(np.random.PCG64(960)), 4, 1, (10, 10))
        pb = synth.make_problem("audit_smooth", 961, P=1, T=(160, 160), K=4, L=(10, 10), rho=0.01,
                                amp="uniform", sigma=0.1, D=D)
    else:
        pb = synth.make_problem("audit_gauss", 962, P=1, T=(160, 160), K=6, L=(10, 10), rho=0.01,
                                amp="uniform", sigma=0.1)
    L1, L2 = pb.D.shape[2:]
    grid = (12, 12)
    log, info = _run(dl, pb, grid, rounds=400)
    assert info["status"] == "OK", info
    H, W = (t - l + 1 for t, l in zip(pb.X.shape[1:], (L1, L2)))
    rounds_seen = min(400, info["n_rounds"]) if info["n_passes"] == 1 else 400
    n_acc = n_rej = 0
    for r in range(rounds_seen):
        rec = log[r]
        if (rec == np.uint64(2 ** 64 - 1)).all():
            break  # the first launch ended before this round
        has, acc, k, h, w = _decode(rec, W)
        assert (k[has] < pb.D.shape[0]).all() and (h[has] < H).all()
        assert _interacting_pairs(acc, h, w, L1, L2) == 0, f"round {r}"
        n_acc += int(acc.sum())
        n_rej += int((has & ~acc).sum())
    assert n_acc > 0 and n_rej > 0  # the test sees real rounds and real soft-locks
    if info["n_passes"] == 1 and info["n_rounds"] <= 400:
        assert n_acc == info["n_updates"] and n_rej == info["n_softlocked"]


def test_interacting_pairs_appear_without_soft_lock(dl):
    D = synth.smooth_dictionary(np.random.Generator(np.random.PCG64(960)), 4, 1, (10, 10))
    pb = synth.make_problem("audit_smooth", 961, P=1, T=(160, 160), K=4, L=(10, 10), rho=0.01,
                            amp="uniform", sigma=0.1, D=D)
    L1, L2 = pb.D.shape[2:]
    H, W = (t - l + 1 for t, l in zip(pb.X.shape[1:], (L1, L2)))
    log, info = _run(dl, pb, (12, 12), rounds=200, no_soft_lock=True)
    pairs = 0
    for r in range(200):
        rec = log[r]
        if (rec == np.uint64(2 ** 64 - 1)).all():
            break
        has, acc, k, h, w = _decode(rec, W)
        assert not (has & ~acc).any()  # nothing is soft-locked
        pairs += _interacting_pairs(acc, h, w, L1, L2)
    assert pairs > 0
