"""nncp_sweep's MU/HALS path, which normalises the factors once at the end
of the call instead of after every mode update (MU and HALS commute with
column scalings of the other factors, so the iterates are those of the
normalised iteration of Algorithm 4 up to rounding): the cases where the
two could part.  Oracle: Algorithm 1 with the per-mode normalisation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import nncp_inputs as gen  # noqa: E402
import oracle  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1909_01149_amd as nn
    nn.lib()
    return nn


def banner(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


@pytest.mark.parametrize("algo", ["mu", "hals"])
def test_zero_column_matches_oracle(nn, algo):
    """A zero column in one start factor.  MU: the oracle's lambda_r is 0
    from the first normalisation on and every factor's column r ends zero;
    the deferred path must end in the same state.  HALS: the column comes
    back (S(r, r) = 0 skips it in the first update only), and both paths
    follow the same trajectory."""
    banner("zero column", algo)
    dims, R = [12, 10, 14], 4
    X64, H64 = gen.small_lowrank(dims, R, R, 31, noise=0.03)
    H64[1][:, 2] = 0.0
    X = torch.from_numpy(X64).cuda()
    H = [torch.from_numpy(h.copy()).cuda() for h in H64]
    ctx = nn.Context(X, H)
    a, oa = (nn.NNCP_MU, oracle.MU) if algo == "mu" else (nn.NNCP_HALS, oracle.HALS)
    rel = ctx.sweep(a, 3).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(X64, H64, np.ones(R), oa, 3)
    np.testing.assert_allclose(rel, rel_o, rtol=1e-10, atol=1e-13)
    if algo == "mu":
        assert ctx.lam[2].item() == 0.0 and lam[2] == 0.0
        for x in ctx.factors:
            assert np.all(x[:, 2].cpu().numpy() == 0.0)
    for x, y in zip(ctx.factors, Hr):
        assert relerr(x.cpu().numpy(), y) <= 1e-10
    assert relerr(ctx.lam.cpu().numpy(), lam) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("algo", ["mu", "hals"])
def test_one_sweep_per_call_equals_one_call(nn, algo):
    """Three calls of one sweep (each folds the lambda the previous call
    left) against one call of three sweeps and against the oracle."""
    banner("split calls", algo)
    dims, R = [9, 11, 8, 7], 5
    X64, H64 = gen.small_lowrank(dims, R, R, 12, noise=0.05)
    X = torch.from_numpy(X64).cuda()
    a, oa = (nn.NNCP_MU, oracle.MU) if algo == "mu" else (nn.NNCP_HALS, oracle.HALS)
    c1 = nn.Context(X, [torch.from_numpy(h.copy()).cuda() for h in H64])
    rel1 = [c1.sweep(a, 1).cpu().numpy()[0] for _ in range(3)]
    c3 = nn.Context(X, [torch.from_numpy(h.copy()).cuda() for h in H64])
    rel3 = c3.sweep(a, 3).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(X64, H64, np.ones(R), oa, 3)
    np.testing.assert_allclose(rel1, rel3, rtol=1e-12, atol=0)
    np.testing.assert_allclose(rel3, rel_o, rtol=1e-10, atol=0)
    for x, y, z in zip(c1.factors, c3.factors, Hr):
        assert relerr(x.cpu().numpy(), y.cpu().numpy()) <= 1e-12
        assert relerr(y.cpu().numpy(), z) <= 1e-10
    assert relerr(c1.lam.cpu().numpy(), lam) <= 1e-10
    # the context's Grams after the call are those of the stored factors
    for n in range(len(dims)):
        S = c3.hadamard(n).cpu().numpy()
        Go = [oracle.gram(f.cpu().numpy()) for f in c3.factors]
        np.testing.assert_allclose(S, oracle.hadamard_except(Go, n), rtol=1e-12, atol=1e-14)
    c1.close()
    c3.close()


def test_rank_above_64_keeps_normalised_path(nn):
    """R > 64 (rows of more than one wave): the per-mode normalised path."""
    banner("R 80 hals")
    dims, R = [40, 36, 30], 80
    X64, H64 = gen.small_lowrank(dims, 10, R, 44, noise=0.05)
    X = torch.from_numpy(X64).cuda()
    ctx = nn.Context(X, [torch.from_numpy(h.copy()).cuda() for h in H64])
    rel = ctx.sweep(nn.NNCP_HALS, 2).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(X64, H64, np.ones(R), oracle.HALS, 2)
    np.testing.assert_allclose(rel, rel_o, rtol=1e-9, atol=1e-12)
    for x, y in zip(ctx.factors, Hr):
        assert relerr(x.cpu().numpy(), y) <= 1e-9
    ctx.close()
