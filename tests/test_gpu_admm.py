"""GPU parity of the ADMM update (Section 4.3.4, Eqs. eqn:admmnls and
eqn:admmupd: rho = trace(S)/R, at most 5 passes, the stopping test of the
cited method, the dual kept per mode) against the CPU oracle, through the C
ABI.  Tolerances (normwise relative): FP64 1e-10 (the GPU applies the
inverse of S + rho I formed by Gauss-Jordan elimination, the oracle solves
with its Cholesky factor; the condition number is at most R + 1); FP32
factors 1e-6."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import nncp_inputs as gen  # noqa: E402
import oracle  # noqa: E402

pytestmark = pytest.mark.gpu

TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


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
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


def prepare(X64, H64, xdt):
    hdt = torch.float64 if xdt == "f64" else torch.float32
    Xc = torch.from_numpy(np.ascontiguousarray(X64)).to(TDT[xdt])
    Hc = [torch.from_numpy(np.ascontiguousarray(h)).to(hdt) for h in H64]
    return Xc.cuda(), [h.cuda() for h in Hc], Xc.double().numpy(), [h.double().numpy() for h in Hc]


@pytest.mark.parametrize("xdt", ["f64", "f32"])
@pytest.mark.parametrize("R", [1, 6, 17, 32, 48, 64])
def test_admm_update_one_mode_twice(nn, xdt, R):
    """Two updates of the same mode in a row: the second starts from the
    first's factor and dual (the dual is kept between updates of a mode)."""
    banner("admm update", xdt, R)
    dims = [50, 20, 30]
    X64, _ = gen.small_lowrank(dims, 3, R, 11, noise=0.05)
    H64 = gen.uniform_factors(dims, R, 12)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    lam0 = np.linspace(0.5, 2.0, R)
    ctx = nn.Context(X, H, lam=torch.from_numpy(lam0))
    n = 1
    M = oracle.mttkrp(Xo, Ho, n)
    M = M - 0.6 * M.mean(axis=1, keepdims=True)
    S = oracle.hadamard_except([oracle.gram(h) for h in Ho], n)
    hdt = torch.float64 if xdt == "f64" else torch.float32
    Md = torch.from_numpy(M).to(hdt).cuda()
    Mo = Md.double().cpu().numpy()
    Sd = torch.from_numpy(S).cuda()
    tol = 1e-10 if xdt == "f64" else 1e-6
    Hh = Ho[n] * lam0[None, :]
    U = np.zeros_like(Hh)
    for rep in range(2):
        ctx.update(nn.NNCP_ADMM, n, Md, Sd)
        torch.cuda.synchronize()
        Hh, U, passes = oracle.update_admm(Hh, U, Mo, S)
        assert passes >= 1
        Hn, lam = oracle.normalize(Hh)
        Hg = ctx.factors[n].double().cpu().numpy()
        assert relerr(Hg, Hn) <= tol, (rep, relerr(Hg, Hn))
        assert relerr(ctx.lam.cpu().numpy(), lam) <= tol
        # the oracle continues from the factor as the GPU stored it
        Hh = Hg * ctx.lam.cpu().numpy()[None, :]
    ctx.close()


def test_admm_needs_r_at_most_64(nn):
    dims = [20, 10, 12]
    X64, H64 = gen.small_lowrank(dims, 3, 70, 5)
    X, H, _, _ = prepare(X64, H64, "f32")
    ctx = nn.Context(X, H)
    with pytest.raises(nn.NNCPError):
        ctx.sweep(nn.NNCP_ADMM, 1)
    ctx.close()


@pytest.mark.parametrize("dims,R,split", [([12, 10, 14], 4, 0), ([6, 5, 4, 7], 3, 1),
                                          ([4, 5, 3, 4, 5], 4, 0), ([40, 30, 20], 24, 0)])
def test_admm_sweep_fp64_trajectory(nn, dims, R, split):
    banner("admm sweep fp64", dims, R, split)
    X64, H64 = gen.small_lowrank(dims, R, R, 79, noise=0.03)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H, split=split)
    rel = ctx.sweep(nn.NNCP_ADMM, 6).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(R), oracle.ADMM, 6)
    np.testing.assert_allclose(rel, rel_o, rtol=1e-9, atol=1e-12)
    for x, y in zip(ctx.factors, Hr):
        assert relerr(x.cpu().numpy(), y) <= 1e-9
    assert relerr(ctx.lam.cpu().numpy(), lam) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("xdt", ["f32", "bf16"])
def test_admm_sweep_low_precision(nn, xdt):
    banner("admm sweep", xdt)
    dims = [64, 64, 64]
    X64, H64 = gen.small_lowrank(dims, 8, 8, 99, noise=0.02)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    ctx = nn.Context(X, H)
    rel = ctx.sweep(nn.NNCP_ADMM, 8).cpu().numpy()
    _, _, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(8), oracle.ADMM, 8, nthreads=4)
    print("gpu", rel, "oracle", rel_o, flush=True)
    assert np.max(np.abs(rel - rel_o)) <= (1e-5 if xdt == "f32" else 3e-5), (rel, rel_o)
    assert rel[-1] < rel[0]
    ctx.close()


def test_admm_graph_replay_matches_eager(nn):
    banner("admm graph")
    dims = [64, 48, 40]
    X64, H64 = gen.small_lowrank(dims, 6, 12, 23, noise=0.05)
    X, H, _, _ = prepare(X64, H64, "bf16")
    cg = nn.Context(X, [h.clone() for h in H], graphs=1)
    ce = nn.Context(X, [h.clone() for h in H], graphs=0)
    hg = torch.empty(2, dtype=torch.float64, device="cuda")
    he = torch.empty(2, dtype=torch.float64, device="cuda")
    for rep in range(3):
        cg.sweep(nn.NNCP_ADMM, 2, hg)
        ce.sweep(nn.NNCP_ADMM, 2, he)
        torch.cuda.synchronize()
        assert torch.equal(hg, he), (rep, hg, he)
        for a, b in zip(cg.factors, ce.factors):
            assert torch.equal(a, b), rep
    cg.close()
    ce.close()
