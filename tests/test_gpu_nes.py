"""GPU parity of the Nesterov-type update (Section 4.3.5, Eqs. eqn:nesnls and
eqn:nesinnerupd: 20 accelerated projected-gradient steps on the proximal
subproblem, step parameters from power-step estimates of the extreme
eigenvalues of S) against the CPU oracle, through the C ABI.  Tolerances
(normwise relative): FP64 1e-10 (both sides take the same power steps; the
GPU adds each matrix-vector product in four partial sums and the norms by a
wave reduction, so the parameters differ by rounding); FP32 factors 1e-6."""
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
def test_nes_update_one_mode_twice(nn, xdt, R):
    """Two updates of the same mode in a row, each from the factor the
    previous one stored (the proximal centre is the start value)."""
    banner("nes update", xdt, R)
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
    _, _, plam, _, _, ok = oracle.nes_params(S)
    assert ok
    print("proximal weight", plam, flush=True)
    for rep in range(2):
        ctx.update(nn.NNCP_NES, n, Md, Sd)
        torch.cuda.synchronize()
        Hh, ok = oracle.update_nes(Hh, Mo, S)
        assert ok
        Hn, lam = oracle.normalize(Hh)
        Hg = ctx.factors[n].double().cpu().numpy()
        assert relerr(Hg, Hn) <= tol, (rep, relerr(Hg, Hn))
        assert relerr(ctx.lam.cpu().numpy(), lam) <= tol
        Hh = Hg * ctx.lam.cpu().numpy()[None, :]
    ctx.close()


def test_nes_proximal_case(nn):
    """A subproblem with an ill-conditioned S (nearly parallel columns), so
    the proximal weight is positive, in FP64."""
    banner("nes proximal")
    dims = [40, 30, 20]
    R = 8
    rng = np.random.default_rng(41)
    base = rng.random((max(dims), 1))
    H64 = [np.ascontiguousarray(base[:d] + 0.05 * rng.random((d, R))) for d in dims]
    X64, _ = gen.small_lowrank(dims, 3, R, 42, noise=0.05)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H)
    n = 2
    M = oracle.mttkrp(Xo, Ho, n)
    S = oracle.hadamard_except([oracle.gram(h) for h in Ho], n)
    _, _, plam, _, _, ok = oracle.nes_params(S)
    assert ok and plam > 0.0
    ctx.update(nn.NNCP_NES, n, torch.from_numpy(M).cuda(), torch.from_numpy(S).cuda())
    torch.cuda.synchronize()
    Hh, ok = oracle.update_nes(Ho[n].copy(), M, S)
    Hn, lam = oracle.normalize(Hh)
    assert relerr(ctx.factors[n].cpu().numpy(), Hn) <= 1e-10
    assert relerr(ctx.lam.cpu().numpy(), lam) <= 1e-10
    ctx.close()


def test_nes_needs_r_at_most_64(nn):
    dims = [20, 10, 12]
    X64, H64 = gen.small_lowrank(dims, 3, 70, 5)
    X, H, _, _ = prepare(X64, H64, "f32")
    ctx = nn.Context(X, H)
    with pytest.raises(nn.NNCPError):
        ctx.sweep(nn.NNCP_NES, 1)
    with pytest.raises(nn.NNCPError):
        ctx.sweep(nn.NNCP_NES_OUTER, 1)
    M = torch.zeros(20, 70, dtype=torch.float32, device="cuda")
    S = torch.eye(70, dtype=torch.float64, device="cuda")
    with pytest.raises(nn.NNCPError):
        ctx.update(nn.NNCP_NES, 0, M, S)
    ctx.close()


@pytest.mark.parametrize("dims,R,split", [([12, 10, 14], 4, 0), ([6, 5, 4, 7], 3, 1),
                                          ([4, 5, 3, 4, 5], 4, 0), ([40, 30, 20], 24, 0)])
def test_nes_sweep_fp64_trajectory(nn, dims, R, split):
    banner("nes sweep fp64", dims, R, split)
    X64, H64 = gen.small_lowrank(dims, R, R, 79, noise=0.03)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H, split=split)
    rel = ctx.sweep(nn.NNCP_NES, 6).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(R), oracle.NES, 6)
    np.testing.assert_allclose(rel, rel_o, rtol=1e-9, atol=1e-12)
    for x, y in zip(ctx.factors, Hr):
        assert relerr(x.cpu().numpy(), y) <= 1e-9
    assert relerr(ctx.lam.cpu().numpy(), lam) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("xdt", ["f32", "bf16"])
def test_nes_sweep_low_precision(nn, xdt):
    banner("nes sweep", xdt)
    dims = [64, 64, 64]
    X64, H64 = gen.small_lowrank(dims, 8, 8, 99, noise=0.02)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    ctx = nn.Context(X, H)
    rel = ctx.sweep(nn.NNCP_NES, 8).cpu().numpy()
    _, _, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(8), oracle.NES, 8, nthreads=4)
    print("gpu", rel, "oracle", rel_o, flush=True)
    assert np.max(np.abs(rel - rel_o)) <= (1e-5 if xdt == "f32" else 3e-5), (rel, rel_o)
    assert rel[-1] < rel[0]
    ctx.close()


def test_nes_graph_replay_matches_eager(nn):
    banner("nes graph")
    dims = [64, 48, 40]
    X64, H64 = gen.small_lowrank(dims, 6, 12, 23, noise=0.05)
    X, H, _, _ = prepare(X64, H64, "bf16")
    cg = nn.Context(X, [h.clone() for h in H], graphs=1)
    ce = nn.Context(X, [h.clone() for h in H], graphs=0)
    hg = torch.empty(2, dtype=torch.float64, device="cuda")
    he = torch.empty(2, dtype=torch.float64, device="cuda")
    for rep in range(3):
        cg.sweep(nn.NNCP_NES, 2, hg)
        ce.sweep(nn.NNCP_NES, 2, he)
        torch.cuda.synchronize()
        assert torch.equal(hg, he), (rep, hg, he)
        for a, b in zip(cg.factors, ce.factors):
            assert torch.equal(a, b), rep
    cg.close()
    ce.close()


# ---------------------------------------------------------------------------
# sweeps with the outer extrapolation (Eq. eqn:nesouterupd)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,R,split", [([12, 10, 14], 4, 0), ([6, 5, 4, 7], 3, 1),
                                          ([4, 5, 3, 4, 5], 4, 0), ([40, 30, 20], 24, 0)])
def test_nes_outer_sweep_fp64_trajectory(nn, dims, R, split):
    banner("nes outer sweep fp64", dims, R, split)
    X64, H64 = gen.small_lowrank(dims, R, R, 81, noise=0.03)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H, split=split)
    rel = ctx.sweep(nn.NNCP_NES_OUTER, 8).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(R), oracle.NES_OUTER, 8)
    _, _, rel_p, _ = oracle.sweeps(Xo, Ho, np.ones(R), oracle.NES, 8)
    print("gpu", rel, "oracle", rel_o, "plain", rel_p, flush=True)
    np.testing.assert_allclose(rel, rel_o, rtol=1e-9, atol=1e-12)
    for x, y in zip(ctx.factors, Hr):
        assert relerr(x.cpu().numpy(), y) <= 1e-9
    assert relerr(ctx.lam.cpu().numpy(), lam) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("xdt", ["f32", "bf16"])
def test_nes_outer_sweep_low_precision(nn, xdt):
    banner("nes outer sweep", xdt)
    dims = [64, 64, 64]
    X64, H64 = gen.small_lowrank(dims, 8, 8, 99, noise=0.02)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    ctx = nn.Context(X, H)
    rel = ctx.sweep(nn.NNCP_NES_OUTER, 8).cpu().numpy()
    _, _, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(8), oracle.NES_OUTER, 8, nthreads=4)
    print("gpu", rel, "oracle", rel_o, flush=True)
    assert np.max(np.abs(rel - rel_o)) <= (1e-5 if xdt == "f32" else 3e-5), (rel, rel_o)
    ctx.close()


def test_nes_outer_graph_replay_matches_eager(nn):
    banner("nes outer graph")
    dims = [64, 48, 40]
    X64, H64 = gen.small_lowrank(dims, 6, 12, 23, noise=0.05)
    X, H, _, _ = prepare(X64, H64, "bf16")
    cg = nn.Context(X, [h.clone() for h in H], graphs=1)
    ce = nn.Context(X, [h.clone() for h in H], graphs=0)
    hg = torch.empty(3, dtype=torch.float64, device="cuda")
    he = torch.empty(3, dtype=torch.float64, device="cuda")
    for rep in range(3):
        cg.sweep(nn.NNCP_NES_OUTER, 3, hg)
        ce.sweep(nn.NNCP_NES_OUTER, 3, he)
        torch.cuda.synchronize()
        assert torch.equal(hg, he), (rep, hg, he)
        for a, b in zip(cg.factors, ce.factors):
            assert torch.equal(a, b), rep
        assert torch.equal(cg.lam, ce.lam), rep
    cg.close()
    ce.close()


@pytest.mark.parametrize("graphs", [0, 1])
def test_nes_outer_iteration_count_continues_across_calls(nn, graphs):
    """The outer iteration i of s_i = i^(1/N) is counted on the device from
    nncp_init / nncp_set_factors, so two calls continue one run (the oracle
    is told the first iteration number of its second call)."""
    banner("nes outer count", graphs)
    dims, R = [12, 10, 14], 4
    X64, H64 = gen.small_lowrank(dims, R, R, 81, noise=0.03)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, [h.clone() for h in H], graphs=graphs)
    r1 = ctx.sweep(nn.NNCP_NES_OUTER, 3).cpu().numpy()
    r2 = ctx.sweep(nn.NNCP_NES_OUTER, 5).cpu().numpy()
    Ha, la, ra, _ = oracle.sweeps(Xo, Ho, np.ones(R), oracle.NES_OUTER, 3)
    Hb, lb, rb, _ = oracle.sweeps(Xo, Ha, la, oracle.NES_OUTER, 5, first_sweep=4)
    np.testing.assert_allclose(np.concatenate([r1, r2]), np.concatenate([ra, rb]), rtol=1e-9,
                               atol=1e-12)
    for x, y in zip(ctx.factors, Hb):
        assert relerr(x.cpu().numpy(), y) <= 1e-9
    # new factors: the count starts again from 1
    ctx.set_factors([h.clone() for h in H], torch.ones(R, dtype=torch.float64, device="cuda"))
    r3 = ctx.sweep(nn.NNCP_NES_OUTER, 3).cpu().numpy()
    np.testing.assert_allclose(r3, ra, rtol=1e-9, atol=1e-12)
    ctx.close()
