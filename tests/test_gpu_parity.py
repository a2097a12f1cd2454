"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
identical inputs.  Tolerances (normwise relative error ||A-B||_F/||B||_F
unless stated):
  FP64 mode                     1e-10
  FP32 tensor, FP32 factors     1e-5
  BF16 tensor, hi+lo KRP        3e-5   (operand ~2^-17, FP32 accumulation)
  FP16 tensor, hi+lo KRP        1e-5
  BF16 tensor, single KRP       4e-3   (operand rounding 2^-9)
  FP16 tensor, single KRP       1e-3   (2^-12)
The oracle always consumes the tensor values as stored (after rounding) and
the factor values as stored (FP32 -> FP64 exactly).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import nncp_inputs as gen  # noqa: E402
import oracle  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {("f64", 1): 1e-10, ("f64", 0): 1e-10, ("f32", 1): 1e-5, ("f32", 0): 1e-5,
       ("bf16", 1): 3e-5, ("f16", 1): 1e-5, ("bf16", 0): 4e-3, ("f16", 0): 1e-3}
TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


@pytest.fixture(scope="module")
def nn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1909_01149_amd as nn
    nn.lib()   # raises if libnncp.so is missing: no fallback
    return nn


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


def prepare(X64, H64, xdt):
    """Round on the host, return (device X, device factors, oracle X, oracle factors)."""
    hdt = torch.float64 if xdt == "f64" else torch.float32
    Xc = torch.from_numpy(np.ascontiguousarray(X64)).to(TDT[xdt])
    Hc = [torch.from_numpy(np.ascontiguousarray(h)).to(hdt) for h in H64]
    Xo = Xc.double().numpy()
    Ho = [h.double().numpy() for h in Hc]
    return Xc.cuda(), [h.cuda() for h in Hc], Xo, Ho


def banner(*a):
    print("[case]", *a, flush=True)


MTTKRP_CASES = [
    # dims, R, dtype, split, generic, krp_split
    ([64, 64, 64], 8, "f64", 0, 0, 1),
    ([64, 64, 64], 16, "f32", 0, 0, 1),
    ([64, 64, 64], 32, "bf16", 0, 0, 1),
    ([64, 64, 64], 32, "bf16", 0, 0, 0),
    ([64, 64, 64], 16, "f16", 0, 0, 1),
    ([64, 64, 64], 16, "f16", 0, 0, 0),
    ([32, 48, 64], 7, "bf16", 0, 0, 1),
    ([128, 64, 96], 64, "bf16", 0, 0, 1),
    ([128, 64, 96], 48, "f32", 0, 0, 1),
    ([64, 32, 128], 40, "f64", 0, 0, 1),
    ([16, 16, 8, 8], 32, "f32", 1, 0, 1),
    ([16, 16, 8, 8], 32, "bf16", 2, 0, 1),
    ([16, 16, 8, 8], 32, "f64", 3, 0, 1),
    ([8, 4, 8, 4, 8], 16, "bf16", 0, 0, 1),
    ([8, 4, 8, 4, 8], 16, "f32", 2, 0, 1),
    ([4, 8, 4, 8, 4, 2], 5, "f64", 0, 0, 1),
    ([64, 96], 20, "f32", 0, 0, 1),
    ([96, 64], 20, "bf16", 0, 0, 1),
    ([1, 64, 1, 32], 5, "f32", 0, 0, 1),
    ([37, 5, 11], 3, "f32", 0, 0, 1),     # odd shape: vector-ALU path
    ([37, 5, 11], 3, "bf16", 0, 0, 1),
    ([17, 63, 65], 1, "f64", 0, 0, 1),
    ([200, 3, 5], 1, "f16", 0, 0, 1),
    ([64, 64, 64], 16, "f32", 0, 1, 1),   # forced vector-ALU path
    ([64, 64, 64], 16, "bf16", 0, 1, 1),
    ([48, 40, 72], 72, "f32", 0, 0, 1),   # R > 64: vector-ALU path
]


@pytest.mark.parametrize("dims,R,xdt,split,generic,hl", MTTKRP_CASES)
def test_mttkrp_all_modes(nn, dims, R, xdt, split, generic, hl):
    banner("mttkrp", dims, R, xdt, split, generic, hl)
    seed = 1000 + sum(dims) + R
    X64, _ = gen.small_lowrank(dims, 3, R, seed, noise=0.1)
    H64 = gen.uniform_factors(dims, R, seed + 7)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    ctx = nn.Context(X, H, split=split, generic=generic, krp_split=hl)
    tol = TOL[(xdt, hl)]
    for n in range(len(dims)):
        M = ctx.mttkrp(n)
        torch.cuda.synchronize()
        ref = oracle.mttkrp(Xo, Ho, n, nthreads=4)
        e = relerr(M.double().cpu().numpy(), ref)
        assert e <= tol, (n, e, tol)
    ctx.close()


def test_paths_chosen(nn):
    """The matrix-core kernels serve the benchmark-shaped problems; odd
    shapes and R > 64 take the vector-ALU kernels."""
    X = torch.rand(64 ** 3, device="cuda").to(torch.bfloat16)
    H = [torch.rand(64, 32, device="cuda") for _ in range(3)]
    ctx = nn.Context(X, H)
    assert ctx.split() == 2 and ctx.gemm_path(0) == 1 and ctx.gemm_path(1) == 1
    ctx.close()
    X = torch.rand(37 * 5 * 11, device="cuda")
    H = [torch.rand(d, 3, device="cuda") for d in (37, 5, 11)]
    ctx = nn.Context(X, H)
    assert ctx.gemm_path(1) == 0
    ctx.close()


def test_split_rule(nn):
    for dims, S in [([64, 64, 64], 2), ([16, 16, 16, 16], 2), ([16] * 5, 3), ([2, 1000], 1),
                    ([1000, 2], 1), ([4, 4, 4, 64], 3)]:
        X = torch.zeros(int(np.prod(dims)), device="cuda")
        H = [torch.rand(d, 2, device="cuda") for d in dims]
        ctx = nn.Context(X, H)
        assert ctx.split() == S, (dims, ctx.split())
        ctx.close()


@pytest.mark.parametrize("xdt", ["f64", "f32"])
@pytest.mark.parametrize("R", [5, 32, 80])
def test_gram_hadamard(nn, xdt, R):
    banner("gram", xdt, R)
    dims = [40, 33, 50]
    X64, _ = gen.small_lowrank(dims, 2, R, 5)
    H64 = gen.uniform_factors(dims, R, 6)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    ctx = nn.Context(X, H)
    Gs = [ctx.gram(n).cpu().numpy() for n in range(3)]
    for n in range(3):
        np.testing.assert_allclose(Gs[n], oracle.gram(Ho[n]), rtol=1e-12)
        S = ctx.hadamard(n).cpu().numpy()
        np.testing.assert_allclose(S, oracle.hadamard_except([oracle.gram(h) for h in Ho], n), rtol=1e-12)
    ctx.close()


@pytest.mark.parametrize("xdt", ["f64", "f32"])
@pytest.mark.parametrize("algo", ["mu", "hals"])
@pytest.mark.parametrize("R", [1, 6, 32, 64, 100])
def test_update_one_mode(nn, xdt, algo, R):
    banner("update", xdt, algo, R)
    dims = [50, 20, 30]
    X64, _ = gen.small_lowrank(dims, 3, R, 11, noise=0.05)
    H64 = gen.uniform_factors(dims, R, 12)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    lam0 = np.linspace(0.5, 2.0, R)
    ctx = nn.Context(X, H, lam=torch.from_numpy(lam0))
    n = 1
    M = oracle.mttkrp(Xo, Ho, n)
    S = oracle.hadamard_except([oracle.gram(h) for h in Ho], n)
    hdt = torch.float64 if xdt == "f64" else torch.float32
    Md = torch.from_numpy(M).to(hdt).cuda()
    Mo = Md.double().cpu().numpy()
    Sd = torch.from_numpy(S).cuda()
    ctx.update(nn.NNCP_MU if algo == "mu" else nn.NNCP_HALS, n, Md, Sd)
    torch.cuda.synchronize()
    Hhat = Ho[n] * lam0[None, :]
    Hhat = oracle.update_mu(Hhat, Mo, S) if algo == "mu" else oracle.update_hals(Hhat, Mo, S)
    Hn, lam = oracle.normalize(Hhat)
    tol = 1e-11 if xdt == "f64" else 1e-6
    assert relerr(ctx.factors[n].double().cpu().numpy(), Hn) <= tol
    assert relerr(ctx.lam.cpu().numpy(), lam) <= 1e-11
    np.testing.assert_allclose(ctx.gram(n).cpu().numpy(), oracle.gram(ctx.factors[n].double().cpu().numpy()), rtol=1e-12)
    ctx.close()


def test_sweep_workload1_fp64_mu(nn):
    """64^3 FP64, rank 8, MU, 20 sweeps: full trajectory parity."""
    w = gen.workload1()
    banner("sweep workload1")
    X, H, Xo, Ho = prepare(w["X"], w["H0"], "f64")
    ctx = nn.Context(X, H)
    rel = ctx.sweep(nn.NNCP_MU, w["nsweeps"]).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(8), oracle.MU, w["nsweeps"], nthreads=4)
    np.testing.assert_allclose(rel, rel_o, rtol=1e-10, atol=0)
    for a, b in zip(ctx.factors, Hr):
        assert relerr(a.cpu().numpy(), b) <= 1e-10
    assert relerr(ctx.lam.cpu().numpy(), lam) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("dims,R,split", [([12, 10, 14], 4, 0), ([6, 5, 4, 7], 3, 1), ([6, 5, 4, 7], 3, 3),
                                          ([4, 5, 3, 4, 5], 4, 0), ([16, 32], 6, 0)])
@pytest.mark.parametrize("algo", ["mu", "hals"])
def test_sweep_fp64_trajectory(nn, dims, R, split, algo):
    banner("sweep fp64", dims, R, split, algo)
    X64, H64 = gen.small_lowrank(dims, R, R, 77, noise=0.03)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H, split=split)
    a = nn.NNCP_MU if algo == "mu" else nn.NNCP_HALS
    rel = ctx.sweep(a, 8).cpu().numpy()
    Hr, lam, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(R), a, 8)
    np.testing.assert_allclose(rel, rel_o, rtol=1e-9, atol=1e-12)
    for x, y in zip(ctx.factors, Hr):
        assert relerr(x.cpu().numpy(), y) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("xdt", ["f32", "bf16", "f16"])
def test_sweep_low_precision_relerr(nn, xdt):
    """Multi-sweep runs in FP32 factors: the relative-error sequences agree
    with the oracle run on the same stored tensor."""
    banner("sweep", xdt)
    dims = [64, 64, 64]
    X64, H64 = gen.small_lowrank(dims, 8, 8, 99, noise=0.02)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    ctx = nn.Context(X, H)
    rel = ctx.sweep(nn.NNCP_HALS, 10).cpu().numpy()
    _, _, rel_o, _ = oracle.sweeps(Xo, Ho, np.ones(8), oracle.HALS, 10, nthreads=4)
    assert np.max(np.abs(rel - rel_o)) <= (1e-5 if xdt != "bf16" else 3e-5), (rel, rel_o)
    ctx.close()


@pytest.mark.parametrize("xdt", ["f64", "f32", "bf16"])
def test_cp_loss(nn, xdt):
    banner("loss", xdt)
    dims = [24, 32, 40]
    X64, H64 = gen.small_lowrank(dims, 4, 4, 5, noise=0.1)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    lam0 = np.array([1.0, 2.0, 0.5, 1.5])
    ctx = nn.Context(X, H, lam=torch.from_numpy(lam0))
    out = ctx.cp_loss().cpu().numpy()
    L = oracle.residual(Xo, Ho, lam0)
    tol = 1e-10 if xdt == "f64" else 2e-4
    assert abs(out[0] - L) <= tol * L
    assert abs(out[1] - np.sqrt(2 * L / oracle.sumsq(Xo))) <= tol
    ctx.close()


@pytest.mark.parametrize("xdt,dims,R", [("f64", [6, 5, 4, 3, 2], 3), ("f64", [16, 16, 16], 8),
                                        ("f32", [16, 16, 16, 16, 16], 32), ("bf16", [16, 16, 16, 16, 16], 32)])
def test_grad_matches_oracle(nn, xdt, dims, R):
    banner("grad", xdt, dims, R)
    X64, H64 = gen.small_lowrank(dims, R, R, 3, noise=0.05)
    X, H, Xo, Ho = prepare(X64, H64, xdt)
    ctx = nn.Context(X, H)
    grads, loss = ctx.grad()
    torch.cuda.synchronize()
    L, go = oracle.grad(Xo, Ho, nthreads=4)
    tol = 1e-9 if xdt == "f64" else (2e-5 if xdt == "f32" else 1e-4)
    for a, b in zip(grads, go):
        assert relerr(a.double().cpu().numpy(), b) <= tol
    assert abs(loss.item() - L) <= (1e-9 if xdt == "f64" else 1e-3) * L
    ctx.close()


def test_autograd_finite_differences(nn):
    """CPLoss.backward against central differences (h = 1e-3, FP64 mode);
    the loss is quadratic in each entry, so the difference is exact up to
    rounding of the identity-based loss."""
    banner("autograd fd")
    dims = [5, 4, 6, 3, 4]
    X64, H64 = gen.small_lowrank(dims, 2, 2, 8, noise=0.1)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H)
    Hs = [h.clone().requires_grad_(True) for h in H]
    L = nn.CPLoss.apply(ctx, *Hs)
    L.backward()
    rng = np.random.default_rng(0)
    for n in range(len(dims)):
        for _ in range(4):
            i, r = rng.integers(dims[n]), rng.integers(2)
            P = [h.detach().clone() for h in H]
            Mn = [h.detach().clone() for h in H]
            P[n][i, r] += 1e-3
            Mn[n][i, r] -= 1e-3
            fd = (oracle.residual(Xo, [p.cpu().numpy() for p in P])
                  - oracle.residual(Xo, [p.cpu().numpy() for p in Mn])) / 2e-3
            g = Hs[n].grad[i, r].item()
            assert abs(g - fd) <= 1e-7 * max(1.0, abs(fd)), (n, i, r, g, fd)
    ctx.close()


def test_pgd_fp64_matches_oracle(nn):
    banner("pgd")
    dims = [8, 6, 7]
    X64, H64 = gen.small_lowrank(dims, 2, 2, 13, noise=0.05)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H)
    lh, eh = ctx.pgd(15)
    Hr, lho, eho = oracle.pgd(Xo, Ho, 15)
    np.testing.assert_allclose(lh, lho, rtol=1e-8)
    np.testing.assert_allclose(eh, eho, rtol=1e-10)
    for a, b in zip(ctx.factors, Hr):
        assert relerr(a.cpu().numpy(), b) <= 1e-8
    ctx.close()


def test_pgd_fp64_five_modes_rank40_matches_oracle(nn):
    """The step size's power iterations at R = 40 (the 64-row variant, lanes
    40..63 idle) over five modes (one wave each)."""
    banner("pgd 5 modes R 40")
    dims = [10, 9, 8, 7, 6]
    X64, H64 = gen.small_lowrank(dims, 6, 40, 21, noise=0.05)
    X, H, Xo, Ho = prepare(X64, H64, "f64")
    ctx = nn.Context(X, H)
    lh, eh = ctx.pgd(5)
    Hr, lho, eho = oracle.pgd(Xo, Ho, 5)
    np.testing.assert_allclose(eh, eho, rtol=1e-10)
    np.testing.assert_allclose(lh, lho, rtol=1e-8)
    for a, b in zip(ctx.factors, Hr):
        assert relerr(a.cpu().numpy(), b) <= 1e-8
    ctx.close()


def test_sweep_is_deterministic(nn):
    banner("determinism")
    dims = [64, 64, 64]
    X64, H64 = gen.small_lowrank(dims, 8, 16, 4, noise=0.05)
    outs = []
    for _ in range(2):
        X, H, _, _ = prepare(X64, H64, "bf16")
        ctx = nn.Context(X, H)
        rel = ctx.sweep(nn.NNCP_HALS, 3)
        torch.cuda.synchronize()
        outs.append(([f.cpu().clone() for f in ctx.factors], rel.cpu().clone()))
        ctx.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        assert torch.equal(a, b)
    assert torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("xdt", ["f32", "bf16"])
def test_fullsize_512cube_sampled_rows(nn, xdt):
    """512^3, R = 32 (the benchmark workload, same launch configuration):
    sampled rows of every mode's MTTKRP against the oracle row by row."""
    banner("512^3 sampled", xdt)
    w = gen.workload2(keep_fp32=False)
    X = w["X32"] if xdt == "f32" else w["Xbf16"]
    H = [torch.from_numpy(h).float().cuda() for h in w["H0"]]
    ctx = nn.Context(X, H)
    Xo = X.double().cpu().numpy().reshape(-1)
    Ho = [h.double().cpu().numpy() for h in H]
    rng = np.random.default_rng(1)
    for n in range(3):
        M = ctx.mttkrp(n).double().cpu().numpy()
        rows = np.sort(rng.choice(512, 6, replace=False))
        ref = oracle.mttkrp_rows(Xo, Ho, n, rows, nthreads=8)
        e = relerr(M[rows], ref)
        assert e <= TOL[(xdt, 1)], (n, e)
    ctx.close()
    del X, Xo


def test_graph_replays_match_eager(nn):
    """The sweep replayed as a HIP graph, several times with other GPU work and
    synchronisations in between, gives bitwise the same factors, lambda and
    relative errors as the same sweeps launched one kernel at a time."""
    banner("graph replays")
    dims = [64, 64, 64]
    X64, H64 = gen.small_lowrank(dims, 8, 16, 21, noise=0.05)
    X, H, _, _ = prepare(X64, H64, "bf16")
    cg = nn.Context(X, [h.clone() for h in H], graphs=1)
    ce = nn.Context(X, [h.clone() for h in H], graphs=0)
    hg = torch.empty(3, dtype=torch.float64, device="cuda")
    he = torch.empty(3, dtype=torch.float64, device="cuda")
    cg.capture(nn.NNCP_HALS, 3, hg)
    for rep in range(4):
        cg.sweep(nn.NNCP_HALS, 3, hg)
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        ce.sweep(nn.NNCP_HALS, 3, he)
        torch.cuda.synchronize()
        del junk
        assert torch.equal(hg, he), (rep, hg, he)
        assert torch.equal(cg.lam, ce.lam), rep
        for a, b in zip(cg.factors, ce.factors):
            assert torch.equal(a, b), rep
    cg.close()
    ce.close()
