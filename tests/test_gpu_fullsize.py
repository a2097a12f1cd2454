"""Full-size workloads (the 4-way 256^4, imaging-shaped 1024x1024x2048 and
5-way 64^5 problems): sampled rows of MTTKRP and of the gradient against the
oracle.  A sampled row i of mode n is computed by the oracle from the tensor
slice with i_n = i (its definition restricted to that slice), so the oracle
never needs the whole tensor in FP64.
Tolerances as in test_gpu_parity.py (normwise over the sampled rows)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import mttkrp_bounds as mb  # noqa: E402
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
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def slice_of(X, dims, n, i):
    """Host FP64 copy of the slice i_n = i (memory order of the other modes)."""
    N = len(dims)
    T = X.view(*dims[::-1])
    return T.select(N - 1 - n, int(i)).contiguous().double().cpu().numpy().reshape(-1)


def oracle_row(X, dims, Hh, n, i, nthreads=16, want_sum=False):
    xs = slice_of(X, dims, n, i)
    Hs = list(Hh)
    Hs[n] = Hh[n][i:i + 1]
    row = oracle.mttkrp_rows(xs, Hs, n, [0], nthreads=nthreads)[0]
    return (row, float(xs.sum())) if want_sum else row


def oracle_grad_row(X, dims, Hh, n, i, nthreads=16):
    xs = slice_of(X, dims, n, i)
    Hs = list(Hh)
    Hs[n] = Hh[n][i:i + 1]
    _, E = oracle.residual(xs, Hs, want_tensor=True)
    return oracle.mttkrp_rows(E, Hs, n, [0], nthreads=nthreads)[0]


def test_256_4way_bf16_sampled_rows(nn):
    banner("256^4 bf16 R=64")
    w = gen.workload3()
    X, dims, R = w["X"], w["dims"], w["R"]
    H = [torch.from_numpy(h).float().cuda() for h in w["H0"]]
    Hh = [h.double().cpu().numpy() for h in H]
    ctx = nn.Context(X, H)
    assert ctx.split() == 2 and ctx.gemm_path(0) == 1 and ctx.gemm_path(1) == 1
    rng = np.random.default_rng(3)
    plans = [ctx.gemm_plan(0), ctx.gemm_plan(1)]
    for n in range(4):
        M = ctx.mttkrp(n).double().cpu().numpy()
        rows = rng.choice(dims[n], 2, replace=False)
        ref = np.stack([oracle_row(X, dims, Hh, n, i) for i in rows])
        e = relerr(M[rows], ref)
        worst, c = mb.check(M[rows], ref, "bf16", dims, 2, n, plans)
        print(f"mode {n}: sampled-row rel err {e:.3e}, max entrywise {worst:.3e} "
              f"(bound {c:.3e})", flush=True)
        assert e <= 3e-5
    rel = ctx.sweep(nn.NNCP_HALS, 2).cpu().numpy()
    assert np.all(np.isfinite(rel)) and rel[1] < rel[0]
    ctx.close()


def test_imaging_fp16_sampled_rows_and_mu_hals(nn):
    banner("imaging fp16 R=16")
    w = gen.workload4()
    X, dims, R = w["X"], w["dims"], w["R"]
    H = [torch.from_numpy(h).float().cuda() for h in w["H0"]]
    Hh = [h.double().cpu().numpy() for h in H]
    ctx = nn.Context(X, H)
    assert ctx.gemm_path(0) == 1 and ctx.gemm_path(1) == 1
    rng = np.random.default_rng(4)
    plans = [ctx.gemm_plan(0), ctx.gemm_plan(1)]
    S = ctx.split()
    for n in range(3):
        M = ctx.mttkrp(n).double().cpu().numpy()
        rows = rng.choice(dims[n], 3, replace=False)
        got = [oracle_row(X, dims, Hh, n, i, want_sum=True) for i in rows]
        ref = np.stack([g[0] for g in got])
        e = relerr(M[rows], ref)
        worst, c = mb.check(M[rows], ref, "f16", dims, S, n, plans, Hh, [g[1] for g in got])
        print(f"mode {n}: sampled-row rel err {e:.3e}, max entrywise {worst:.3e} "
              f"(bound {c:.3e} + the FP16 range term)", flush=True)
        assert e <= 1e-5
    ctx.close()
    for algo in (nn.NNCP_MU, nn.NNCP_HALS):
        c = nn.Context(X, [h.clone() for h in H])
        rel = c.sweep(algo, 4).cpu().numpy()
        print("algo", algo, "relerr", rel, flush=True)
        assert np.all(np.isfinite(rel)) and np.all(np.diff(rel) <= 1e-6)
        c.close()


@pytest.mark.parametrize("xdt", ["f32", "bf16"])
def test_64_5way_gradient_rows(nn, xdt):
    banner("64^5 gradient", xdt)
    w = gen.workload5(keep_bf16=(xdt == "bf16"))
    X = w["X32"] if xdt == "f32" else w["Xbf16"]
    dims = w["dims"]
    H = [torch.from_numpy(h).float().cuda() for h in w["H0"]]
    Hh = [h.double().cpu().numpy() for h in H]
    ctx = nn.Context(X, H)
    assert ctx.split() == 3
    grads, loss = ctx.grad()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for n in range(5):
        i = int(rng.integers(dims[n]))
        ref = oracle_grad_row(X, dims, Hh, n, i)
        g = grads[n][i].double().cpu().numpy()
        e = relerr(g, ref)
        print(f"mode {n} row {i}: gradient rel err {e:.3e}", flush=True)
        assert e <= (2e-5 if xdt == "f32" else 1e-4)
    # 100 projected-gradient steps: the loss never increases
    L0 = loss.item()
    lh, eh = ctx.pgd(100)
    print("pgd loss", L0, lh[0], lh[-1], "accepted", sum(1 for e in eh if e > 0), flush=True)
    assert lh[0] <= L0 and np.all(np.diff(lh) <= 1e-9 * L0) and lh[-1] < 0.5 * L0
    ctx.close()


def test_64_5way_fp64_finite_differences(nn):
    """Central differences (h = 1e-3) of the FP64 loss on the full 64^5
    tensor against the adjoint, on sampled entries of every factor."""
    banner("64^5 fp64 fd")
    w = gen.workload5(keep_bf16=False)
    X = w["X32"].double()
    del w["X32"]
    H = [torch.from_numpy(h).double().cuda() for h in w["H0"]]
    ctx = nn.Context(X, H)
    grads, loss = ctx.grad()
    # the loss comes from the FP64 identity 0.5 (alpha - 2 beta + gamma): its
    # rounding (a few ulps of alpha) divided by 2h bounds the FD error
    alpha = float(torch.sum(X * X))
    rng = np.random.default_rng(6)
    h = 1e-3
    fd_tol = 64 * 2.0 ** -52 * alpha / (2 * h)
    for n in range(5):
        for _ in range(6):
            i, r = int(rng.integers(64)), int(rng.integers(32))
            orig = H[n][i, r].item()
            vals = []
            for s in (+1, -1):
                H[n][i, r] = orig + s * h
                ctx.set_factors(H)
                vals.append(ctx.cp_loss()[0].item())
            H[n][i, r] = orig
            fd = (vals[0] - vals[1]) / (2 * h)
            ctx.set_factors(H)
            g = grads[n][i, r].item()
            assert abs(g - fd) <= fd_tol + 1e-8 * abs(fd), (n, i, r, g, fd, fd_tol)
    ctx.close()
