"""The gradient's single pass over X (both root partial MTTKRPs in one
kernel) against the oracle's gradient (the MTTKRP of the explicit residual
tensor, an independent route) and against the two-pass path on the same
inputs.  fused_grad = 2 runs the fused kernel on these oracle-sized
problems, whose grids are smaller than the default path would fuse."""
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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [
    # dims, R: right subtree a single mode (M^(N-1) straight from the partials),
    # R < 16 (one 16-column tile), 5 modes with a two-mode right subtree and
    # a ragged last workgroup (m = 32000 columns, 31.25 workgroups), R < 32
    ([64, 48, 96], 24),
    ([128, 40, 64], 12),
    ([64, 20, 25, 32, 16], 28),
    # the walks' multi-TTVs are grouped into launches by their data
    # dependencies: a three-mode right subtree (its node shares a buffer with
    # the left subtree's), and a four-mode left subtree (node 2 overwrites the
    # left root that earlier jobs read)
    ([64, 6, 8, 8, 16, 12], 20),
    ([8, 8, 8, 8, 16, 16], 16),
    # both at once (four left and three right modes), R < 16
    ([64, 4, 4, 4, 8, 8, 8], 16),
]


@pytest.mark.parametrize("dims,R", CASES)
def test_fused_grad_matches_oracle_and_two_pass(nn, dims, R):
    banner("fused grad", dims, R)
    X64, H64 = gen.small_lowrank(dims, R, R, 77, noise=0.05)
    X = torch.from_numpy(X64).float().to(torch.bfloat16).cuda()
    H = [torch.from_numpy(h).float().cuda() for h in H64]
    Xo = X.double().cpu().numpy()
    Ho = [h.double().cpu().numpy() for h in H]
    cf = nn.Context(X, [h.clone() for h in H], fused_grad=2)
    c2 = nn.Context(X, [h.clone() for h in H], fused_grad=0)
    assert cf.uses_fused_grad() and not c2.uses_fused_grad()
    gf, lf = cf.grad()
    g2, l2 = c2.grad()
    torch.cuda.synchronize()
    L, go = oracle.grad(Xo, Ho, nthreads=16)
    for n, (a, b, ref) in enumerate(zip(gf, g2, go)):
        ea = relerr(a.double().cpu().numpy(), ref)
        eb = relerr(a.double().cpu().numpy(), b.double().cpu().numpy())
        print(f"mode {n}: fused vs oracle {ea:.3e}, fused vs two-pass {eb:.3e}", flush=True)
        # the BF16 gradient tolerance of the other gradient tests
        assert ea <= 1e-4 and eb <= 1e-4
    assert abs(lf.item() - L) <= 1e-3 * L and abs(lf.item() - l2.item()) <= 1e-4 * L
    # the fused path is deterministic
    gf2, _ = cf.grad()
    torch.cuda.synchronize()
    for a, b in zip(gf, gf2):
        assert torch.equal(a, b)
    cf.close()
    c2.close()


def test_fused_path_eligibility(nn):
    """Where the fused kernel runs by default (the 64^5 gradient shape, a
    grid of 256 workgroups) and where it does not (FP32 tensor, R > 32, too
    small a grid, a single left mode)."""
    banner("fused eligibility")

    def ctx_of(dims, R, dt, **kw):
        X = torch.zeros(int(np.prod(dims)), dtype=dt, device="cuda")
        H = [torch.zeros(d, R, dtype=torch.float32, device="cuda") for d in dims]
        return nn.Context(X, H, **kw)

    c = ctx_of([64] * 5, 32, torch.bfloat16)
    assert c.uses_fused_grad()
    c.close()
    for dims, R, dt, kw in (([64] * 5, 32, torch.float32, {}),
                            ([64] * 5, 48, torch.bfloat16, {}),
                            ([64, 48, 96], 24, torch.bfloat16, {}),
                            ([64] * 5, 32, torch.bfloat16, {"fused_grad": 0})):
        c = ctx_of(dims, R, dt, **kw)
        assert not c.uses_fused_grad(), (dims, R, dt, kw)
        c.close()


def test_cploss_uses_fused_pass(nn):
    """CPLoss through the fused pass: backward gives the oracle gradient."""
    banner("cploss fused")
    dims, R = [64, 20, 25, 32, 16], 28
    X64, H64 = gen.small_lowrank(dims, R, R, 5, noise=0.05)
    X = torch.from_numpy(X64).float().to(torch.bfloat16).cuda()
    H = [torch.from_numpy(h).float().cuda() for h in H64]
    ctx = nn.Context(X, [h.clone() for h in H], fused_grad=2)
    Hs = [h.clone().requires_grad_(True) for h in H]
    loss = nn.CPLoss.apply(ctx, *Hs)
    loss.backward()
    L, go = oracle.grad(X.double().cpu().numpy(), [h.double().cpu().numpy() for h in H], nthreads=16)
    assert abs(loss.item() - L) <= 1e-3 * L
    for h, ref in zip(Hs, go):
        assert relerr(h.grad.double().cpu().numpy(), ref) <= 1e-4
    ctx.close()


def test_grad_rejects_overlapping_buffers(nn):
    """The gradient buffers keep the MTTKRPs until the last launch, so a
    gradient buffer that is a factor (or another gradient buffer) is refused
    before anything runs."""
    banner("grad buffer overlap")
    dims, R = [16, 12, 20], 8
    X64, H64 = gen.small_lowrank(dims, R, R, 3, noise=0.05)
    X = torch.from_numpy(X64).float().cuda()
    ctx = nn.Context(X, [torch.from_numpy(h).float().cuda() for h in H64])
    g = [torch.empty_like(f) for f in ctx.factors]
    with pytest.raises(ValueError, match="overlap"):
        ctx.grad([ctx.factors[0]] + g[1:])
    big = torch.empty(40, R, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="overlap"):
        ctx.grad([big[0:16], g[1], big[10:30]])
    ctx.close()
