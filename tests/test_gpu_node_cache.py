"""nncp_mttkrp's node cache (the reuse of Algorithm 3 across separate calls):
a node is reused only while every factor it was contracted with is
unchanged, and the results equal a from-root computation on a fresh
context bit for bit (the same kernels on the same values).  The number of
partial-MTTKRP launches (timing categories 0 and 1) shows when X is read."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import nncp_inputs as gen  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1909_01149_amd as nn
    nn.lib()
    return nn


def banner(*a):
    print("[case]", *a, flush=True)


def fresh(nn, X, factors, mode):
    c = nn.Context(X, [f.clone() for f in factors])
    M = c.mttkrp(mode)
    torch.cuda.synchronize()
    c.close()
    return M


def root_launches(ctx):
    _, n = ctx.timers_read()
    return n[0] + n[1]


@pytest.mark.parametrize("xdt", [torch.bfloat16, torch.float64])
def test_node_reuse_and_invalidation(nn, xdt):
    banner("node cache", xdt)
    dims, R = [48, 40, 36, 44], 16
    X64, H64 = gen.small_lowrank(dims, R, R, 8, noise=0.05)
    hdt = torch.float64 if xdt == torch.float64 else torch.float32
    X = torch.from_numpy(X64).to(hdt).to(xdt).cuda()
    H = [torch.from_numpy(h).to(hdt).cuda() for h in H64]
    ctx = nn.Context(X, H)
    assert ctx.split() == 2
    ctx.timers_enable(True)
    # modes 0..3 in order: one root product per side
    Ms = [ctx.mttkrp(n) for n in range(4)]
    assert root_launches(ctx) == 2
    for n in range(4):
        assert torch.equal(Ms[n], fresh(nn, X, ctx.factors, n)), n
    # the right root node is the newest: mode 3 again reads nothing more
    ctx.timers_enable(True)
    M3 = ctx.mttkrp(3)
    assert root_launches(ctx) == 0 and torch.equal(M3, Ms[3])
    # mode 1 after mode 3: the left root was overwritten by the right one
    ctx.timers_enable(True)
    M1 = ctx.mttkrp(0)
    M1 = ctx.mttkrp(1)
    assert root_launches(ctx) == 1 and torch.equal(M1, Ms[1])
    # an update of mode 0 keeps the left root (contracted with modes 2, 3
    # only): mode 1 needs no pass over X, and sees the new factor
    S0 = ctx.hadamard(0)
    ctx.update(nn.NNCP_HALS, 0, ctx.mttkrp(0), S0)
    ctx.timers_enable(True)
    M1b = ctx.mttkrp(1)
    assert root_launches(ctx) == 0
    assert torch.equal(M1b, fresh(nn, X, ctx.factors, 1))
    # a caller's own write to factor 3, reported: the left root is stale
    with torch.no_grad():
        ctx.factors[3].mul_(0.5)
    ctx.refresh_grams(3)
    ctx.timers_enable(True)
    M1c = ctx.mttkrp(1)
    assert root_launches(ctx) == 1
    assert torch.equal(M1c, fresh(nn, X, ctx.factors, 1))
    # a sweep drops the cache
    ctx.timers_enable(False)
    ctx.sweep(nn.NNCP_HALS, 1)
    ctx.timers_enable(True)
    M1d = ctx.mttkrp(1)
    assert root_launches(ctx) == 1
    assert torch.equal(M1d, fresh(nn, X, ctx.factors, 1))
    ctx.close()
