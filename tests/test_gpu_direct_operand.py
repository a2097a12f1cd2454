"""The matrix-core products that form their Khatri-Rao operand from the
factors themselves (one fast mode, at most one slow mode) against the same
products fed by the operand kernel (options.krp_kernel = 1): the operand
takes the same roundings on both paths, so the results agree bit for bit,
and the Gram step carried by the product launch instead of the operand
launch leaves the sweep unchanged."""
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


XDT = {"bf16": torch.bfloat16, "f32": torch.float32, "f64": torch.float64, "f16": torch.float16}


def contexts(nn, dims, R, xdt, seed):
    X64, H64 = gen.small_lowrank(dims, R, R, seed, noise=0.05)
    hdt = torch.float64 if xdt == "f64" else torch.float32
    X = torch.from_numpy(X64).to(hdt).to(XDT[xdt]).cuda()
    H = [torch.from_numpy(h).to(hdt).cuda() for h in H64]
    a = nn.Context(X, [h.clone() for h in H])
    b = nn.Context(X, [h.clone() for h in H], krp_kernel=1)
    return a, b


@pytest.mark.parametrize("xdt", ["bf16", "f32", "f64"])
# both products direct; both direct with a slow mode on each side; the left
# product direct and the right one (two slow modes) through the operand kernel
@pytest.mark.parametrize("dims,R", [([64, 48, 96], 32), ([96, 40, 64, 32], 16),
                                    ([64, 12, 20, 64, 4], 16)])
def test_direct_operand_bitwise(nn, xdt, dims, R):
    banner("direct operand", xdt, dims, R)
    a, b = contexts(nn, dims, R, xdt, 3)
    # the direct path is taken on at least one side here, never with
    # krp_kernel = 1
    assert all(b.gemm_plan(s)["direct"] == 0 for s in (0, 1))
    assert any(a.gemm_plan(s)["direct"] for s in (0, 1)), "no product on the direct path"
    for n in range(len(dims)):
        assert torch.equal(a.mttkrp(n), b.mttkrp(n)), n
    ra = a.sweep(nn.NNCP_HALS, 2).cpu().numpy()
    rb = b.sweep(nn.NNCP_HALS, 2).cpu().numpy()
    assert np.array_equal(ra, rb)
    for x, y in zip(a.factors, b.factors):
        assert torch.equal(x, y)
    assert torch.equal(a.lam, b.lam)
    ra = a.sweep(nn.NNCP_MU, 1).cpu().numpy()
    rb = b.sweep(nn.NNCP_MU, 1).cpu().numpy()
    assert np.array_equal(ra, rb)
    a.close()
    b.close()


def test_direct_operand_applies_where_stated(nn):
    """R not a multiple of 16, an FP16 tensor: the operand kernel; the 512^3
    rank-32 shape: both products direct."""
    banner("direct operand eligibility")

    def plans(dims, R, dt):
        X = torch.zeros(int(np.prod(dims)), dtype=dt, device="cuda")
        hdt = torch.float64 if dt == torch.float64 else torch.float32
        H = [torch.zeros(d, R, dtype=hdt, device="cuda") for d in dims]
        c = nn.Context(X, H)
        p = [c.gemm_plan(0), c.gemm_plan(1)]
        c.close()
        return p

    p = plans([512, 512, 512], 32, torch.bfloat16)
    assert p[0]["direct"] == 1 and p[1]["direct"] == 1
    p = plans([256, 256, 256, 256], 64, torch.bfloat16)
    assert p[0]["direct"] == 1 and p[1]["direct"] == 1
    for dims, R, dt in (([64, 48, 96], 24, torch.bfloat16), ([64, 48, 96], 32, torch.float16)):
        p = plans(dims, R, dt)
        assert p[0]["direct"] == 0 and p[1]["direct"] == 0, (dims, R, dt)
