"""The factor updates at the benchmark's real shape (512^3 BF16 tensor, R = 32,
the start factors of the benchmark): one update of mode 1 for each rule, with
the GPU's own M^(1) and S^(1) handed to both sides, against the oracle's
update of the whole factor (512 rows, cheap on the CPU).  Compared on
Hhat = H diag(lambda) and on lambda, normwise relative: 1e-6 (FP32 factor
storage; both sides compute in FP64)."""
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


@pytest.fixture(scope="module")
def w2():
    w = gen.workload2(keep_fp32=False)
    yield w
    del w
    torch.cuda.empty_cache()


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("algo", ["hals", "mu", "bpp", "admm", "nes"])
def test_update_at_512_cube(nn, w2, algo):
    print("[case] 512^3 bf16 update", algo, flush=True)
    H = [torch.from_numpy(h).float().cuda() for h in w2["H0"]]
    ctx = nn.Context(w2["Xbf16"], [h.clone() for h in H])
    n = 1
    M = ctx.mttkrp(n)
    S = ctx.hadamard(n)
    torch.cuda.synchronize()
    Mo = M.double().cpu().numpy()
    So = S.cpu().numpy()
    Hh = ctx.factors[n].double().cpu().numpy() * ctx.lam.cpu().numpy()[None, :]
    code = {"hals": nn.NNCP_HALS, "mu": nn.NNCP_MU, "bpp": nn.NNCP_BPP, "admm": nn.NNCP_ADMM,
            "nes": nn.NNCP_NES}[algo]
    ctx.update(code, n, M, S)
    torch.cuda.synchronize()
    if algo == "hals":
        want = oracle.update_hals(Hh, Mo, So)
    elif algo == "mu":
        want = oracle.update_mu(Hh, Mo, So, 1e-16)
    elif algo == "bpp":
        want, failed = oracle.update_bpp(Mo, So, Hh)
        assert failed == 0
    elif algo == "admm":
        want, _, passes = oracle.update_admm(Hh, np.zeros_like(Hh), Mo, So)
        assert passes >= 1
    else:
        want, ok = oracle.update_nes(Hh, Mo, So)
        assert ok
    got_lam = ctx.lam.cpu().numpy()
    got = ctx.factors[n].double().cpu().numpy() * got_lam[None, :]
    e = relerr(got, want)
    el = relerr(got_lam, np.linalg.norm(want, axis=0))
    print(f"{algo}: Hhat rel err {e:.3e}, lambda rel err {el:.3e}", flush=True)
    assert e <= 1e-6 and el <= 1e-6
    ctx.close()
