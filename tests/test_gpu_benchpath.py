"""The benchmark's own path against the oracle.

* The 512^3 R = 32 HALS sweep exactly as the benchmark runs it (warm-up
  sweeps, factors reset, the sweeps captured once and replayed as a HIP graph;
  carried Gram steps, split partials of the right product added inside the
  row update, eight-workgroup normalisation) against the oracle's sweeps
  (Algorithm 1, Algorithm 4) on the same stored tensor, for the FP32 tensor
  and its BF16 rounding.
* The entrywise error bound of the BF16/FP16 MTTKRP (tests/mttkrp_bounds.py)
  at 512^3, every mode, every entry.
* Error sequences of down-scaled versions of the 4-way and imaging workloads
  (same generators) against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import mttkrp_bounds as mb  # noqa: E402
import nncp_inputs as gen  # noqa: E402
import oracle  # noqa: E402

pytestmark = pytest.mark.gpu

NTHR = 16


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


def banner(*a):
    print("[case]", *a, flush=True)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# |delta eps| per sweep (eps is an absolute quantity ~0.1): the per-call
# MTTKRP tolerances (FP32 tensor 1e-5, BF16 tensor 3e-5 normwise)
EPS_TOL = {"f32": 1e-5, "bf16": 3e-5}


@pytest.mark.parametrize("xdt", ["f32", "bf16"])
def test_512cube_graph_sweeps_match_oracle(nn, w2, xdt):
    banner("512^3 graph-replayed HALS sweeps vs oracle", xdt)
    X = w2["X32"] if xdt == "f32" else w2["Xbf16"]
    H0 = [torch.from_numpy(h).float().cuda() for h in w2["H0"]]
    nsw = 3
    # the benchmark's sequence: context, warm-up sweeps, reset, capture, replay
    ctx = nn.Context(X, [h.clone() for h in H0])
    ctx.sweep(nn.NNCP_HALS, 2)
    torch.cuda.synchronize()
    for f, h0 in zip(ctx.factors, H0):
        f.copy_(h0)
    ctx.lam.fill_(1.0)
    ctx.refresh_grams()
    rel = torch.empty(nsw, dtype=torch.float64, device="cuda")
    ctx.capture(nn.NNCP_HALS, nsw, rel)
    ctx.sweep(nn.NNCP_HALS, nsw, rel)
    torch.cuda.synchronize()
    rel_g = rel.cpu().numpy()
    Hg = [f.double().cpu().numpy() for f in ctx.factors]
    lam_g = ctx.lam.cpu().numpy()
    ctx.close()
    Xo = X.double().cpu().numpy().reshape(-1)
    Ho = [h.double().cpu().numpy() for h in H0]
    Hr, lam_r, rel_r, _ = oracle.sweeps(Xo, Ho, np.ones(32), oracle.HALS, nsw, nthreads=NTHR)
    del Xo
    d_eps = np.abs(rel_g - rel_r)
    e_fac = [relerr(a, b) for a, b in zip(Hg, Hr)]
    e_lam = relerr(lam_g, lam_r)
    print(f"{xdt}: eps gpu {rel_g.tolist()} oracle {rel_r.tolist()} |d| {d_eps.max():.3e}; "
          f"factors {[f'{e:.2e}' for e in e_fac]} lambda {e_lam:.2e}", flush=True)
    assert d_eps.max() <= EPS_TOL[xdt]
    # factors and lambda after the sweeps, normwise, within the per-call
    # MTTKRP tolerance of the tensor's type: the HALS sweeps do not amplify
    # the MTTKRP's rounding over these 3 sweeps (measured: FP32 tensor
    # <= 2.7e-6, BF16 tensor <= 9.2e-6); a wrong column, row or mode order
    # gives errors of order one
    assert max(e_fac) <= EPS_TOL[xdt] and e_lam <= EPS_TOL[xdt]


@pytest.mark.parametrize("xdt", ["bf16", "f16"])
def test_512cube_entrywise_bound(nn, w2, xdt):
    banner("512^3 entrywise MTTKRP bound", xdt)
    dt = torch.bfloat16 if xdt == "bf16" else torch.float16
    X = w2["Xbf16"] if xdt == "bf16" else w2["X32"].to(dt)
    dims = w2["dims"]
    H = [torch.from_numpy(h).float().cuda() for h in w2["H0"]]
    Hh = [h.double().cpu().numpy() for h in H]
    ctx = nn.Context(X, H)
    S = ctx.split()
    plans = [ctx.gemm_plan(0), ctx.gemm_plan(1)]
    assert plans[0]["mfma"] and plans[1]["mfma"] and plans[0]["hl"] and plans[1]["hl"]
    Xo = X.double().cpu().numpy().reshape(-1)
    X32o = w2["X32"].double().cpu().numpy().reshape(-1)
    sums = [None] * 3
    if xdt == "f16":
        T = Xo.reshape(dims[::-1])
        sums = [T.sum(axis=(0, 1)), T.sum(axis=(0, 2)), T.sum(axis=(1, 2))]
    for n in range(3):
        M = ctx.mttkrp(n).double().cpu().numpy()
        Mref = oracle.mttkrp(Xo, Hh, n, nthreads=NTHR)
        worst, c = mb.check(M, Mref, xdt, dims, S, n, plans, Hh, sums[n])
        Mun = oracle.mttkrp(X32o, Hh, n, nthreads=NTHR)
        un = float(np.max(np.abs(M - Mun) / Mun))
        print(f"{xdt} mode {n}: max entrywise rel err {worst:.3e} (bound {c:.3e}, "
              f"normwise {relerr(M, Mref):.3e}); against the unrounded FP32 tensor {un:.3e}",
              flush=True)
    ctx.close()


def _eps_sequences(nn, X, H0, algo, oalgo, nsw, R):
    ctx = nn.Context(X, [h.clone() for h in H0])
    rel = ctx.sweep(algo, nsw).cpu().numpy()
    ctx.close()
    Xo = X.double().cpu().numpy().reshape(-1)
    Ho = [h.double().cpu().numpy() for h in H0]
    _, _, rel_r, _ = oracle.sweeps(Xo, Ho, np.ones(R), oalgo, nsw, nthreads=NTHR)
    return rel, rel_r


def test_4way_downscaled_bf16_eps(nn):
    """The 256^4 recipe at 32^4 (rank-64 exponential(1) factors, 2% |Gaussian|
    noise, BF16 storage, R = 64, HALS): error after each of 3 sweeps."""
    banner("32^4 bf16 R=64 HALS eps")
    dims, R = [32] * 4, 64
    seed = gen.SEED_BASE + 2
    X0 = gen.lowrank_tensor(gen.exponential_factors(dims, R, seed))
    Xh = gen.add_noise(X0, "abs_gaussian", 0.02, seed + 1)
    X = torch.from_numpy(Xh).float().to(torch.bfloat16).cuda()
    H0 = [torch.from_numpy(h).float().cuda() for h in gen.uniform_factors(dims, R, seed + 1000)]
    rel, rel_r = _eps_sequences(nn, X, H0, nn.NNCP_HALS, oracle.HALS, 3, R)
    print("gpu", rel.tolist(), "oracle", rel_r.tolist(), flush=True)
    assert np.max(np.abs(rel - rel_r)) <= 3e-5


@pytest.mark.parametrize("algo", ["mu", "hals"])
def test_imaging_downscaled_f16_eps(nn, algo):
    """The imaging recipe at 64 x 64 x 128 (FP16, R = 16): error after each of
    3 sweeps of MU and of HALS."""
    banner("imaging 64x64x128 f16 eps", algo)
    w = gen.workload4(dims=(64, 64, 128), R=16)
    H0 = [torch.from_numpy(h).float().cuda() for h in w["H0"]]
    a, oa = (nn.NNCP_MU, oracle.MU) if algo == "mu" else (nn.NNCP_HALS, oracle.HALS)
    rel, rel_r = _eps_sequences(nn, w["X"], H0, a, oa, 3, 16)
    print("gpu", rel.tolist(), "oracle", rel_r.tolist(), flush=True)
    assert np.max(np.abs(rel - rel_r)) <= 1e-5
