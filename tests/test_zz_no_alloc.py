"""nncp_mttkrp_noalloc (the MTTKRP entry point for callers that cannot
allocate) against nncp_mttkrp on a context of the same problem, both called
through the C ABI: the two run the same kernels in the same order, so every
output must agree bitwise.  Two calls in a row on the GPU's one scratch
array, the second on a smaller problem (its buffers sit at the same scratch
offsets and overlap what the first call left there)."""
import ctypes

import numpy as np
import pytest
import torch

import nncp_inputs as gen
import paper_1909_01149_amd as nn
from paper_1909_01149_amd import binding as B

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _problem(dims, R, seed, xdtype):
    X64, H64 = gen.small_lowrank(dims, R, R, seed, noise=0.03)
    hdt = torch.float64 if xdtype == torch.float64 else torch.float32
    X = torch.from_numpy(X64).to(DEV).to(hdt).to(xdtype).contiguous()
    H = [torch.from_numpy(h).to(DEV).to(hdt).contiguous() for h in H64]
    return X, H


def _noalloc_c(X, H, mode, M, split=0):
    """Raw C call (no Python-side checks beyond the ones below)."""
    dims = [int(h.shape[0]) for h in H]
    R = int(H[0].shape[1])
    assert X.numel() == int(np.prod(dims)) and M.shape == (dims[mode], R)
    o = B._opts(split=split)
    return nn.lib().nncp_mttkrp_noalloc(len(dims), B._dims(dims), R, B._DT[X.dtype], B._ptr(X),
                                        B._DT[H[0].dtype], B._ptr_array(H), int(mode), B._ptr(M),
                                        B._stream_handle(X.device), ctypes.byref(o))


def _with_context(X, H, mode, split=0):
    ctx = nn.Context(X, H, split=split)
    M = ctx.mttkrp(mode)
    torch.cuda.synchronize()
    ctx.close()
    return M


CASES = [
    # (dims, R, tensor dtype, forced split)
    ([512, 512, 512], 32, torch.bfloat16, 0),   # the benchmark shape
    ([40, 36, 28], 8, torch.float32, 0),        # smaller: overlaps the first call's scratch
    ([24, 20, 18, 16], 20, torch.float64, 1),   # 4-way, forced split, FP64
    ([64, 48, 32, 16], 40, torch.float16, 0),
]


@pytest.mark.parametrize("order", [(0, 1), (2, 3)])
def test_noalloc_matches_context_mttkrp(order):
    for ci in order:
        dims, R, xdt, split = CASES[ci]
        X, H = _problem(dims, R, 20260 + ci, xdt)
        for mode in range(len(dims)):
            ref = _with_context(X, H, mode, split)
            M = torch.full_like(ref, float("nan"))
            rc = _noalloc_c(X, H, mode, M, split)
            assert rc == 0, nn.lib().nncp_last_error().decode()
            torch.cuda.synchronize()
            assert torch.equal(M, ref), (dims, mode, float((M - ref).abs().max()))


def test_noalloc_two_calls_smaller_second():
    """The same entry point twice in a row without a synchronisation between
    the calls, the second problem smaller than the first."""
    X1, H1 = _problem([256, 192, 160], 32, 777, torch.bfloat16)
    X2, H2 = _problem([48, 40, 36], 16, 778, torch.float32)
    ref1 = _with_context(X1, H1, 1)
    ref2 = _with_context(X2, H2, 1)
    M1 = torch.empty_like(ref1)
    M2 = torch.empty_like(ref2)
    assert _noalloc_c(X1, H1, 1, M1) == 0
    assert _noalloc_c(X2, H2, 1, M2) == 0
    torch.cuda.synchronize()
    assert torch.equal(M1, ref1)
    assert torch.equal(M2, ref2)


def test_noalloc_binding_checks_and_oracle():
    """The Python wrapper checks shapes before the call; the result also
    agrees with the CPU oracle (FP64, exact definition)."""
    import oracle
    X, H = _problem([30, 22, 26], 6, 31337, torch.float64)
    M = torch.empty(22, 6, dtype=torch.float64, device=DEV)
    nn.nncp_mttkrp_noalloc(X, H, 1, M)
    torch.cuda.synchronize()
    Mo = oracle.mttkrp(X.cpu().numpy(), [h.cpu().numpy() for h in H], 1)
    np.testing.assert_allclose(M.cpu().numpy(), Mo, rtol=1e-12, atol=0)
    with pytest.raises(ValueError):
        nn.nncp_mttkrp_noalloc(X, H, 1, torch.empty(21, 6, dtype=torch.float64, device=DEV))
