"""Host-only checks of the C ABI: the library loads, exports every function
declared in include/nncp.h, and rejects invalid arguments before launching
anything (these calls never reach the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nncp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nncp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def B():
    from paper_1909_01149_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1909_01149_amd import build
        build.build()
    return binding


def test_every_declared_symbol_is_exported(B):
    L = B.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(B.EXPORTS) == names


def test_binding_module_has_the_c_names(B):
    import paper_1909_01149_amd as pkg
    for n in _declared():
        if n == "nncp_last_error":
            continue
        assert callable(getattr(pkg, n)), n


def test_workspace_size_validation(B):
    L = B.lib()
    dims = (ctypes.c_int64 * 3)(8, 8, 8)
    ok = L.nncp_workspace_size(3, dims, 4, B.NNCP_F32, B.NNCP_F32, None)
    assert ok > 0
    assert L.nncp_workspace_size(1, dims, 4, B.NNCP_F32, B.NNCP_F32, None) == 0
    assert b"N = 1" in L.nncp_last_error()
    assert L.nncp_workspace_size(3, dims, 0, B.NNCP_F32, B.NNCP_F32, None) == 0
    assert L.nncp_workspace_size(3, dims, 4, B.NNCP_BF16, B.NNCP_BF16, None) == 0
    assert b"unsupported" in L.nncp_last_error()
    assert L.nncp_workspace_size(3, dims, 4, B.NNCP_F64, B.NNCP_F32, None) == 0
    assert L.nncp_workspace_size(3, dims, 300, B.NNCP_F32, B.NNCP_F32, None) == 0
    bad = (ctypes.c_int64 * 3)(8, 0, 8)
    assert L.nncp_workspace_size(3, bad, 4, B.NNCP_F32, B.NNCP_F32, None) == 0
    o = B.nncp_options(5, 1, 0, 1e-16, 1)   # split outside [1, N-1]
    assert L.nncp_workspace_size(3, dims, 4, B.NNCP_F32, B.NNCP_F32, ctypes.byref(o)) == 0


def test_init_rejects_before_launch(B):
    L = B.lib()
    dims = (ctypes.c_int64 * 3)(8, 8, 8)
    ctx = ctypes.c_void_p()
    H = (ctypes.c_void_p * 3)(16, 32, 48)
    # NULL X
    rc = L.nncp_init(ctypes.byref(ctx), 3, dims, 4, B.NNCP_F32, None, B.NNCP_F32, H,
                     ctypes.c_void_p(64), ctypes.c_void_p(256), 1 << 30, None, None)
    assert rc == B.NNCP_E_INVAL
    # bad dtype pair
    rc = L.nncp_init(ctypes.byref(ctx), 3, dims, 4, B.NNCP_F16, ctypes.c_void_p(256), B.NNCP_F64, H,
                     ctypes.c_void_p(64), ctypes.c_void_p(256), 1 << 30, None, None)
    assert rc == B.NNCP_E_DTYPE
    # misaligned X
    rc = L.nncp_init(ctypes.byref(ctx), 3, dims, 4, B.NNCP_F32, ctypes.c_void_p(258), B.NNCP_F32, H,
                     ctypes.c_void_p(64), ctypes.c_void_p(256), 1 << 30, None, None)
    assert rc == B.NNCP_E_INVAL and b"aligned" in L.nncp_last_error()
    # workspace too small
    rc = L.nncp_init(ctypes.byref(ctx), 3, dims, 4, B.NNCP_F32, ctypes.c_void_p(256), B.NNCP_F32, H,
                     ctypes.c_void_p(64), ctypes.c_void_p(256), 16, None, None)
    assert rc == B.NNCP_E_WORKSPACE
    assert not ctx.value


def test_calls_on_null_context_fail(B):
    L = B.lib()
    assert L.nncp_mttkrp(None, 0, ctypes.c_void_p(16)) == B.NNCP_E_STATE
    assert L.nncp_sweep(None, 0, 1, None) == B.NNCP_E_STATE
    assert L.nncp_destroy(None) == B.NNCP_E_STATE
    assert L.nncp_split(None) == B.NNCP_E_STATE


def test_update_entry_points_on_null_context_fail(B):
    L = B.lib()
    for name in ("nncp_update_hals", "nncp_update_bpp", "nncp_update_admm", "nncp_update_nes"):
        assert getattr(L, name)(None, 0, ctypes.c_void_p(16), ctypes.c_void_p(16)) == B.NNCP_E_STATE
    assert L.nncp_update_mu(None, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), 1e-16) == B.NNCP_E_STATE
    assert L.nncp_sweep(None, B.NNCP_NES_OUTER, 1, None) == B.NNCP_E_STATE


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_binding_checks_shapes_before_any_call(B):
    """The binding compares X, the factors and lambda on the host (the C ABI
    sees only pointers, so a mismatch would otherwise become an out-of-bounds
    access on the device)."""
    import torch
    dims, R = [4, 3, 5], 2
    X = torch.rand(5, 3, 4)
    H = [torch.rand(d, R) for d in dims]
    assert B.check_problem(X, H) == (dims, R)
    assert B.check_problem(X.reshape(-1), H, torch.ones(R)) == (dims, R)
    bad = [
        (X.reshape(4, 3, 5), H, None),                      # shape not (I_2, I_1, I_0)
        (X[:4], [torch.rand(d, R) for d in dims], None),    # too few entries
        (X.transpose(0, 2), H, None),                       # not contiguous
        (X.to(torch.int32), H, None),                       # unsupported dtype
        (X, [H[0], H[1], torch.rand(5, R + 1)], None),      # ranks differ
        (X, [H[0], H[1].double(), H[2]], None),             # factor dtype
        (X.double(), H, None),                              # FP64 tensor needs FP64 factors
        (X, [h.t().contiguous().t() for h in H], None),     # non-contiguous factors
        (X, H, torch.ones(R + 1)),                          # lambda length
        (X, H[:1], None),                                   # one factor
        (X, [h.reshape(-1) for h in H], None),              # not 2-D
    ]
    for Xb, Hb, lb in bad:
        with pytest.raises(ValueError):
            B.check_problem(Xb, Hb, lb)
    with pytest.raises(ValueError):
        B.Context(X, H)                                     # host tensor: not a GPU tensor


def test_mttkrp_noalloc_rejects_before_launch(B):
    """nncp_mttkrp_noalloc validates its arguments and the scratch it would
    need before touching the GPU (fake, aligned, never dereferenced
    pointers are enough to reach every rejection)."""
    L = B.lib()
    fake = ctypes.c_void_p(1 << 20)
    H = (ctypes.c_void_p * 3)(1 << 20, 1 << 20, 1 << 20)
    dims = (ctypes.c_int64 * 3)(8, 8, 8)
    f32 = B.NNCP_F32
    assert L.nncp_mttkrp_noalloc(3, dims, 4, f32, fake, f32, H, 3, fake, None, None) == B.NNCP_E_INVAL
    assert b"mode" in L.nncp_last_error()
    assert L.nncp_mttkrp_noalloc(3, dims, 4, f32, None, f32, H, 0, fake, None, None) == B.NNCP_E_INVAL
    assert L.nncp_mttkrp_noalloc(3, dims, 4, f32, fake, f32, H, 0, ctypes.c_void_p((1 << 20) + 4),
                                 None, None) == B.NNCP_E_INVAL
    assert L.nncp_mttkrp_noalloc(3, dims, 4, B.NNCP_BF16, fake, B.NNCP_BF16, H, 0, fake, None,
                                 None) == B.NNCP_E_DTYPE
    # 2048 x 2048 x 64 at R = 64: the left node alone is 1 GiB
    big = (ctypes.c_int64 * 3)(2048, 2048, 64)
    assert L.nncp_mttkrp_noalloc(3, big, 64, f32, fake, f32, H, 0, fake, None,
                                 None) == B.NNCP_E_WORKSPACE
    assert b"scratch" in L.nncp_last_error()
    assert B.NNCP_NOALLOC_SCRATCH_BYTES == 64 << 20
    src = open(HEADER).read()
    assert "#define NNCP_NOALLOC_SCRATCH_BYTES (64u << 20)" in src
