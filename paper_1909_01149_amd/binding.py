"""ctypes binding of libnncp.so: the C ABI of include/nncp.h under the same
names, taking torch tensors for device buffers.  Argument marshalling only:
every step of the computation runs in the library's HIP kernels.

Tensors: X is a contiguous tensor of shape (I_{N-1}, ..., I_0) (mode 0
fastest) or a flat contiguous tensor of prod(dims) entries; factors are
contiguous (I_n, R); lambda, Gram and loss buffers are float64.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnncp.so")

NNCP_OK = 0
NNCP_E_INVAL = -1
NNCP_E_DTYPE = -2
NNCP_E_WORKSPACE = -3
NNCP_E_HIP = -4
NNCP_E_STATE = -5
NNCP_E_UNSUPPORTED = -6

NNCP_F64, NNCP_F32, NNCP_BF16, NNCP_F16 = 0, 1, 2, 3
NNCP_MU, NNCP_HALS, NNCP_BPP, NNCP_ADMM, NNCP_NES, NNCP_NES_OUTER = 0, 1, 2, 3, 4, 5
NNCP_MAX_MODES = 16

EXPORTS = [
    "nncp_workspace_size", "nncp_init", "nncp_set_factors", "nncp_mttkrp", "nncp_gram",
    "nncp_hadamard", "nncp_update_mu", "nncp_update_hals", "nncp_cp_loss", "nncp_sweep",
    "nncp_grad", "nncp_pgd", "nncp_destroy", "nncp_last_error", "nncp_split",
    "nncp_gemm_path", "nncp_timers_enable", "nncp_timers_read", "nncp_sweep_capture",
    "nncp_update_bpp", "nncp_update_admm", "nncp_update_nes", "nncp_mttkrp_noalloc",
    "nncp_gemm_plan", "nncp_read_probe", "nncp_uses_fused_grad", "nncp_factors_changed",
]
NNCP_NOALLOC_SCRATCH_BYTES = 64 << 20
NNCP_TIMER_CATEGORIES = 5

_DT = {torch.float64: NNCP_F64, torch.float32: NNCP_F32, torch.bfloat16: NNCP_BF16,
       torch.float16: NNCP_F16}


class NNCPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nncp error {code}: {msg}")
        self.code = code


class nncp_options(ctypes.Structure):
    _fields_ = [("split", ctypes.c_int), ("krp_split", ctypes.c_int), ("generic", ctypes.c_int),
                ("eps_mu", ctypes.c_double), ("graphs", ctypes.c_int), ("fused_grad", ctypes.c_int),
                ("krp_kernel", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libnncp.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          f"`python -m paper_1909_01149_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    ci, cd, optp = ctypes.c_int, ctypes.c_double, ctypes.POINTER(nncp_options)
    dp = ctypes.c_void_p
    L.nncp_workspace_size.argtypes = [ci, i64p, ci, ci, ci, optp]
    L.nncp_workspace_size.restype = ctypes.c_size_t
    L.nncp_init.argtypes = [ctypes.POINTER(vp), ci, i64p, ci, ci, vp, ci, ctypes.POINTER(vp), dp, vp,
                            ctypes.c_size_t, vp, optp]
    L.nncp_set_factors.argtypes = [vp, ctypes.POINTER(vp), dp]
    L.nncp_mttkrp.argtypes = [vp, ci, vp]
    L.nncp_mttkrp_noalloc.argtypes = [ci, i64p, ci, ci, vp, ci, ctypes.POINTER(vp), ci, vp, vp,
                                      optp]
    L.nncp_gram.argtypes = [vp, ci, dp]
    L.nncp_hadamard.argtypes = [vp, ci, dp]
    L.nncp_update_mu.argtypes = [vp, ci, vp, dp, cd]
    L.nncp_update_hals.argtypes = [vp, ci, vp, dp]
    L.nncp_update_bpp.argtypes = [vp, ci, vp, dp]
    L.nncp_update_admm.argtypes = [vp, ci, vp, dp]
    L.nncp_update_nes.argtypes = [vp, ci, vp, dp]
    L.nncp_cp_loss.argtypes = [vp, dp, dp]
    L.nncp_sweep.argtypes = [vp, ci, ci, dp]
    L.nncp_sweep_capture.argtypes = [vp, ci, ci, dp]
    L.nncp_grad.argtypes = [vp, ctypes.POINTER(vp), dp]
    L.nncp_pgd.argtypes = [vp, ci, cd, ci, ci, ctypes.POINTER(cd), ctypes.POINTER(cd)]
    L.nncp_destroy.argtypes = [vp]
    L.nncp_last_error.restype = ctypes.c_char_p
    L.nncp_split.argtypes = [vp]
    L.nncp_gemm_path.argtypes = [vp, ci]
    L.nncp_gemm_plan.argtypes = [vp, ci, i64p]
    L.nncp_read_probe.argtypes = [vp, ctypes.c_size_t, ci, vp, vp]
    L.nncp_uses_fused_grad.argtypes = [vp]
    L.nncp_factors_changed.argtypes = [vp, ci]
    L.nncp_timers_enable.argtypes = [vp, ci]
    L.nncp_timers_read.argtypes = [vp, ctypes.POINTER(cd), ctypes.POINTER(ctypes.c_int64)]
    for name in ("nncp_timers_enable", "nncp_timers_read",
                 "nncp_init", "nncp_set_factors", "nncp_mttkrp", "nncp_gram", "nncp_hadamard",
                 "nncp_update_mu", "nncp_update_hals", "nncp_cp_loss", "nncp_sweep", "nncp_grad",
                 "nncp_pgd", "nncp_destroy", "nncp_split", "nncp_gemm_path",
                 "nncp_sweep_capture", "nncp_update_bpp", "nncp_update_admm",
                 "nncp_update_nes", "nncp_mttkrp_noalloc", "nncp_gemm_plan", "nncp_read_probe",
                 "nncp_uses_fused_grad", "nncp_factors_changed"):
        getattr(L, name).restype = ci
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc < 0:
        raise NNCPError(rc, lib().nncp_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dims(dims):
    arr = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
    return arr


def _opts(split=0, krp_split=1, generic=0, eps_mu=1e-16, graphs=1, fused_grad=1, krp_kernel=0):
    return nncp_options(int(split), int(krp_split), int(generic), float(eps_mu), int(graphs),
                        int(fused_grad), int(krp_kernel))


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# ---------------------------------------------------------------------------
# functions with the C names (thin wrappers)
# ---------------------------------------------------------------------------

def nncp_workspace_size(dims, R, x_dtype, h_dtype, **opts) -> int:
    o = _opts(**opts)
    n = lib().nncp_workspace_size(len(dims), _dims(dims), int(R), int(x_dtype), int(h_dtype),
                                  ctypes.byref(o))
    if n == 0:
        raise NNCPError(NNCP_E_INVAL, lib().nncp_last_error().decode())
    return int(n)


def nncp_init(dims, R, X, factors, lam, workspace, **opts) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    o = _opts(**opts)
    x_dt, h_dt = _DT[X.dtype], _DT[factors[0].dtype]
    _check(lib().nncp_init(ctypes.byref(ctx), len(dims), _dims(dims), int(R), x_dt, _ptr(X), h_dt,
                           _ptr_array(factors), _ptr(lam), _ptr(workspace),
                           workspace.numel() * workspace.element_size(),
                           _stream_handle(X.device), ctypes.byref(o)))
    return ctx


def nncp_set_factors(ctx, factors, lam=None):
    return _check(lib().nncp_set_factors(ctx, _ptr_array(factors), _ptr(lam)))


def nncp_mttkrp(ctx, mode, M):
    return _check(lib().nncp_mttkrp(ctx, int(mode), _ptr(M)))


def nncp_mttkrp_noalloc(X, factors, mode, M, **opts):
    """MTTKRP of one mode without a context or workspace (the library's
    per-GPU scratch array holds the temporaries); checked like Context."""
    dims, R = check_problem(X, factors)
    if not 0 <= int(mode) < len(dims):
        raise ValueError(f"mode {mode} outside [0, {len(dims)})")
    _need(M, "M", (dims[int(mode)], R), factors[0].dtype, X.device)
    o = _opts(**opts)
    return _check(lib().nncp_mttkrp_noalloc(len(dims), _dims(dims), int(R), _DT[X.dtype], _ptr(X),
                                            _DT[factors[0].dtype], _ptr_array(factors), int(mode),
                                            _ptr(M), _stream_handle(X.device), ctypes.byref(o)))


def nncp_gram(ctx, mode, G):
    return _check(lib().nncp_gram(ctx, int(mode), _ptr(G)))


def nncp_hadamard(ctx, mode, S):
    return _check(lib().nncp_hadamard(ctx, int(mode), _ptr(S)))


def nncp_update_mu(ctx, mode, M, S, eps=-1.0):
    return _check(lib().nncp_update_mu(ctx, int(mode), _ptr(M), _ptr(S), float(eps)))


def nncp_update_hals(ctx, mode, M, S):
    return _check(lib().nncp_update_hals(ctx, int(mode), _ptr(M), _ptr(S)))


def nncp_update_bpp(ctx, mode, M, S):
    return _check(lib().nncp_update_bpp(ctx, int(mode), _ptr(M), _ptr(S)))


def nncp_update_admm(ctx, mode, M, S):
    return _check(lib().nncp_update_admm(ctx, int(mode), _ptr(M), _ptr(S)))


def nncp_update_nes(ctx, mode, M, S):
    return _check(lib().nncp_update_nes(ctx, int(mode), _ptr(M), _ptr(S)))


def nncp_cp_loss(ctx, loss=None, relerr=None):
    return _check(lib().nncp_cp_loss(ctx, _ptr(loss), _ptr(relerr)))


def nncp_sweep(ctx, algo, nsweeps, relerr_hist=None):
    return _check(lib().nncp_sweep(ctx, int(algo), int(nsweeps), _ptr(relerr_hist)))


def nncp_sweep_capture(ctx, algo, nsweeps, relerr_hist=None):
    return _check(lib().nncp_sweep_capture(ctx, int(algo), int(nsweeps), _ptr(relerr_hist)))


def nncp_grad(ctx, grads, loss=None):
    return _check(lib().nncp_grad(ctx, _ptr_array(grads), _ptr(loss)))


def nncp_pgd(ctx, nsteps, armijo_c=1e-4, max_halvings=30, power_iters=50):
    lh = (ctypes.c_double * max(1, nsteps))()
    eh = (ctypes.c_double * max(1, nsteps))()
    _check(lib().nncp_pgd(ctx, int(nsteps), float(armijo_c), int(max_halvings), int(power_iters),
                          lh, eh))
    return list(lh)[:nsteps], list(eh)[:nsteps]


def nncp_destroy(ctx):
    return _check(lib().nncp_destroy(ctx))


def nncp_split(ctx) -> int:
    return _check(lib().nncp_split(ctx))


def nncp_gemm_path(ctx, side) -> int:
    return _check(lib().nncp_gemm_path(ctx, int(side)))


def nncp_uses_fused_grad(ctx) -> int:
    return _check(lib().nncp_uses_fused_grad(ctx))


def nncp_factors_changed(ctx, mode=-1):
    return _check(lib().nncp_factors_changed(ctx, int(mode)))


def nncp_read_probe(buf, workgroups=8192):
    """Launch one streaming read of the device tensor buf on the current
    stream (time it with torch events on that stream)."""
    if not isinstance(buf, torch.Tensor) or not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous GPU tensor")
    nbytes = buf.numel() * buf.element_size()
    out = torch.empty(1, dtype=torch.int32, device=buf.device)
    _check(lib().nncp_read_probe(_ptr(buf), nbytes - nbytes % 16, int(workgroups), _ptr(out),
                                 _stream_handle(buf.device)))
    return out


GEMM_PLAN_KEYS = ("mfma", "Pf", "Ps", "nsplit", "tiles", "W", "hl", "direct")


def nncp_gemm_plan(ctx, side) -> dict:
    """Launch plan of one partial MTTKRP (see include/nncp.h)."""
    info = (ctypes.c_int64 * len(GEMM_PLAN_KEYS))()
    _check(lib().nncp_gemm_plan(ctx, int(side), info))
    return dict(zip(GEMM_PLAN_KEYS, [int(v) for v in info]))


def nncp_timers_enable(ctx, on: bool):
    return _check(lib().nncp_timers_enable(ctx, 1 if on else 0))


def nncp_timers_read(ctx):
    """(milliseconds, launches) per timing category (see include/nncp.h)."""
    ms = (ctypes.c_double * NNCP_TIMER_CATEGORIES)()
    n = (ctypes.c_int64 * NNCP_TIMER_CATEGORIES)()
    _check(lib().nncp_timers_read(ctx, ms, n))
    return list(ms), list(n)


# ---------------------------------------------------------------------------
# convenience: a context that owns references to its torch buffers
# ---------------------------------------------------------------------------

def _need(t, name, shape, dtype, device):
    """Raise ValueError unless t is a contiguous tensor of this shape, dtype
    and device (checked on the host, before anything is launched: the C ABI
    only sees pointers, so a wrong size would become an out-of-bounds access)."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _factor_dtype(x_dtype):
    return torch.float64 if x_dtype == torch.float64 else torch.float32


def check_problem(X, factors, lam=None):
    """Check a tensor, its factors and lambda against each other (shapes,
    dtypes, one device, contiguity) and return (dims, R); raises ValueError.
    Runs on the host before anything is launched."""
    if not isinstance(X, torch.Tensor):
        raise ValueError("X must be a torch tensor")
    if X.dtype not in _DT:
        raise ValueError(f"X has unsupported dtype {X.dtype}")
    if not X.is_contiguous():
        raise ValueError("X must be contiguous")
    factors = list(factors)
    if not 2 <= len(factors) <= NNCP_MAX_MODES:
        raise ValueError(f"need 2..{NNCP_MAX_MODES} factors, got {len(factors)}")
    for n, f in enumerate(factors):
        if not isinstance(f, torch.Tensor) or f.dim() != 2:
            raise ValueError(f"factor {n} must be a 2-D tensor")
    dims = [int(f.shape[0]) for f in factors]
    R = int(factors[0].shape[1])
    hdt = _factor_dtype(X.dtype)
    for n, f in enumerate(factors):
        _need(f, f"factor {n}", (dims[n], R), hdt, X.device)
    total = 1
    for d in dims:
        total *= d
    if X.numel() != total:
        raise ValueError(f"X has {X.numel()} entries, the factors need {total}")
    if X.dim() > 1 and tuple(X.shape) != tuple(dims[::-1]):
        raise ValueError(f"X has shape {tuple(X.shape)}, expected {tuple(dims[::-1])} "
                         "(mode 0 fastest) or a flat tensor")
    if lam is not None and (not isinstance(lam, torch.Tensor) or lam.numel() != R):
        raise ValueError(f"lam must be a tensor of {R} entries")
    return dims, R


class Context:
    """Holds X, the factors, lambda and the workspace (torch tensors on one
    GPU) for an nncp context.  Factors are updated in place.

    X is a contiguous GPU tensor of shape (I_{N-1}, ..., I_0) or flat with
    prod(I) entries (float64, float32, bfloat16 or float16); the factors are
    contiguous (I_n, R) tensors on the same GPU, float64 for a float64 X and
    float32 otherwise; lam has R entries.  Shapes, dtypes and devices are
    checked here and in every method before the library is called."""

    def __init__(self, X, factors, lam=None, *, split=0, krp_split=1, generic=0, eps_mu=1e-16,
                 graphs=1, fused_grad=1, krp_kernel=0):
        if not isinstance(X, torch.Tensor) or not X.is_cuda:
            raise ValueError("X must be a GPU tensor")
        dims, R = check_problem(X, factors, lam)
        factors = list(factors)
        dev = X.device
        self.dims = dims
        self.R = R
        self.X = X
        self.factors = factors
        self.lam = (lam.to(device=dev, dtype=torch.float64).contiguous() if lam is not None
                    else torch.ones(self.R, dtype=torch.float64, device=dev))
        self.opts = dict(split=split, krp_split=krp_split, generic=generic, eps_mu=eps_mu,
                         graphs=graphs, fused_grad=fused_grad, krp_kernel=krp_kernel)
        nbytes = nncp_workspace_size(self.dims, self.R, _DT[X.dtype], _DT[self.factors[0].dtype],
                                     **self.opts)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.ctx = nncp_init(self.dims, self.R, self.X, self.factors, self.lam, self.workspace,
                             **self.opts)

    @property
    def N(self):
        return len(self.dims)

    @property
    def hdtype(self):
        return self.factors[0].dtype

    def split(self) -> int:
        return nncp_split(self.ctx)

    def gemm_path(self, side: int) -> int:
        return nncp_gemm_path(self.ctx, side)

    def gemm_plan(self, side: int) -> dict:
        return nncp_gemm_plan(self.ctx, side)

    def uses_fused_grad(self) -> bool:
        return bool(nncp_uses_fused_grad(self.ctx))

    def _mode(self, mode):
        if not 0 <= int(mode) < self.N:
            raise ValueError(f"mode {mode} outside [0, {self.N})")
        return int(mode)

    def _check_factors(self, factors, what="factor"):
        factors = list(factors)
        if len(factors) != self.N:
            raise ValueError(f"need {self.N} {what}s, got {len(factors)}")
        for n, f in enumerate(factors):
            _need(f, f"{what} {n}", (self.dims[n], self.R), self.hdtype, self.X.device)
        return factors

    def set_factors(self, factors, lam=None):
        factors = self._check_factors(factors)
        if lam is not None:
            _need(lam, "lam", (self.R,), torch.float64, self.X.device)
        self.factors = factors
        if lam is not None:
            self.lam = lam
        nncp_set_factors(self.ctx, self.factors, self.lam if lam is not None else None)

    def mttkrp(self, mode: int, out=None):
        mode = self._mode(mode)
        shape = (self.dims[mode], self.R)
        if out is None:
            M = torch.empty(*shape, dtype=self.hdtype, device=self.X.device)
        else:
            _need(out, "out", shape, self.hdtype, self.X.device)
            M = out
        nncp_mttkrp(self.ctx, mode, M)
        return M

    def gram(self, mode: int):
        G = torch.empty(self.R, self.R, dtype=torch.float64, device=self.X.device)
        nncp_gram(self.ctx, mode, G)
        return G

    def hadamard(self, mode: int):
        S = torch.empty(self.R, self.R, dtype=torch.float64, device=self.X.device)
        nncp_hadamard(self.ctx, mode, S)
        return S

    def update(self, algo: int, mode: int, M, S, eps: float = -1.0):
        mode = self._mode(mode)
        _need(M, "M", (self.dims[mode], self.R), self.hdtype, self.X.device)
        _need(S, "S", (self.R, self.R), torch.float64, self.X.device)
        if algo == NNCP_MU:
            nncp_update_mu(self.ctx, mode, M, S, eps)
        elif algo == NNCP_BPP:
            nncp_update_bpp(self.ctx, mode, M, S)
        elif algo == NNCP_ADMM:
            nncp_update_admm(self.ctx, mode, M, S)
        elif algo == NNCP_NES:
            nncp_update_nes(self.ctx, mode, M, S)
        else:
            nncp_update_hals(self.ctx, mode, M, S)

    def cp_loss(self):
        out = torch.empty(2, dtype=torch.float64, device=self.X.device)
        nncp_cp_loss(self.ctx, out[0:1], out[1:2])
        return out

    def _check_hist(self, relerr_hist, nsweeps):
        if relerr_hist is None:
            return
        if (not isinstance(relerr_hist, torch.Tensor) or relerr_hist.dtype != torch.float64
                or relerr_hist.device != self.X.device or not relerr_hist.is_contiguous()
                or relerr_hist.numel() < nsweeps):
            raise ValueError(f"relerr_hist must be a contiguous float64 tensor on {self.X.device} "
                             f"with at least {nsweeps} entries")

    def sweep(self, algo: int, nsweeps: int, relerr_hist=None):
        if relerr_hist is None:
            relerr_hist = torch.empty(max(1, nsweeps), dtype=torch.float64, device=self.X.device)
        self._check_hist(relerr_hist, nsweeps)
        nncp_sweep(self.ctx, algo, nsweeps, relerr_hist)
        return relerr_hist

    def capture(self, algo: int, nsweeps: int, relerr_hist):
        self._check_hist(relerr_hist, nsweeps)
        nncp_sweep_capture(self.ctx, algo, nsweeps, relerr_hist)

    def refresh_grams(self, mode: int = -1):
        """Report factor tensors overwritten in place (same buffers, so
        captured graphs stay valid): their Gram matrices are recomputed and
        no cached dimension-tree node built from the old values is reused."""
        nncp_factors_changed(self.ctx, mode)

    def grad(self, grads=None, loss=None):
        if grads is None:
            grads = [torch.empty_like(f) for f in self.factors]
        grads = self._check_factors(grads, "gradient")
        # the gradient buffers hold the MTTKRPs until the last launch: they
        # must not share memory with each other, the factors or the workspace
        spans = [(t.data_ptr(), t.data_ptr() + t.numel() * t.element_size(), name)
                 for t, name in [(g, f"gradient {n}") for n, g in enumerate(grads)]
                 + [(f, f"factor {n}") for n, f in enumerate(self.factors)]
                 + [(self.workspace, "workspace")]]
        spans.sort()
        for (a0, a1, an), (b0, b1, bn) in zip(spans, spans[1:]):
            if b0 < a1:
                raise ValueError(f"{an} and {bn} overlap")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=self.X.device)
        _need(loss, "loss", (1,), torch.float64, self.X.device)
        nncp_grad(self.ctx, grads, loss)
        return grads, loss

    def pgd(self, nsteps: int, armijo_c=1e-4, max_halvings=30, power_iters=50):
        return nncp_pgd(self.ctx, nsteps, armijo_c, max_halvings, power_iters)

    def timers_enable(self, on: bool = True):
        nncp_timers_enable(self.ctx, on)

    def timers_read(self):
        return nncp_timers_read(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            nncp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CPLoss(torch.autograd.Function):
    """L = 0.5 ||X - [[H^(0), ..., H^(N-1)]]||^2 (lambda = 1) with the
    hand-written adjoint dL/dH^(n) = H^(n) S^(n) - M^(n) computed by the
    library (all N MTTKRPs at the same point; one pass over X where the
    fused path applies, the same pass count as the loss alone, else two).

    Usage: ``CPLoss.apply(ctx, *factors)`` with ctx a ``Context`` over X."""

    @staticmethod
    def forward(fctx, ctx: Context, *factors):
        # set_factors checks every factor against the context's shapes
        ctx.set_factors([f.detach() for f in factors])
        grads = [torch.empty_like(f) for f in factors]
        loss = torch.empty(1, dtype=torch.float64, device=factors[0].device)
        nncp_grad(ctx.ctx, grads, loss)
        fctx.save_for_backward(*grads)
        return loss.reshape(()).to(factors[0].dtype)

    @staticmethod
    def backward(fctx, g):
        grads = fctx.saved_tensors
        return (None, *[g.to(t.dtype) * t for t in grads])
