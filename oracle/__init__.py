"""CPU FP64 oracle for dense nonnegative CP by alternating updates.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the GPU library (``paper_1909_01149_amd``) and neither imports the other.

The arithmetic lives in ``nncp_oracle.c`` (plain C, FP64), which follows the
paper's definitions (PLANC, arXiv 1909.01149): MTTKRP by its entrywise
definition (Section 4.2.1, Appendix B), Algorithm 1 with the MU rule
(Eq. eqn:muupd) and the HALS rule (Eq. eqn:halsupd), column normalisation and
the relative-error identity (Appendix B, Algorithm 4).  This module only
marshals NumPy arrays into that library.

Layout conventions: a tensor with dims (I_0, ..., I_{N-1}) is a 1-D float64
array in memory order with mode 0 fastest (NumPy: ``x.reshape(dims[::-1])``
in C order).  Factors are (I_n, R) float64 C-contiguous arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nncp_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

MU = 0
HALS = 1
BPP = 2
ADMM = 3
NES = 4
NES_OUTER = 5


def build(force: bool = False) -> str:
    """Compile nncp_oracle.c into a shared library next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load(path: str) -> ctypes.CDLL:
    """Open an oracle shared library and declare its entry points."""
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    d = ctypes.c_double
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    pd = P(d)
    ppd = P(pd)
    pi64 = P(i64)
    L.orc_mttkrp.argtypes = [ci, pi64, ci, pd, ppd, ci, pd, ci]
    L.orc_mttkrp_rows.argtypes = [ci, pi64, ci, pd, ppd, ci, pi64, ci, pd, ci]
    L.orc_gram.argtypes = [i64, ci, pd, pd]
    L.orc_hadamard_except.argtypes = [ci, ci, ppd, ci, pd]
    L.orc_sumsq.argtypes = [i64, pd]
    L.orc_sumsq.restype = d
    L.orc_update_mu.argtypes = [i64, ci, pd, pd, pd, d]
    L.orc_update_hals.argtypes = [i64, ci, pd, pd, pd]
    L.orc_normalize.argtypes = [i64, ci, pd, pd, pd]
    L.orc_update_bpp.argtypes = [i64, ci, pd, pd, pd]
    L.orc_update_bpp.restype = i64
    L.orc_bpp_row.argtypes = [ci, pd, pd, pd, pd]
    L.orc_bpp_row.restype = ci
    L.orc_update_admm.argtypes = [i64, ci, pd, pd, pd, pd, ci, d]
    L.orc_update_admm.restype = ci
    L.orc_nes_params.argtypes = [ci, pd, ci, d, pd]
    L.orc_nes_params.restype = ci
    L.orc_update_nes.argtypes = [i64, ci, pd, pd, pd, ci, ci, d]
    L.orc_update_nes.restype = ci
    L.orc_nes_outer_candidate.argtypes = [ci, pi64, ci, pd, ppd, pd, ppd, pd, d, d, ppd, pd, ci]
    L.orc_nes_outer_candidate.restype = d
    L.orc_sweeps.argtypes = [ci, pi64, ci, pd, ppd, pd, ci, d, ci, pd, pd, ci]
    L.orc_sweeps_from.argtypes = [ci, pi64, ci, pd, ppd, pd, ci, d, ci, i64, pd, pd, ci]
    L.orc_residual.argtypes = [ci, pi64, ci, pd, ppd, pd, pd]
    L.orc_residual.restype = d
    L.orc_grad.argtypes = [ci, pi64, ci, pd, ppd, ppd, ci]
    L.orc_grad.restype = d
    L.orc_power_lmax.argtypes = [ci, pd, ci]
    L.orc_power_lmax.restype = d
    L.orc_pgd.argtypes = [ci, pi64, ci, pd, ppd, ci, d, ci, ci, pd, pd, ci]
    L.orc_max_threads.restype = ci
    return L


# a different build of the same source (the sanitizer build) can be selected
# for a whole process through this environment variable
_ENV_LIB = "NNCP_ORACLE_LIB"


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get(_ENV_LIB)
        if not path:
            path = build()
        _lib = _load(path)
    return _lib


SANITIZE_FLAGS = ("-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-omit-frame-pointer")


def build_sanitized(out_path: str) -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only; load it into a process started with libasan preloaded
    and NNCP_ORACLE_LIB pointing at it)."""
    return build_variant(out_path, extra_flags=SANITIZE_FLAGS)


class using_library:
    """Context manager: route every oracle call through another build of the
    oracle source (the sanitizer build, or a deliberately altered copy that
    the pin tests use to show that a planted mistake is caught)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def build_variant(out_path: str, source: str | None = None, extra_flags=()) -> str:
    """Compile the oracle (or the given replacement source text) into
    out_path with extra compiler flags; returns out_path."""
    src = _SRC
    tmp_src = None
    if source is not None:
        tmp_src = out_path + ".c"
        with open(tmp_src, "w") as f:
            f.write(source)
        src = tmp_src
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           *extra_flags, src, "-o", out_path, "-lm"])
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _pd(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int64))
    return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _ptr_array(arrs):
    arr = (ctypes.POINTER(ctypes.c_double) * len(arrs))(*[_pd(a) for a in arrs])
    return arr


def mttkrp(X, factors, mode: int, nthreads: int = 1) -> np.ndarray:
    """M^(mode) by its definition.  X: flat memory-order tensor; factors: list of (I_n, R)."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    X = _f64(X).reshape(-1)
    Hs = [_f64(f) for f in factors]
    d, dp = _dims(dims)
    M = np.zeros((dims[mode], R), dtype=np.float64)
    rc = lib().orc_mttkrp(len(dims), dp, R, _pd(X), _ptr_array(Hs), mode, _pd(M), nthreads)
    if rc != 0:
        raise ValueError(f"orc_mttkrp failed ({rc})")
    return M


def mttkrp_rows(X, factors, mode: int, rows, nthreads: int = 1) -> np.ndarray:
    """Selected rows of M^(mode) (one row costs 2 (I/I_n) R flops)."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    X = _f64(X).reshape(-1)
    Hs = [_f64(f) for f in factors]
    d, dp = _dims(dims)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.zeros((len(rows), R), dtype=np.float64)
    rc = lib().orc_mttkrp_rows(len(dims), dp, R, _pd(X), _ptr_array(Hs), mode,
                               rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               len(rows), _pd(out), nthreads)
    if rc != 0:
        raise ValueError(f"orc_mttkrp_rows failed ({rc})")
    return out


def gram(H) -> np.ndarray:
    H = _f64(H)
    I, R = H.shape
    G = np.zeros((R, R), dtype=np.float64)
    lib().orc_gram(I, R, _pd(H), _pd(G))
    return G


def hadamard_except(grams, mode: int) -> np.ndarray:
    Gs = [_f64(g) for g in grams]
    R = Gs[0].shape[0]
    S = np.zeros((R, R), dtype=np.float64)
    lib().orc_hadamard_except(len(Gs), R, _ptr_array(Gs), mode, _pd(S))
    return S


def sumsq(X) -> float:
    X = _f64(X).reshape(-1)
    return float(lib().orc_sumsq(X.size, _pd(X)))


def update_mu(Hhat, M, S, eps: float = 1e-16) -> np.ndarray:
    H = _f64(Hhat).copy()
    M = _f64(M)
    S = _f64(S)
    lib().orc_update_mu(H.shape[0], H.shape[1], _pd(H), _pd(M), _pd(S), eps)
    return H


def update_hals(Hhat, M, S) -> np.ndarray:
    H = _f64(Hhat).copy()
    M = _f64(M)
    S = _f64(S)
    lib().orc_update_hals(H.shape[0], H.shape[1], _pd(H), _pd(M), _pd(S))
    return H


def update_bpp(M, S, Hhat0=None):
    """Exact NNLS solve of every row (BPP), each search starting from the
    support of Hhat0's row (all zero if None).  Returns (Hhat, failed_rows)."""
    M = _f64(M)
    S = _f64(S)
    H = np.zeros_like(M) if Hhat0 is None else _f64(Hhat0).copy()
    failed = lib().orc_update_bpp(M.shape[0], M.shape[1], _pd(H), _pd(M), _pd(S))
    return H, int(failed)


def bpp_row(S, m, x0=None):
    """One row: returns (x, number of solves or -1); x0 gives the start support."""
    S = _f64(S)
    m = _f64(m)
    R = m.shape[0]
    x = np.zeros(R) if x0 is None else _f64(x0).copy()
    work = np.zeros(R * R + 4 * R)
    n = lib().orc_bpp_row(R, _pd(S), _pd(m), _pd(x), _pd(work))
    return x, int(n)


def update_admm(Hhat, U, M, S, maxit: int = 5, tol: float = 0.01):
    """ADMM passes from the start value Hhat with dual U.  Returns
    (Hhat, U, passes)."""
    H = _f64(Hhat).copy()
    Uc = _f64(U).copy()
    M = _f64(M)
    S = _f64(S)
    n = lib().orc_update_admm(H.shape[0], H.shape[1], _pd(H), _pd(Uc), _pd(M), _pd(S), int(maxit),
                              float(tol))
    return H, Uc, int(n)


def nes_params(S, power: int = 20, kappa: float = 100.0):
    """Step parameters of the Nesterov-type update: (L, mu, lam, alpha, beta, ok)."""
    S = _f64(S)
    out = np.zeros(5)
    rc = lib().orc_nes_params(S.shape[0], _pd(S), int(power), float(kappa), _pd(out))
    return (*[float(v) for v in out], rc == 0)


def update_nes(Hhat, M, S, iters: int = 20, power: int = 20, kappa: float = 100.0):
    """Nesterov-type update from the start value Hhat (also the proximal
    centre).  Returns (Hhat, ok)."""
    H = _f64(Hhat).copy()
    M = _f64(M)
    S = _f64(S)
    rc = lib().orc_update_nes(H.shape[0], H.shape[1], _pd(H), _pd(M), _pd(S), int(iters),
                              int(power), float(kappa))
    return H, rc == 0


def normalize(Hhat):
    Hhat = _f64(Hhat)
    H = np.zeros_like(Hhat)
    lam = np.zeros(Hhat.shape[1], dtype=np.float64)
    lib().orc_normalize(Hhat.shape[0], Hhat.shape[1], _pd(Hhat), _pd(H), _pd(lam))
    return H, lam


def sweeps(X, factors, lam, algo: int, nsweeps: int, eps_mu: float = 1e-16, nthreads: int = 1,
           first_sweep: int = 1):
    """Run nsweeps outer iterations, the first being outer iteration
    first_sweep (it sets s_i of the outer extrapolation).  Returns
    (factors, lambda, relerr, relerr2_raw)."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    X = _f64(X).reshape(-1)
    Hs = [_f64(f).copy() for f in factors]
    lam = _f64(lam).copy()
    d, dp = _dims(dims)
    rel = np.zeros(nsweeps, dtype=np.float64)
    raw = np.zeros(nsweeps, dtype=np.float64)
    rc = lib().orc_sweeps_from(len(dims), dp, R, _pd(X), _ptr_array(Hs), _pd(lam), algo,
                               eps_mu, nsweeps, int(first_sweep), _pd(rel), _pd(raw), nthreads)
    if rc != 0:
        raise ValueError(f"orc_sweeps failed ({rc})")
    return Hs, lam, rel, raw


def nes_outer_candidate(X, factors, lam, prev_factors, prev_lam, si: float, nthreads: int = 1):
    """Candidate of the outer extrapolation (Eq. eqn:nesouterupd) from the
    iterate after a sweep and the one before it, with step si.  Returns
    (normalised candidate factors, lambda_c, squared relative error)."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    X = _f64(X).reshape(-1)
    Hs = [_f64(f) for f in factors]
    Hp = [_f64(f) for f in prev_factors]
    lam = _f64(lam)
    lamp = _f64(prev_lam)
    Hc = [np.zeros_like(h) for h in Hs]
    lamc = np.zeros(R)
    d, dp = _dims(dims)
    e2 = lib().orc_nes_outer_candidate(len(dims), dp, R, _pd(X), _ptr_array(Hs), _pd(lam),
                                       _ptr_array(Hp), _pd(lamp), float(si), sumsq(X),
                                       _ptr_array(Hc), _pd(lamc), nthreads)
    return Hc, lamc, float(e2)


def residual(X, factors, lam=None, want_tensor: bool = False):
    """0.5 ||X - [[lam; H]]||^2 by explicit reconstruction (and the residual tensor)."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    X = _f64(X).reshape(-1)
    Hs = [_f64(f) for f in factors]
    d, dp = _dims(dims)
    E = np.zeros(X.size, dtype=np.float64) if want_tensor else None
    lam_keep = _f64(lam) if lam is not None else None
    lp = _pd(lam_keep) if lam_keep is not None else ctypes.POINTER(ctypes.c_double)()
    L = lib().orc_residual(len(dims), dp, R, _pd(X), _ptr_array(Hs), lp,
                           _pd(E) if E is not None else ctypes.POINTER(ctypes.c_double)())
    return (float(L), E) if want_tensor else float(L)


def grad(X, factors, nthreads: int = 1):
    """(L, [dL/dH^(n)]) for L = 0.5 ||X - [[H]]||^2 with lambda = 1."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    X = _f64(X).reshape(-1)
    Hs = [_f64(f) for f in factors]
    gs = [np.zeros_like(h) for h in Hs]
    d, dp = _dims(dims)
    L = lib().orc_grad(len(dims), dp, R, _pd(X), _ptr_array(Hs), _ptr_array(gs), nthreads)
    return float(L), gs


def power_lmax(A, iters: int = 50) -> float:
    A = _f64(A)
    return float(lib().orc_power_lmax(A.shape[0], _pd(A), iters))


def pgd(X, factors, nsteps: int, armijo_c: float = 1e-4, max_halvings: int = 30,
        power_iters: int = 50, nthreads: int = 1):
    """Projected-gradient steps with Armijo backtracking.  Returns (factors, loss_hist, eta_hist)."""
    dims = [f.shape[0] for f in factors]
    R = factors[0].shape[1]
    X = _f64(X).reshape(-1)
    Hs = [_f64(f).copy() for f in factors]
    d, dp = _dims(dims)
    lh = np.zeros(nsteps, dtype=np.float64)
    eh = np.zeros(nsteps, dtype=np.float64)
    rc = lib().orc_pgd(len(dims), dp, R, _pd(X), _ptr_array(Hs), nsteps, armijo_c,
                       max_halvings, power_iters, _pd(lh), _pd(eh), nthreads)
    if rc != 0:
        raise ValueError(f"orc_pgd failed ({rc})")
    return Hs, lh, eh
