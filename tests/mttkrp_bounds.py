"""Entrywise error bound of a BF16/FP16-tensor MTTKRP against the exact
(FP64) MTTKRP of the same stored tensor.

Every quantity is nonnegative (tensor, factors), so each term X(idx) K(idx, r)
of M^(n)(i, r) = sum_idx X(idx) K(idx, r) enters with a positive sign, and a
relative perturbation of every term by at most c gives |dM| <= c M entrywise.
The terms are perturbed by:
  * the Khatri-Rao operand held on chip in the tensor's 16-bit type: a hi + lo
    pair carries it to 2^-16 (BF16) or 2^-22 (FP16) relative, a single rounding
    to 2^-8 / 2^-11 (unit roundoff of the format, squared for the pair);
  * the slow part of the operand rounded to FP32 once (2^-24);
  * FP32 arithmetic on the way into M: every term passes through at most D
    roundings (products and additions), so it is scaled by at most
    (1 + 2^-24)^D - 1 <= gamma_D = D u / (1 - D u), u = 2^-24.
D follows the kernels' accumulation structure, read from the launch plan
(nncp_gemm_plan): one accumulator block of Pf reduced indices (twice that
for a hi + lo operand), the Ps blocks after it (a product and an addition
each), the waves and the split partials, then one multi-TTV per tree level
(its reduction length plus the product roundings).
FP16 only: entries of the operand below FP16's normal range after the
per-column power-of-two scaling (largest entry in [2^13, 2^14)) are held with
an absolute error of at most 2^-25 in scaled units, i.e. colmax * 2^-38; a
term's operand error is then at most 2^-38 prod_{k != n} max_i H^(k)(i, r),
which adds 2^-38 P_r sum_{idx: i_n = i} X(idx) to the bound.
"""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24


def gamma(n: int, u: float = U32) -> float:
    return n * u / (1.0 - n * u)


def depth(dims, S, n, plans) -> int:
    """Upper bound on the FP32 roundings one term passes through into
    M^(n) (plans[side] = the dict of nncp_gemm_plan)."""
    N = len(dims)
    side = 0 if n < S else 1
    p = plans[side]
    lo, hi = (0, S) if side == 0 else (S, N)
    red = math.prod(dims[S:]) if side == 0 else math.prod(dims[:S])
    if p["mfma"]:
        d = (2 if p["hl"] else 1) * p["Pf"] + 2 * p["Ps"] + 8 + p["nsplit"] + 2
    else:
        d = red + p["nsplit"] + 16
    for a in range(lo + 1, n + 1):          # contiguous multi-TTVs down to n
        d += dims[a - 1] + 1
    if n < hi - 1:                          # strided multi-TTV over the rest
        d += math.prod(dims[n + 1:hi]) + (hi - n - 1) + 1
    return d


def rel_bound(xdt: str, dims, S, n, plans) -> float:
    hl = plans[0 if n < S else 1]["hl"]
    uK = {"bf16": 2.0 ** -16 if hl else 2.0 ** -8,
          "f16": 2.0 ** -22 if hl else 2.0 ** -11}[xdt]
    return uK + U32 + gamma(depth(dims, S, n, plans)) + len(dims) * 2.0 ** -50


def abs_term_f16(Hh, n, slice_sums) -> np.ndarray:
    """(rows x R) absolute part of the FP16 bound for rows with the given
    sums of their tensor slices."""
    P = np.ones(Hh[0].shape[1])
    for k, h in enumerate(Hh):
        if k != n:
            P = P * h.max(axis=0)
    return 2.0 * 2.0 ** -38 * np.outer(np.asarray(slice_sums, dtype=np.float64), P)


def check(M, Mref, xdt, dims, S, n, plans, Hh=None, slice_sums=None):
    """Assert |M - Mref| <= c Mref (+ the FP16 absolute term) entrywise and
    return (max entrywise relative error, c)."""
    M = np.asarray(M, dtype=np.float64)
    Mref = np.asarray(Mref, dtype=np.float64)
    assert np.all(Mref >= 0)
    c = rel_bound(xdt, dims, S, n, plans)
    allow = c * Mref
    if xdt == "f16":
        allow = allow + abs_term_f16(Hh, n, slice_sums)
    err = np.abs(M - Mref)
    bad = err > allow
    assert not bad.any(), (n, xdt, int(bad.sum()), float((err - allow).max()), c)
    pos = Mref > 0
    return float((err[pos] / Mref[pos]).max()), c
