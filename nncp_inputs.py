"""Seeded synthetic inputs for dense NNCP, shaped like the paper's workloads.

This module only *makes data*: factor matrices, low-rank-plus-noise tensors
and start iterates.  It holds none of the method's arithmetic (no MTTKRP, no
Gram, no update, no loss) and is shared by the oracle tests, the GPU tests
and the benchmark.  Neither the oracle nor the GPU library imports it.

Conventions
-----------
* A tensor with dims (I_0, ..., I_{N-1}) is kept in memory order with mode 0
  varying fastest, i.e. a C-contiguous array of shape (I_{N-1}, ..., I_0).
* Factors are (I_n, R) arrays, row-major.
* "p% noise" means a noise tensor scaled so that its Frobenius norm is
  p/100 of the noiseless tensor's.
* Host generation uses ``numpy.random.default_rng(seed)``; large tensors are
  made on the GPU with a seeded ``torch.Generator`` (Philox) in row chunks.
  Base seed 190901149 + workload index; start factors use seed + 1000.

The workloads (all nonnegative):
  W1  64^3 FP64, rank-8 uniform[0,1) factors + 1% uniform noise, R=8, MU.
  W2  512^3 FP32 (and its BF16 rounding), rank-32 uniform factors + 5% |Gaussian|
      noise, R=32, HALS.
  W3  256^4 BF16, rank-64 exponential(1) factors + 2% |Gaussian| noise, R=64.
  W4  1024x1024x2048 FP16 imaging-shaped: 16 separable Gaussian blobs times
      sparse exponential-decay spike trains, Poisson counts; stands in for the
      paper's mouse calcium-imaging tensor (not available here).
  W5  64^5 FP32 (+BF16 copy), rank-32 uniform factors + 1% uniform noise, R=32.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

SEED_BASE = 190901149
START_OFFSET = 1000


# ---------------------------------------------------------------------------
# host (numpy) generation
# ---------------------------------------------------------------------------

def uniform_factors(dims: Sequence[int], R: int, seed: int) -> List[np.ndarray]:
    rng = np.random.default_rng(seed)
    return [rng.random((int(d), R)) for d in dims]


def exponential_factors(dims: Sequence[int], R: int, seed: int) -> List[np.ndarray]:
    rng = np.random.default_rng(seed)
    return [rng.exponential(1.0, (int(d), R)) for d in dims]


def integer_factors(dims: Sequence[int], R: int, seed: int, hi: int = 4) -> List[np.ndarray]:
    """Small nonnegative integers (sums of products stay exact in FP64)."""
    rng = np.random.default_rng(seed)
    return [rng.integers(0, hi, (int(d), R)).astype(np.float64) for d in dims]


def integer_tensor(dims: Sequence[int], seed: int, hi: int = 5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi, int(np.prod(dims))).astype(np.float64)


def _rows_product(factors: Sequence[np.ndarray]) -> np.ndarray:
    """(prod I, R) matrix whose row for multi-index (i_a.., i_b) (first factor
    fastest) is the entrywise product of the factor rows."""
    out = factors[0]
    for f in factors[1:]:
        out = (f[:, None, :] * out[None, :, :]).reshape(-1, out.shape[1])
    return out


def lowrank_tensor(factors: Sequence[np.ndarray]) -> np.ndarray:
    """Flat (memory-order) tensor sum_r H0[:,r] o H1[:,r] o ... (float64)."""
    N = len(factors)
    s = max(1, N // 2)
    left = _rows_product(factors[:s])     # (m, R), mode 0 fastest
    right = _rows_product(factors[s:])    # (k, R)
    return (right @ left.T).reshape(-1)


def add_noise(X0: np.ndarray, kind: str, frac: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        Nz = rng.random(X0.shape)
    elif kind == "abs_gaussian":
        Nz = np.abs(rng.standard_normal(X0.shape))
    else:
        raise ValueError(kind)
    scale = frac * np.linalg.norm(X0) / np.linalg.norm(Nz)
    return X0 + scale * Nz


def workload1():
    """64^3 FP64, rank-8 + 1% uniform noise; R=8, MU, 20 sweeps."""
    seed = SEED_BASE + 0
    dims = [64, 64, 64]
    X0 = lowrank_tensor(uniform_factors(dims, 8, seed))
    X = add_noise(X0, "uniform", 0.01, seed + 1)
    H0 = uniform_factors(dims, 8, seed + START_OFFSET)
    return dict(name="64x64x64 fp64 rank-8 MU", dims=dims, R=8, X=X, H0=H0,
                algo="mu", nsweeps=20)


def small_lowrank(dims, R0, R, seed, noise=0.0, kind="uniform"):
    """Down-scaled problem of the same recipe (uniform factors, optional noise)."""
    X = lowrank_tensor(uniform_factors(dims, R0, seed))
    if noise > 0:
        X = add_noise(X, kind, noise, seed + 1)
    H0 = uniform_factors(dims, R, seed + START_OFFSET)
    return X, H0


# ---------------------------------------------------------------------------
# device (torch) generation for tensors too large to build on the host
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _rows_product_t(factors):
    out = factors[0]
    for f in factors[1:]:
        out = (f[:, None, :] * out[None, :, :]).reshape(-1, out.shape[1])
    return out


def device_lowrank_noisy(dims, factors, noise_kind, noise_frac, seed, out_dtype,
                         device="cuda", chunk_rows=None, keep_fp32=False):
    """Build X = X0 + noise on the GPU, in row chunks of the (k x m) matrix view
    (k = product of the slow half of the modes, m = the fast half).  Returns the
    stored tensor (flat, memory order) in ``out_dtype`` and, if keep_fp32, the
    fp32 tensor it was rounded from.  Noise is scaled to noise_frac of ||X0||."""
    torch = _torch()
    N = len(dims)
    s = max(1, N // 2)
    Ft = [torch.as_tensor(f, dtype=torch.float32, device=device) for f in factors]
    left = _rows_product_t(Ft[:s])    # (m, R)
    right = _rows_product_t(Ft[s:])   # (k, R)
    m, k = left.shape[0], right.shape[0]
    if chunk_rows is None:
        chunk_rows = max(1, (1 << 27) // m)
    gen = torch.Generator(device=device)

    def noise_chunk(c0, c1):
        gen.manual_seed(seed * 7919 + c0)
        if noise_kind == "uniform":
            return torch.rand((c1 - c0, m), generator=gen, device=device)
        return torch.randn((c1 - c0, m), generator=gen, device=device).abs_()

    # pass 1: norms (FP64 accumulation of FP32 chunks)
    x0sq = 0.0
    nzsq = 0.0
    for c0 in range(0, k, chunk_rows):
        c1 = min(k, c0 + chunk_rows)
        x0 = right[c0:c1] @ left.T
        x0sq += float(torch.sum(x0.double() ** 2))
        if noise_frac > 0:
            nz = noise_chunk(c0, c1)
            nzsq += float(torch.sum(nz.double() ** 2))
    scale = noise_frac * math.sqrt(x0sq) / math.sqrt(nzsq) if noise_frac > 0 else 0.0
    out = torch.empty(k * m, dtype=out_dtype, device=device)
    full = torch.empty(k * m, dtype=torch.float32, device=device) if keep_fp32 else None
    for c0 in range(0, k, chunk_rows):
        c1 = min(k, c0 + chunk_rows)
        x = right[c0:c1] @ left.T
        if noise_frac > 0:
            x.add_(noise_chunk(c0, c1), alpha=scale)
        out[c0 * m:c1 * m] = x.reshape(-1).to(out_dtype)
        if full is not None:
            full[c0 * m:c1 * m] = x.reshape(-1)
    return out, full


def workload2(device="cuda", keep_fp32=True):
    """512^3, rank-32 uniform factors + 5% |Gaussian| noise; FP32 and BF16."""
    torch = _torch()
    seed = SEED_BASE + 1
    dims = [512, 512, 512]
    F = uniform_factors(dims, 32, seed)
    x32, _ = device_lowrank_noisy(dims, F, "abs_gaussian", 0.05, seed + 1, torch.float32, device)
    xbf = x32.to(torch.bfloat16)  # round to nearest even, once
    H0 = uniform_factors(dims, 32, seed + START_OFFSET)
    return dict(name="512x512x512 rank-32 HALS", dims=dims, R=32, X32=x32, Xbf16=xbf, H0=H0,
                algo="hals", nsweeps=50)


def workload3(device="cuda"):
    """256^4 BF16, rank-64 exponential(1) factors + 2% |Gaussian| noise."""
    torch = _torch()
    seed = SEED_BASE + 2
    dims = [256, 256, 256, 256]
    F = exponential_factors(dims, 64, seed)
    xbf, _ = device_lowrank_noisy(dims, F, "abs_gaussian", 0.02, seed + 1, torch.bfloat16, device)
    H0 = uniform_factors(dims, 64, seed + START_OFFSET)
    return dict(name="256^4 bf16 rank-64 HALS", dims=dims, R=64, X=xbf, H0=H0, algo="hals",
                nsweeps=50)


def imaging_components(dims=(1024, 1024, 2048), R=16, seed=SEED_BASE + 3,
                       spike_p=0.01, sigma=(5.0, 40.0), tau=(5.0, 50.0)):
    """Spatial Gaussian blobs (separable, so rank one in (x, y)) and temporal
    exponential-decay spike trains.  Returns host factors A (Ix x R),
    B (Iy x R), C (It x R)."""
    rng = np.random.default_rng(seed)
    Ix, Iy, It = dims
    sig = rng.uniform(sigma[0], sigma[1], R)
    cx = rng.uniform(0, Ix, R)
    cy = rng.uniform(0, Iy, R)
    x = np.arange(Ix)[:, None]
    y = np.arange(Iy)[:, None]
    A = np.exp(-((x - cx[None, :]) ** 2) / (2 * sig[None, :] ** 2))
    B = np.exp(-((y - cy[None, :]) ** 2) / (2 * sig[None, :] ** 2))
    taus = rng.uniform(tau[0], tau[1], R)
    C = np.zeros((It, R))
    for r in range(R):
        spikes = rng.random(It) < spike_p
        amps = rng.exponential(1.0, It) * spikes
        acc = 0.0
        decay = math.exp(-1.0 / taus[r])
        for t in range(It):
            acc = acc * decay + amps[t]
            C[t, r] = acc
    return A, B, C


def workload4(device="cuda", dims=(1024, 1024, 2048), R=16):
    """Imaging-shaped FP16 tensor: Poisson(kappa X0)/kappa, kappa = 100/max X0."""
    torch = _torch()
    seed = SEED_BASE + 3
    A, B, C = imaging_components(dims, R, seed)
    Ft = [torch.as_tensor(f, dtype=torch.float32, device=device) for f in (A, B, C)]
    left = _rows_product_t(Ft[:2])       # (Ix*Iy, R)
    right = Ft[2]                        # (It, R)
    m, k = left.shape[0], right.shape[0]
    # max of X0 over all entries, chunked
    xmax = 0.0
    rows = max(1, (1 << 27) // m)
    for c0 in range(0, k, rows):
        xmax = max(xmax, float((right[c0:c0 + rows] @ left.T).max()))
    kappa = 100.0 / xmax
    gen = torch.Generator(device=device)
    out = torch.empty(k * m, dtype=torch.float16, device=device)
    for c0 in range(0, k, rows):
        c1 = min(k, c0 + rows)
        gen.manual_seed((seed + 1) * 7919 + c0)
        lam = (right[c0:c1] @ left.T).clamp_min_(0).mul_(kappa)
        out[c0 * m:c1 * m] = (torch.poisson(lam, generator=gen) / kappa).reshape(-1).to(torch.float16)
    H0 = uniform_factors(list(dims), R, seed + START_OFFSET)
    return dict(name="imaging 1024x1024x2048 fp16", dims=list(dims), R=R, X=out, H0=H0,
                kappa=kappa)


def workload5(device="cuda", keep_bf16=True):
    """64^5 FP32 (+BF16 copy), rank-32 uniform factors + 1% uniform noise."""
    torch = _torch()
    seed = SEED_BASE + 4
    dims = [64] * 5
    F = uniform_factors(dims, 32, seed)
    x32, _ = device_lowrank_noisy(dims, F, "uniform", 0.01, seed + 1, torch.float32, device)
    H0 = uniform_factors(dims, 32, seed + START_OFFSET)
    d = dict(name="64^5 rank-32 gradient", dims=dims, R=32, X32=x32, H0=H0)
    if keep_bf16:
        d["Xbf16"] = x32.to(torch.bfloat16)
    return d
