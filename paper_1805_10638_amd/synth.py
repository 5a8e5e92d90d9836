"""Seeded synthetic inputs for the K-Means workloads.

This module only draws random numbers and stores them in the requested
element type.  It contains none of the clustering arithmetic (no distances,
no means, no energies), so both the GPU library and the CPU reference can
consume its arrays without sharing any part of the method.

Every generator takes an explicit seed tuple; the same tuple always yields
bit-identical arrays (NumPy PCG64).

Workloads (all Gaussian mixtures; the paper's real datasets are not used):
  * ``plain_small``   N=10,000 d=2 K=10: 10 isotropic unit-variance
    components, centres uniform in [-10,10]^2, equal weights.
  * ``plain_large``   N=1,000,000 d=32 K=256: centres N(0, 25 I), per
    component and per dimension standard deviation U[0.5, 2], Dirichlet(1)
    weights.
  * ``precision``     N=4,000,000 d=128 K=1024: 1024 centres N(0, 4 I),
    95 % inliers centre + N(0, I) with uniform component choice, 5 % outliers
    uniform over the inliers' axis-aligned bounding box, rows shuffled,
    stored as bfloat16.
  * ``instance_sizes``  per-instance (N, d, K) for batched/served streams:
    N log-uniform in [2e3, 2e5], d from {3, 16, 64}, K log-uniform in [8, 512].
"""

from __future__ import annotations

import numpy as np

SEED_BASE = 180510638


def rng_for(*key: int) -> np.random.Generator:
    """PCG64 generator keyed by ``[SEED_BASE, *key]``."""
    return np.random.Generator(np.random.PCG64([SEED_BASE, *[int(k) for k in key]]))


# ---------------------------------------------------------------------------
# bfloat16 storage (round-to-nearest-even of float32 bit patterns)
# ---------------------------------------------------------------------------

def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 array -> uint16 bfloat16 bit patterns, round to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (u >> np.uint32(16)) & np.uint32(1)
    r = (u + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """uint16 bfloat16 bit patterns -> the float32 values they denote (exact)."""
    return (np.ascontiguousarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


# ---------------------------------------------------------------------------
# Mixtures
# ---------------------------------------------------------------------------

def gaussian_mixture(rng: np.random.Generator, n: int, centers: np.ndarray,
                     stds: np.ndarray, weights: np.ndarray | None) -> np.ndarray:
    """Draw ``n`` float32 rows x = centers[z] + stds[z] * N(0, I), z ~ Cat(weights)."""
    k, d = centers.shape
    if weights is None:
        z = rng.integers(0, k, size=n)
    else:
        z = rng.choice(k, size=n, p=weights)
    noise = rng.standard_normal((n, d), dtype=np.float32)
    x = centers.astype(np.float32)[z] + stds.astype(np.float32)[z] * noise
    return np.ascontiguousarray(x, dtype=np.float32), z


def plain_small(rep: int = 0, n: int = 10_000, k: int = 10):
    """N=10,000, d=2, K=10 mixture; returns (X float32 [n,2], component labels)."""
    rng = rng_for(1, rep)
    centers = rng.uniform(-10.0, 10.0, size=(k, 2))
    stds = np.ones((k, 2))
    return gaussian_mixture(rng, n, centers, stds, None)


def plain_large(rep: int = 0, n: int = 1_000_000, d: int = 32, k: int = 256, cfg: int = 2):
    """N=1M, d=32, K=256 mixture (defaults); returns (X float32 [n,d], labels)."""
    rng = rng_for(cfg, rep)
    centers = rng.normal(0.0, 5.0, size=(k, d))
    stds = rng.uniform(0.5, 2.0, size=(k, d))
    weights = rng.dirichlet(np.ones(k))
    return gaussian_mixture(rng, n, centers, stds, weights)


def precision(rep: int = 0, n: int = 4_000_000, d: int = 128, k: int = 1024,
              outlier_frac: float = 0.05):
    """Inliers around N(0,4I) centres plus uniform outliers; returns
    (X bfloat16 bits uint16 [n,d], labels with -1 for outliers)."""
    rng = rng_for(3, rep)
    centers = rng.normal(0.0, 2.0, size=(k, d))
    n_out = int(round(outlier_frac * n))
    n_in = n - n_out
    xin, z = gaussian_mixture(rng, n_in, centers, np.ones((k, d)), None)
    lo = xin.min(axis=0)
    hi = xin.max(axis=0)
    xout = rng.uniform(lo, hi, size=(n_out, d)).astype(np.float32)
    x = np.concatenate([xin, xout], axis=0)
    lab = np.concatenate([z, -np.ones(n_out, dtype=z.dtype)])
    order = rng.permutation(n)
    return to_bf16_bits(x[order]), lab[order]


def instance_sizes(count: int, rep: int = 0, cfg: int = 4):
    """(N, d, K) triples for a batch/stream of independent instances."""
    rng = rng_for(cfg, rep)
    ns = np.round(np.exp(rng.uniform(np.log(2e3), np.log(2e5), size=count))).astype(np.int64)
    ds = rng.choice(np.array([3, 16, 64]), size=count)
    ks = np.round(np.exp(rng.uniform(np.log(8), np.log(512), size=count))).astype(np.int64)
    ks = np.minimum(ks, ns)
    return [(int(a), int(b), int(c)) for a, b, c in zip(ns, ds, ks)]


def instance(n: int, d: int, k: int, seed: int, cfg: int = 4):
    """One mixture instance of the batched workload: same law as plain_large
    with ``k`` components in ``d`` dimensions."""
    return plain_large(rep=seed, n=n, d=d, k=k, cfg=100 + cfg)


# ---------------------------------------------------------------------------
# Initial centroids: K distinct samples chosen by a seeded generator
# ---------------------------------------------------------------------------

def init_indices(n: int, k: int, seed: int) -> np.ndarray:
    """K distinct row indices in [0, n)."""
    rng = rng_for(1_000_000, seed)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def init_centroids(x: np.ndarray, k: int, seed: int) -> np.ndarray:
    """Rows of ``x`` at :func:`init_indices` (float32 copy; bfloat16 bit
    arrays are decoded to their float32 values)."""
    idx = init_indices(x.shape[0], k, seed)
    rows = x[idx]
    if rows.dtype == np.uint16:
        rows = bf16_bits_to_f32(rows)
    return np.ascontiguousarray(rows, dtype=np.float32)


# ---------------------------------------------------------------------------
# On-device generation for the batched and served streams (torch generator;
# the law of plain_large, drawn on the GPU so that thousands of instances
# cost milliseconds each)
# ---------------------------------------------------------------------------

def device_instance(n: int, d: int, k: int, seed: int, device="cuda", bf16: bool = False):
    """(X, C0) on ``device``: a k-component mixture with centres N(0, 25 I),
    per-component per-dimension std U[0.5, 2], Dirichlet(1) weights; X float32,
    or bfloat16 stored as int16 bit patterns (round to nearest even); C0 = k
    distinct rows of X as float32."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(SEED_BASE * 7919 + int(seed))
    centers = 5.0 * torch.randn(k, d, generator=g, device=device)
    stds = 0.5 + 1.5 * torch.rand(k, d, generator=g, device=device)
    w = -torch.log(torch.rand(k, generator=g, device=device).clamp_min(1e-30))   # Gamma(1) draws
    z = torch.multinomial(w / w.sum(), n, replacement=True, generator=g)
    x = centers[z] + stds[z] * torch.randn(n, d, generator=g, device=device)
    idx = torch.randperm(n, generator=g, device=device)[:k]
    if bf16:
        xb = x.to(torch.bfloat16)
        c0 = xb[idx].to(torch.float32).contiguous()
        return xb.view(torch.int16).contiguous(), c0
    return x.contiguous(), x[idx].contiguous()
