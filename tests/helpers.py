"""Shared helpers of the GPU parity tests (oracle comparisons)."""

from __future__ import annotations

import numpy as np

from oracle import kmeans_oracle as ko
from paper_1805_10638_amd import synth


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def x_tensor(x):
    """float32 array -> float32 tensor; uint16 bf16 bits -> int16 tensor of the bits."""
    import torch
    if x.dtype == np.uint16:
        return dev(x.view(np.int16))
    return dev(x.astype(np.float32))


def x_values(x):
    """Stored values of X as float64 (bf16 bits decoded exactly)."""
    if x.dtype == np.uint16:
        return synth.bf16_bits_to_f32(x).astype(np.float64)
    return x.astype(np.float64)


def spread(X64):
    """RMS deviation of the samples from their mean (scale for centroid errors)."""
    return float(np.sqrt(((X64 - X64.mean(axis=0)) ** 2).sum(axis=1).mean()))


def centroid_errors(Cg, Co, X64):
    """Per-centroid ||dc|| / max(||c||, s_X)."""
    s = spread(X64)
    num = np.linalg.norm(np.asarray(Cg, np.float64) - Co, axis=1)
    den = np.maximum(np.linalg.norm(Co, axis=1), s)
    return num / np.maximum(den, 1e-300)


def check_g(X, C32, rho, Cn, E, rows=None, rtol_c=1e-5, rtol_e=1e-6):
    """Tier-1 parity of one G application against the oracle.

    Labels must equal the oracle's except on oracle near ties; centroids are
    compared with the oracle's means of the GPU labels; E with the oracle's
    energy of its own labels.  With ``rows`` only those rows are checked for
    labels (full-size runs) and E is compared with the oracle energy of the
    GPU labels.  Returns a dict of counts."""
    X64 = x_values(X)
    C64 = C32.astype(np.float64)
    rho = np.asarray(rho).astype(np.int64)
    if rows is None:
        a = ko.assign(X64, C64)
        mism = np.flatnonzero(a.rho != rho)
        bad = mism[~a.near_tie[mism]]
        assert bad.size == 0, f"{bad.size} label mismatches outside near ties, e.g. rows {bad[:5]}"
        Eo = ko.energy(X64, a.rho, C64)
        near = int(a.near_tie.sum())
    else:
        a = ko.assign(X64[rows], C64)
        mism = np.flatnonzero(a.rho != rho[rows])
        bad = mism[~a.near_tie[mism]]
        assert bad.size == 0, f"{bad.size} sampled label mismatches outside near ties"
        Eo = ko.energy(X64, rho, C64)
        near = int(a.near_tie.sum())
    assert abs(E - Eo) <= rtol_e * abs(Eo), (E, Eo)
    Co, _ = ko.update(X64, rho, C64)
    err = centroid_errors(Cn, Co, X64)
    assert err.max() <= rtol_c, err.max()
    return {"mismatch": int(mism.size), "near_ties": near, "max_c_err": float(err.max())}
