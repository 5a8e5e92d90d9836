"""Seeded generators: reproducibility and the stated distributions."""

import numpy as np
import pytest

from paper_1805_10638_amd import synth


def test_same_seed_same_bits():
    a, za = synth.plain_small(rep=4)
    b, zb = synth.plain_small(rep=4)
    assert a.dtype == np.float32 and a.shape == (10_000, 2)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(za, zb)
    c, _ = synth.plain_small(rep=5)
    assert not np.array_equal(a, c)


def test_plain_large_shape_and_moments():
    x, z = synth.plain_large(rep=0, n=200_000)
    assert x.shape == (200_000, 32) and x.dtype == np.float32
    assert z.max() < 256
    # centre spread N(0,25 I): overall per-dimension variance is ~25 + E[std^2] ~ 26.75
    v = x.var(axis=0).mean()
    assert 20.0 < v < 34.0


def test_precision_bf16_and_outliers():
    xb, lab = synth.precision(rep=0, n=20_000, d=16, k=32)
    assert xb.dtype == np.uint16 and xb.shape == (20_000, 16)
    assert (lab == -1).sum() == 1000
    x = synth.bf16_bits_to_f32(xb)
    assert np.isfinite(x).all()
    # round trip of representable values is exact
    assert np.array_equal(synth.to_bf16_bits(x), xb)


def test_bf16_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, -2.5, 1.0 + 2**-9], dtype=np.float32)
    got = synth.bf16_bits_to_f32(synth.to_bf16_bits(vals))
    want = np.array([1.0, 1.0, 1.0 + 4 * 2**-8, -2.5, 1.0], dtype=np.float32)
    assert np.array_equal(got, want)


def test_init_distinct_rows():
    x, _ = synth.plain_small(rep=0)
    idx = synth.init_indices(x.shape[0], 10, 3)
    assert len(set(idx.tolist())) == 10
    c = synth.init_centroids(x, 10, 3)
    assert np.array_equal(c, x[idx])


def test_instance_sizes_ranges():
    s = synth.instance_sizes(512)
    ns = np.array([a for a, _, _ in s]); ds = np.array([b for _, b, _ in s]); ks = np.array([c for _, _, c in s])
    assert ns.min() >= 2000 and ns.max() <= 200_000
    assert set(ds.tolist()) <= {3, 16, 64}
    assert ks.min() >= 8 and ks.max() <= 512 and (ks <= ns).all()
