"""GPU parity of one application of G (assignment + update, energy) against
the FP64 oracle, through the C ABI."""

import math

import numpy as np
import pytest

from oracle import kmeans_oracle as ko
from paper_1805_10638_amd import synth

from helpers import check_g, dev, x_tensor, x_values  # noqa: F401

pytestmark = pytest.mark.gpu


def _lib():
    import paper_1805_10638_amd as km
    return km


def _mixture(n, d, k, seed):
    x, _ = synth.plain_large(rep=seed, n=n, d=d, k=max(1, k // 2 + 1), cfg=50)
    return x


# sizes span several tiles, ragged tails and every register-tile width
SHAPES = [
    (1000, 2, 10), (4099, 32, 256), (3001, 3, 17), (777, 16, 5), (2049, 64, 100),
    (1500, 96, 40), (600, 128, 33), (300, 200, 7), (257, 1, 3), (5000, 5, 64),
    (333, 250, 20), (2500, 48, 129), (900, 33, 31),
]


@pytest.mark.parametrize("N,d,K", SHAPES)
def test_g_parity_f32(N, d, K):
    km = _lib()
    X = _mixture(N, d, K, seed=N + d)
    C = synth.init_centroids(X, K, seed=K) + np.float32(0.25)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    r = check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)
    assert st.recheck_rows >= 0
    assert r["max_c_err"] <= 1e-5


@pytest.mark.parametrize("N,d,K", [(2000, 32, 64), (3000, 128, 100), (1111, 16, 9)])
def test_g_parity_bf16_storage(N, d, K):
    km = _lib()
    Xb, _ = synth.precision(rep=1, n=N, d=d, k=max(2, K // 2))
    C = synth.init_centroids(Xb, K, seed=3)
    rho, Cn, E, st = km.kmeans_g(x_tensor(Xb), dev(C))
    check_g(Xb, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)


def test_g_changed_count_and_empty_clusters():
    km = _lib()
    X = _mixture(3000, 8, 10, seed=1)
    C = synth.init_centroids(X, 10, seed=2)
    C[9] = 1e4          # far away: an empty cluster keeps its centroid
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    assert st.empty_clusters >= 1
    assert np.array_equal(Cn.cpu().numpy()[9], C[9])
    prev = rho.clone()
    prev[::7] = (prev[::7] + 1) % 10
    _, _, _, st2 = km.kmeans_g(x_tensor(X), dev(C), rho_prev=prev)
    assert st2.changed == int((prev != rho).sum().item())


def test_g_exact_ties_lowest_index():
    km = _lib()
    # samples on dyadic bisectors: exact ties resolved to the lowest index
    X = np.array([[0.5, 0.0], [0.5, 1.0], [1.5, 0.0], [2.25, 0.0], [0.0, 0.0]] * 40, np.float32)
    C = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0], [1.0, 0.0]], np.float32)  # duplicate centroid
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    a = ko.assign(X.astype(np.float64), C.astype(np.float64))
    assert np.array_equal(rho.cpu().numpy(), a.rho)
    assert st.recheck_rows > 0
    assert st.near_tie_rows == int(a.near_tie.sum()) == 120


def test_g_cancellation_heavy_offsets():
    """Large common offset: ||x||^2 >> distances, so the GEMM form cancels
    badly and most decisions go through the exact re-check."""
    km = _lib()
    rng = np.random.default_rng(0)
    X = (1000.0 + rng.normal(size=(4000, 8))).astype(np.float32)
    C = X[rng.choice(4000, 50, replace=False)].copy()
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    r = check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)
    assert st.recheck_rows > 0
    assert r["mismatch"] <= r["near_ties"]
    assert st.near_tie_rows == r["near_ties"]


@pytest.mark.parametrize("N,d,K,prec,xbf", [(3000, 16, 20, "f32", False), (2500, 5, 12, "f32", False),
                                            (4000, 64, 300, "f32", False), (3000, 128, 40, "bf16", True),
                                            (2000, 32, 600, "bf16", False), (5000, 2, 9, "f32", False)])
def test_g_near_tie_count_matches_oracle(N, d, K, prec, xbf):
    """Duplicated centroids make every sample nearest to them an exact tie;
    the GPU's near-tie count equals the oracle's (every near tie is among
    the re-checked rows, whatever the GEMM precision or width)."""
    km = _lib()
    if xbf:
        X, _ = synth.precision(rep=3, n=N, d=d, k=max(2, K // 2))
    else:
        X = _mixture(N, d, K, seed=N + K)
    C = synth.init_centroids(X, K, seed=4)
    C[K - 1] = C[0]
    C[K - 2] = C[1]
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C), prec=prec)
    r = check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)
    assert r["near_ties"] > 0
    assert st.near_tie_rows == r["near_ties"]
    assert st.recheck_rows >= st.near_tie_rows


def test_g_k1_and_k_equals_n():
    km = _lib()
    X = _mixture(700, 4, 4, seed=5)
    rho, Cn, E, _ = km.kmeans_g(x_tensor(X), dev(X[:1].copy()))
    assert (rho.cpu().numpy() == 0).all()
    np.testing.assert_allclose(Cn.cpu().numpy()[0], X.astype(np.float64).mean(axis=0), rtol=1e-6, atol=1e-6)
    Xs = X[:300].copy()
    rho, Cn, E, _ = km.kmeans_g(x_tensor(Xs), dev(Xs))
    a = ko.assign(Xs.astype(np.float64), Xs.astype(np.float64))
    assert np.array_equal(rho.cpu().numpy(), a.rho)
    assert E == 0.0


def test_g_full_size():
    """N=1,000,000, d=32, K=256 in the benchmark's launch configuration:
    every label against the oracle's assignment, the energy against the
    oracle's, all centroids against the oracle means of the GPU labels."""
    km = _lib()
    X, _ = synth.plain_large(rep=0)
    C = synth.init_centroids(X, 256, seed=0)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)


def test_g_deterministic():
    km = _lib()
    X = _mixture(20000, 32, 64, seed=9)
    C = synth.init_centroids(X, 64, seed=1)
    Xt, Ct = x_tensor(X), dev(C)
    r1 = km.kmeans_g(Xt, Ct)
    r2 = km.kmeans_g(Xt, Ct)
    assert np.array_equal(r1[0].cpu().numpy(), r2[0].cpu().numpy())
    assert np.array_equal(r1[1].cpu().numpy().view(np.uint32), r2[1].cpu().numpy().view(np.uint32))
    assert r1[2] == r2[2]


def test_invalid_arguments():
    import torch
    km = _lib()
    X = x_tensor(_mixture(100, 4, 4, seed=0))
    C = dev(np.zeros((5, 4), np.float32))
    with pytest.raises(km.KMError) as e:
        km.kmeans_g(X, dev(np.zeros((200, 4), np.float32)))   # K > N
    assert e.value.status == -1
    with pytest.raises(km.KMError) as e:
        km.kmeans_g(dev(np.zeros((100, 300), np.float32)), dev(np.zeros((5, 300), np.float32)))
    assert e.value.status == -4
    with pytest.raises(km.KMError) as e:
        km.kmeans_solve(X, C, m_max=65)
    assert e.value.status == -1
    with pytest.raises(km.KMError) as e:
        km.kmeans_solve(X, C, tol=-1.0)
    assert e.value.status == -1
    Xo = torch.zeros(401, dtype=torch.float32, device="cuda")[1:].view(100, 4)  # 4-byte offset
    with pytest.raises(km.KMError) as e:
        km.kmeans_g(Xo, C)
    assert e.value.status == -1
    Xn = _mixture(100, 4, 4, seed=0)
    Xn[3, 1] = np.nan
    with pytest.raises(km.KMError) as e:
        km.kmeans_g(x_tensor(Xn), C)
    assert e.value.status == -5


# ---------------------------------------------------------------------------
# bfloat16 distance GEMM (precision mode): same exactness contract
# ---------------------------------------------------------------------------

BF_SHAPES = [(3000, 128, 100), (2049, 32, 64), (1500, 96, 40), (777, 16, 5), (2500, 64, 129),
             (600, 200, 33), (1000, 3, 10), (4099, 48, 256)]


@pytest.mark.parametrize("N,d,K", BF_SHAPES)
def test_g_parity_bf16_gemm_bf16_x(N, d, K):
    km = _lib()
    Xb, _ = synth.precision(rep=2, n=N, d=d, k=max(2, K // 2))
    C = synth.init_centroids(Xb, K, seed=5) + np.float32(0.125)
    rho, Cn, E, st = km.kmeans_g(x_tensor(Xb), dev(C), prec="bf16")
    check_g(Xb, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)


@pytest.mark.parametrize("N,d,K", [(3000, 128, 100), (1500, 96, 40), (900, 33, 31)])
def test_g_parity_bf16_gemm_f32_x(N, d, K):
    km = _lib()
    X = _mixture(N, d, K, seed=N + 7)
    C = synth.init_centroids(X, K, seed=K + 1)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C), prec="bf16")
    check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)


def test_bf16_and_f32_gemm_agree():
    """Both precisions return the exact argmin: identical labels except rows
    that the oracle itself calls near ties."""
    km = _lib()
    Xb, _ = synth.precision(rep=3, n=20000, d=128, k=256)
    C = synth.init_centroids(Xb, 256, seed=9)
    Xt, Ct = x_tensor(Xb), dev(C)
    r32 = km.kmeans_g(Xt, Ct, prec="f32")
    r16 = km.kmeans_g(Xt, Ct, prec="bf16")
    a = r32[0].cpu().numpy(), r16[0].cpu().numpy()
    diff = np.flatnonzero(a[0] != a[1])
    if diff.size:
        o = ko.assign(x_values(Xb[diff]), C.astype(np.float64))
        assert o.near_tie.all()
    assert abs(r32[2] - r16[2]) <= 1e-9 * abs(r32[2])


def test_solve_bf16_gemm_matches_f32():
    km = _lib()
    Xb, _ = synth.precision(rep=4, n=30000, d=64, k=64)
    C0 = synth.init_centroids(Xb, 64, seed=4)
    Xt, Ct = x_tensor(Xb), dev(C0)
    a = km.kmeans_solve(Xt, Ct, m_max=10, tol=1e-6, prec="f32")
    b = km.kmeans_solve(Xt, Ct, m_max=10, tol=1e-6, prec="bf16")
    assert a[3] == b[3]
    assert b[2] == pytest.approx(a[2], rel=1e-9)
    assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_g_many_flags_streamed_centroids(prec):
    """Large common offset with K too large for LDS residency: most rows are
    flagged, so every workgroup re-checks many batches of listed rows against
    several staged centroid chunks; every label must still be the exact
    argmin."""
    km = _lib()
    rng = np.random.default_rng(11)
    # bf16 keeps the offset small enough that the noise is not rounded away
    X = ((300.0 if prec == "f32" else 40.0) + rng.normal(size=(3000, 64))).astype(np.float32)
    if prec == "bf16":
        X = synth.to_bf16_bits(X)
    C = synth.init_centroids(X, 300, seed=3)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C), prec=prec)
    r = check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)
    assert st.recheck_rows > 1000
    assert r["mismatch"] <= r["near_ties"]


def test_g_phase_timing():
    """With timing on, kmeans_g reports positive device times for the
    assignment and the update; with timing off both are -1; results are the
    same either way."""
    km = _lib()
    X = _mixture(50000, 16, 64, seed=21)
    C = synth.init_centroids(X, 64, seed=2)
    Xt, Ct = x_tensor(X), dev(C)
    ctx = km.Context(0)
    r0 = km.kmeans_g(Xt, Ct, ctx=ctx)
    assert r0[3].assign_ms == -1.0 and r0[3].update_ms == -1.0
    ctx.set_timing(True)
    r1 = km.kmeans_g(Xt, Ct, ctx=ctx)
    ctx.set_timing(False)
    assert r1[3].assign_ms > 0.0 and r1[3].update_ms > 0.0
    assert np.array_equal(r0[0].cpu().numpy(), r1[0].cpu().numpy())
    assert np.array_equal(r0[1].cpu().numpy().view(np.uint32), r1[1].cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_g_max_sizes(prec):
    """Largest supported width and cluster count (d = 256, K = 4096): the
    widest register tile and centroids streamed through LDS in many chunks,
    with the deferred re-check over several chunk rounds.  Labels of sampled
    rows, the energy and all centroids against the oracle."""
    km = _lib()
    X = _mixture(8192, 256, 4096, seed=31)
    if prec == "bf16":
        X = synth.to_bf16_bits(X)
    C = synth.init_centroids(X, 4096, seed=4)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C), prec=prec)
    rows = np.random.default_rng(2).choice(X.shape[0], 400, replace=False)
    check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E, rows=rows)


def test_g_served_large_shape_bf16():
    """The served large-job shape (d = 96, K = 2048, bfloat16 rows and GEMM)
    at N = 30,000: sampled labels, energy and centroids against the oracle."""
    km = _lib()
    X = synth.to_bf16_bits(_mixture(30000, 96, 2048, seed=33))
    C = synth.init_centroids(X, 2048, seed=5)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C), prec="bf16")
    rows = np.random.default_rng(3).choice(X.shape[0], 1000, replace=False)
    check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E, rows=rows)


def test_g_full_size_precision_sampled():
    """N = 4,000,000, d = 128, K = 1024, bfloat16 rows and GEMM (the precision
    benchmark's data and launch configuration): labels of 3000 sampled rows
    against the oracle (outside its near ties), the energy against the
    oracle's energy of the GPU labels (summed over row chunks), and all 1024
    centroids against the oracle's means of the GPU labels."""
    km = _lib()
    N, d, K = 4_000_000, 128, 1024
    Xb, _ = synth.precision(rep=0, n=N, d=d, k=K)
    C = synth.init_centroids(Xb, K, 1)
    C64 = C.astype(np.float64)
    rho, Cn, E, st = km.kmeans_g(x_tensor(Xb), dev(C), prec="bf16")
    rho = rho.cpu().numpy().astype(np.int64)
    Cn = Cn.cpu().numpy()
    rng = np.random.default_rng(4)
    rows = rng.choice(N, 3000, replace=False)
    a = ko.assign(x_values(Xb[rows]), C64)
    bad = np.flatnonzero((a.rho != rho[rows]) & ~a.near_tie)
    assert bad.size == 0, f"{bad.size} sampled label mismatches outside near ties"
    step = 500_000
    Eo = math.fsum(ko.energy(x_values(Xb[s:s + step]), rho[s:s + step], C64) for s in range(0, N, step))
    assert abs(E - Eo) <= 1e-6 * Eo, (E, Eo)
    X64 = x_values(Xb)
    Co, counts = ko.update(X64, rho, C64)
    del X64
    err = np.linalg.norm(Cn.astype(np.float64) - Co, axis=1) / np.maximum(np.linalg.norm(Co, axis=1), 1.0)
    assert err.max() <= 1e-5, (int(err.argmax()), float(err.max()))
    assert np.array_equal(Cn[counts == 0], C[counts == 0])


def _mean_bound_check(X, C, rho, Cn):
    """Means against the oracle's means of the GPU labels, to float32 rounding
    plus the fixed-point bound N * max|x| * 2^-61 (with a factor 2 margin)."""
    X64 = x_values(X)
    Co, _ = ko.update(X64, np.asarray(rho).astype(np.int64), C.astype(np.float64))
    tol = np.abs(Co) * 2.0**-23 + X64.shape[0] * np.abs(X64).max() * 2.0**-60
    err = np.abs(np.asarray(Cn).astype(np.float64) - Co)
    assert (err <= tol).all(), float((err / tol).max())


# The fixed-point sums take K * (d | 1) + K <= 10240 (80 KB of LDS
# accumulators); larger shapes take the counting sort.  Both sides of the
# limit, float32 and bfloat16 rows, d with and without 4-coordinate groups.
@pytest.mark.parametrize("d,K,xt", [(16, 568, "f32"), (16, 569, "f32"), (7, 1280, "bf16"),
                                    (7, 1281, "bf16"), (12, 100, "bf16"), (5, 64, "f32")])
def test_update_sums_both_paths(d, K, xt):
    km = _lib()
    X = _mixture(20000, d, K, seed=d * K)
    if xt == "bf16":
        X = synth.to_bf16_bits(X)
    C = synth.init_centroids(X, K, seed=1)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)
    _mean_bound_check(X, C, rho.cpu().numpy(), Cn.cpu().numpy())


def test_update_fixed_point_wide_range():
    """Coordinates spanning eight decades (max |x| near 4e5, the smallest
    dimension near 1e-3): every mean within the fixed-point bound."""
    km = _lib()
    rng = np.random.default_rng(5)
    N, d, K = 30000, 8, 40
    X = (rng.normal(size=(N, d)) * np.logspace(-3, 5, d)).astype(np.float32)
    C = X[rng.choice(N, K, replace=False)].copy()
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    _mean_bound_check(X, C, rho.cpu().numpy(), Cn.cpu().numpy())
    a = ko.assign(X.astype(np.float64), C.astype(np.float64))
    mism = np.flatnonzero(a.rho != rho.cpu().numpy())
    assert (a.near_tie[mism]).all()


@pytest.mark.parametrize("xt", ["f32", "bf16"])
@pytest.mark.parametrize("pos", [0, 1, 2, 3, 4, 5, 6, 7, 40001, -1])
def test_update_bound_sees_every_position(xt, pos):
    """One coordinate 3e4 times larger than the rest, at each position inside
    a 16-byte word and in the ragged tail: the |x| bound must include it, or
    the fixed-point sums of its cluster overflow."""
    km = _lib()
    rng = np.random.default_rng(7)
    N, d, K = 9001, 9, 12                 # N*d not a multiple of 8: a ragged tail
    X = rng.normal(size=(N, d)).astype(np.float32)
    X.reshape(-1)[pos] = 3e4
    if xt == "bf16":
        X = synth.to_bf16_bits(X)
    C = x_values(X)[rng.choice(N, K, replace=False)].astype(np.float32)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C))
    _mean_bound_check(X, C, rho.cpu().numpy(), Cn.cpu().numpy())
