"""Streamed bfloat16 centroids: K exceeds what one LDS chunk holds, so the
centroid pair streams through LDS chunk by chunk and the undecided rows go
to the pass-wide re-check.  Checked against the FP64 oracle and against the
float32 GEMM (an independent kernel) on every row, for each tile shape, with
ragged final chunks (K not a multiple of the chunk), padding rows (K not a
multiple of 16) and several row groups per workgroup."""

import numpy as np
import pytest

from oracle import kmeans_oracle as ko
from paper_1805_10638_amd import synth

from helpers import check_g, dev, x_tensor, x_values

pytestmark = pytest.mark.gpu

# more rows than one round of row groups of every shape (256 CUs x up to 2
# workgroups x 256-512 rows), so most workgroups take two or three groups
N_BIG = 300_000


def _lib():
    import paper_1805_10638_amd as km
    return km


_f32_ref = {}


def _big(K):
    """bf16 data of the precision benchmark's kind at d = 128, its centroids,
    and the float32-GEMM labels and energy (computed once per K)."""
    if K not in _f32_ref:
        km = _lib()
        Xb, _ = synth.precision(rep=K, n=N_BIG, d=128, k=K // 2)
        C = synth.init_centroids(Xb, K, seed=K + 1)
        rho, _, E, _ = km.kmeans_g(x_tensor(Xb), dev(C), prec="f32")
        _f32_ref[K] = (Xb, C, rho.cpu().numpy(), E)
    return _f32_ref[K]


@pytest.mark.parametrize("K", [300, 1000])
@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_stream_bf16_every_row_against_f32_gemm(K, shape):
    """Every row's label equals the float32 GEMM's label unless the oracle
    calls the row a near tie; the energies agree to 1e-9; 3000 sampled rows,
    the energy and the means against the oracle."""
    km = _lib()
    Xb, C, r32, E32 = _big(K)
    ctx = km.Context(0, tuned=False)
    ctx.set_tile_shape("bf16", "bf16", 128, K, shape)
    assert ctx.tile_shape("bf16", "bf16", 128, K) == shape
    rho, Cn, E, st = km.kmeans_g(x_tensor(Xb), dev(C), prec="bf16", ctx=ctx)
    r16 = rho.cpu().numpy()
    diff = np.flatnonzero(r16 != r32)
    if diff.size:
        o = ko.assign(x_values(Xb[diff]), C.astype(np.float64))
        assert o.near_tie.all(), f"{int((~o.near_tie).sum())} rows differ outside near ties"
    assert abs(E - E32) <= 1e-9 * abs(E32)
    rows = np.random.default_rng(shape).choice(N_BIG, 3000, replace=False)
    check_g(Xb, C, r16, Cn.cpu().numpy(), E, rows=rows)


@pytest.mark.parametrize("N,d,K", [(40000, 32, 1500), (40000, 96, 700), (40000, 256, 100), (30001, 128, 1009)])
def test_stream_bf16_widths(N, d, K):
    """Other lane-group widths (8, 24, 64 dims per lane group) and a prime K:
    all labels against the oracle."""
    km = _lib()
    Xb, _ = synth.precision(rep=d, n=N, d=d, k=max(2, K // 3))
    C = synth.init_centroids(Xb, K, seed=d + K)
    rho, Cn, E, st = km.kmeans_g(x_tensor(Xb), dev(C), prec="bf16")
    check_g(Xb, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)


def test_stream_bf16_gemm_float32_rows():
    """float32 rows on the bf16 GEMM (rows split into hi and lo parts) with
    streamed centroids: all labels against the oracle."""
    km = _lib()
    X, _ = synth.plain_large(rep=3, n=40000, d=128, k=200, cfg=50)
    C = synth.init_centroids(X, 400, seed=11)
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C), prec="bf16")
    check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)


def test_stream_bf16_solve_matches_f32():
    """The solver's candidate and fall-back passes with streamed bf16
    centroids: the same iterations, labels and energy as the float32 GEMM."""
    km = _lib()
    Xb, _ = synth.precision(rep=7, n=60000, d=128, k=150)
    C0 = synth.init_centroids(Xb, 300, seed=8)
    Xt, Ct = x_tensor(Xb), dev(C0)
    a = km.kmeans_solve(Xt, Ct, m_max=10, tol=1e-6, prec="f32")
    b = km.kmeans_solve(Xt, Ct, m_max=10, tol=1e-6, prec="bf16")
    assert a[3] == b[3]
    assert b[2] == pytest.approx(a[2], rel=1e-9)
    assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())


@pytest.mark.parametrize("prec,K,scale,offset", [("bf16", 300, 1.0, 1000.0), ("f32", 1500, 1.0, 1000.0),
                                                 ("bf16", 300, 1e-20, 0.0)])
def test_recheck_filter_extremes(prec, K, scale, offset):
    """The pass-wide re-check scores every centroid in float32 and computes
    float64 distances only for those within its rigorous bound of the best;
    every row must still get the float64 argmin and the float64 near-tie
    count.  A large common offset makes the scores cancel (wide bound, many
    candidates); values of 1e-20 make float32 products underflow (every
    centroid stays a candidate).  A duplicated centroid adds exact ties.
    f32 at K = 1500 streams the centroids, so its rows are listed too."""
    km = _lib()
    rng = np.random.default_rng(K)
    N, d = 6000, 64
    X = (offset + scale * rng.normal(size=(N, d))).astype(np.float32)
    C = X[rng.choice(N, K, replace=False)].copy()
    C[K - 1] = C[0]
    rho, Cn, E, st = km.kmeans_g(x_tensor(X), dev(C), prec=prec)
    r = check_g(X, C, rho.cpu().numpy(), Cn.cpu().numpy(), E)
    assert st.recheck_rows > 0
    assert r["mismatch"] <= r["near_ties"]
    assert st.near_tie_rows == r["near_ties"]
