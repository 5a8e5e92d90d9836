"""kmeans_g_noalloc: one application of G whose scratch is the library's
fixed device array (no device allocation in the call), checked against
kmeans_g and the FP64 oracle through the C ABI.

Two calls in a row share the array, the second on a smaller input, so that a
buffer left over from the first call cannot go unnoticed.  Both update paths
(fixed-point sums and the counting sort) and both GEMM precisions are
covered; a shape whose scratch would not fit is refused before any launch."""

import numpy as np
import pytest

from paper_1805_10638_amd import synth

from helpers import check_g, dev, x_tensor

pytestmark = pytest.mark.gpu


def _lib():
    import paper_1805_10638_amd as km
    return km


def _mixture(n, d, k, seed):
    x, _ = synth.plain_large(rep=seed, n=n, d=d, k=max(1, k // 2 + 1), cfg=51)
    return x


def _pair(km, X, C, prec, rho_prev=None):
    """kmeans_g_noalloc into caller tensors, then kmeans_g on the same input."""
    import torch
    Xd, Cd = x_tensor(X), dev(C)
    rho = torch.full((X.shape[0],), -1, dtype=torch.int32, device="cuda")
    Cn = torch.full_like(Cd, float("nan"))
    pv = dev(rho_prev.astype(np.int32)) if rho_prev is not None else None
    r1, C1, E1, s1 = km.kmeans_g_noalloc(Xd, Cd, (rho, Cn), prec=prec, rho_prev=pv)
    assert r1.data_ptr() == rho.data_ptr() and C1.data_ptr() == Cn.data_ptr()
    r2, C2, E2, s2 = km.kmeans_g(Xd, Cd, prec=prec, rho_prev=pv)
    assert torch.equal(r1, r2)
    assert torch.equal(C1, C2)
    assert E1 == E2
    assert (s1.changed, s1.recheck_rows, s1.near_tie_rows, s1.empty_clusters) == \
        (s2.changed, s2.recheck_rows, s2.near_tie_rows, s2.empty_clusters)
    return r1.cpu().numpy(), C1.cpu().numpy(), E1, s1


# (first call, second smaller call): fixed-point update (K*(d|1)+K <= 10240)
# and counting sort, float32 and bfloat16 GEMM, ragged N and K
CASES = [
    ((20000, 32, 256, "f32"), (7001, 32, 100, "f32")),
    ((30000, 64, 300, "f32"), (9999, 48, 200, "f32")),
    ((20000, 64, 300, "bf16"), (5003, 64, 170, "bf16")),
    ((12000, 16, 600, "f32"), (3000, 7, 11, "f32")),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_matches_kmeans_g_twice(first, second):
    km = _lib()
    for (N, d, K, prec) in (first, second):
        X = _mixture(N, d, K, seed=N + d + K)
        C = synth.init_centroids(X, K, seed=K) + np.float32(0.125)
        rho, Cn, E, st = _pair(km, X, C, prec)
        r = check_g(X, C, rho, Cn, E)
        assert r["max_c_err"] <= 1e-5
        assert rho.min() >= 0 and rho.max() < K


def test_noalloc_bf16_storage_and_changed_count():
    km = _lib()
    Xb, _ = synth.precision(rep=2, n=9000, d=128, k=40)
    C = synth.init_centroids(Xb, 80, seed=5)
    rho0, _, _, _ = _pair(km, Xb, C, "bf16")
    C2 = C + np.float32(0.5)
    rho, Cn, E, st = _pair(km, Xb, C2, "bf16", rho_prev=rho0)
    check_g(Xb, C2, rho, Cn, E)
    assert st.changed == int((rho != rho0).sum())


def test_noalloc_refuses_shape_beyond_scratch():
    import torch
    km = _lib()
    # 17M rows of one dimension: the flagged-row slots alone exceed 64 MiB
    N, d, K = 17 << 20, 1, 2
    X = torch.zeros((N, d), dtype=torch.float32, device="cuda")
    C = torch.zeros((K, d), dtype=torch.float32, device="cuda")
    rho = torch.empty(N, dtype=torch.int32, device="cuda")
    Cn = torch.empty_like(C)
    with pytest.raises(km.KMError) as e:
        km.kmeans_g_noalloc(X, C, (rho, Cn))
    assert e.value.status == -4
    assert "scratch" in str(e.value)
    # the context still works afterwards
    Xs = _mixture(2000, 4, 6, seed=9)
    Cs = synth.init_centroids(Xs, 6, seed=1)
    _pair(km, Xs, Cs, "f32")
