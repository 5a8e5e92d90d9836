"""Batched and served solving: each job's result equals kmeans_solve on that
job alone (labels, iteration count and decisions exactly; centroids and
energy within the float rounding of differently split energy partials),
and agrees with the FP64 oracle."""

import numpy as np
import pytest

from oracle import kmeans_oracle as ko
from paper_1805_10638_amd import synth

from helpers import centroid_errors, dev, x_tensor, x_values

pytestmark = pytest.mark.gpu


def _lib():
    import paper_1805_10638_amd as km
    return km


def _problems(sizes, seed0=0, bf16=False):
    out = []
    for i, (n, d, k) in enumerate(sizes):
        x, _ = synth.instance(n, d, k, seed=seed0 + i)
        if bf16:
            x = synth.to_bf16_bits(x)
        c0 = synth.init_centroids(x, k, seed0 + i)
        out.append((x, c0))
    return out


def _solo(km, X, C0, **kw):
    C, rho, E, it, st = km.kmeans_solve(X, C0, **kw)
    return C.cpu().numpy(), rho.cpu().numpy(), E, it, st


def _same(solo, batched):
    C1, r1, E1, it1, st1 = solo
    C2, r2, res = batched
    C2 = C2.cpu().numpy()
    r2 = r2.cpu().numpy()
    assert res.iters == it1
    assert (res.accepted, res.rejected, res.assign_passes) == (st1.accepted, st1.rejected, st1.assign_passes)
    assert np.array_equal(r1, r2)
    assert res.E == pytest.approx(E1, rel=1e-12)
    scale = np.maximum(np.abs(C1), 1.0)
    assert np.max(np.abs(C1 - C2) / scale) <= 1e-6


MIXED = [(2000, 3, 8), (5000, 16, 40), (3000, 64, 100), (12000, 3, 200), (2500, 16, 8),
         (8000, 64, 24), (4000, 3, 60), (6000, 16, 130), (2100, 64, 300)]


def test_batch_matches_solo():
    km = _lib()
    probs = _problems(MIXED, seed0=10)
    ts = [(x_tensor(x), dev(c)) for x, c in probs]
    kw = dict(m_max=10, tol=1e-6)
    solo = [_solo(km, X, C0, **kw) for X, C0 in ts]
    out = km.kmeans_solve_batch(ts, **kw)
    assert len(out) == len(ts)
    for s, b in zip(solo, out):
        assert b[2].status in (0, 1)
        _same(s, b)


def test_batch_against_oracle():
    km = _lib()
    probs = _problems([(1500, 3, 8), (1200, 16, 20)], seed0=40)
    out = km.kmeans_solve_batch([(x_tensor(x), dev(c)) for x, c in probs], m_max=10, tol=1e-6)
    for (x, c0), (C, rho, res) in zip(probs, out):
        o = ko.solve(x_values(x), c0.astype(np.float64), m_max=10, tol=1e-6)
        assert res.iters == o.iters
        assert res.E == pytest.approx(o.E, rel=1e-6)
        a = ko.assign(x_values(x), C.cpu().numpy().astype(np.float64))
        r = rho.cpu().numpy()
        assert np.all((a.rho == r) | a.near_tie)


def test_batch_bf16_gemm_matches_solo():
    km = _lib()
    probs = _problems([(3000, 16, 30), (2000, 64, 70), (4000, 3, 12)], seed0=60, bf16=True)
    ts = [(x_tensor(x), dev(c)) for x, c in probs]
    kw = dict(m_max=10, tol=1e-6, prec="bf16")
    solo = [_solo(km, X, C0, **kw) for X, C0 in ts]
    out = km.kmeans_solve_batch(ts, **kw)
    for s, b in zip(solo, out):
        _same(s, b)


def test_batch_many_instances_compaction():
    """64 instances: finished jobs are compacted out several times while the
    rest continue; every result equals its solo solve."""
    km = _lib()
    sizes = synth.instance_sizes(64, rep=3)
    sizes = [(min(n, 20000), d, min(k, 128)) for n, d, k in sizes]
    probs = _problems(sizes, seed0=100)
    ts = [(x_tensor(x), dev(c)) for x, c in probs]
    out = km.kmeans_solve_batch(ts, m_max=10, tol=1e-6)
    for i in range(0, 64, 7):
        _same(_solo(km, *ts[i], m_max=10, tol=1e-6), out[i])


def test_engine_staggered_admission():
    """Jobs submitted while others run (continuous batching) give the same
    results as alone."""
    km = _lib()
    probs = _problems(MIXED[:7], seed0=200)
    ts = [(x_tensor(x), dev(c)) for x, c in probs]
    eng = km.Engine(m_max=10, tol=1e-6, graphs=False)
    tickets = {}
    got = {}
    for i in range(3):
        tickets[eng.submit(*ts[i])] = i
    for _ in range(4):
        eng.step()
        for t, C, rho, res in eng.poll():
            got[tickets[t]] = (C, rho, res)
    for i in range(3, 7):
        tickets[eng.submit(*ts[i])] = i
        eng.step()
        for t, C, rho, res in eng.poll():
            got[tickets[t]] = (C, rho, res)
    for _ in range(2000):
        if len(got) == len(ts):
            break
        eng.step()
        for t, C, rho, res in eng.poll():
            got[tickets[t]] = (C, rho, res)
    eng.close()
    assert len(got) == len(ts)
    for i, (X, C0) in enumerate(ts):
        _same(_solo(km, X, C0, m_max=10, tol=1e-6), got[i])
        assert got[i][2].latency_ms > 0


def _oracle_same(X, C0, C, rho, res, prec):
    """End-to-end parity of one engine result with the FP64 oracle from the
    same C^0: iterations and decisions equal, energy to 1e-6, centroids to
    1e-5, labels equal except oracle near ties."""
    X64 = x_values(X)
    o = ko.solve(X64, C0.astype(np.float64), m_max=10, tol=1e-6)
    assert (res.iters, res.accepted, res.rejected) == (o.iters, o.accepted, o.rejected), prec
    assert res.E == pytest.approx(o.E, rel=1e-6)
    assert centroid_errors(C.cpu().numpy(), o.C, X64).max() <= 1e-5
    a = ko.assign(X64, C.cpu().numpy().astype(np.float64))
    assert np.all((a.rho == rho.cpu().numpy()) | a.near_tie)


def test_engine_served_against_oracle():
    """Continuous batching compared with the oracle itself (not only with the
    solo GPU solve): jobs admitted while others run, on both update paths
    (K*(d|1) + K above and below 10240) and both GEMM precisions."""
    km = _lib()
    spec = [(3000, 16, 30, False), (4000, 64, 200, False), (2500, 64, 170, True), (5000, 3, 12, False)]
    probs = []
    for i, (n, d, k, bf) in enumerate(spec):
        x, _ = synth.instance(n, d, k, seed=700 + i)
        if bf:
            x = synth.to_bf16_bits(x)
        probs.append((x, synth.init_centroids(x, k, 700 + i), "bf16" if bf else "f32"))
    eng = km.Engine(m_max=10, tol=1e-6, graphs=True)
    tickets, got = {}, {}

    def drain(steps):
        for _ in range(steps):
            if len(got) == len(probs):
                return
            eng.step()
            for t, C, rho, res in eng.poll():
                got[tickets[t]] = (C, rho, res)

    for i in (0, 1):
        x, c0, prec = probs[i]
        tickets[eng.submit(x_tensor(x), dev(c0), prec=prec)] = i
    drain(3)
    for i in (2, 3):
        x, c0, prec = probs[i]
        tickets[eng.submit(x_tensor(x), dev(c0), prec=prec)] = i
        drain(2)
    drain(5000)
    eng.close()
    assert len(got) == len(probs)
    for i, (x, c0, prec) in enumerate(probs):
        _oracle_same(x, c0, *got[i], prec)


def test_engine_budget_admission():
    """With a budget of about two jobs' device memory, jobs wait for room;
    the device never holds more than the budget."""
    km = _lib()
    probs = _problems([(6000, 16, 40)] * 5, seed0=300)
    ts = [(x_tensor(x), dev(c)) for x, c in probs]
    probe = km.Engine(m_max=10, tol=1e-6)
    # the budget counts each job's workspace plus its X, C0, C_out and labels
    ws = probe.workspace_bytes(ts[0][0], 40) + 6000 * 16 * 4 + 2 * 40 * 16 * 4 + 6000 * 4
    probe.close()
    budget = int(2.5 * ws)
    eng = km.Engine(m_max=10, tol=1e-6, hbm_budget=budget, graphs=True)
    tickets = {eng.submit(X, C0): i for i, (X, C0) in enumerate(ts)}
    got = {}
    max_active = 0
    saw_queue = False
    for _ in range(5000):
        a, q, r = eng.step()
        max_active = max(max_active, a)
        saw_queue |= q > 0
        for t, C, rho, res in eng.poll():
            got[tickets[t]] = (C, rho, res)
        if len(got) == len(ts):
            break
    eng.close()
    assert len(got) == len(ts)
    assert saw_queue and max_active * ws <= budget
    for i, (X, C0) in enumerate(ts):
        _same(_solo(km, X, C0, m_max=10, tol=1e-6), got[i])


def test_engine_rejects_bad_jobs():
    km = _lib()
    x, _ = synth.instance(500, 3, 8, seed=1)
    X = x_tensor(x)
    eng = km.Engine(m_max=10, tol=1e-6, hbm_budget=1024)
    with pytest.raises(km.KMError) as e:
        eng.submit(X, dev(synth.init_centroids(x, 8, 1)))
    assert e.value.status == -2          # workspace beyond the budget
    eng.close()
    eng = km.Engine(m_max=10, tol=1e-6)
    with pytest.raises(km.KMError) as e:
        eng.submit(X, dev(np.zeros((600, 3), np.float32)))   # K > N
    assert e.value.status == -1
    eng.close()


def test_batch_mixed_precisions():
    """float32 and bfloat16 GEMM jobs in one batch, each equal to its solo solve."""
    km = _lib()
    p32 = _problems([(3000, 16, 30), (2500, 64, 50)], seed0=400)
    p16 = _problems([(3500, 16, 25), (2000, 64, 64)], seed0=410, bf16=True)
    items = [(x_tensor(x), dev(c), "f32") for x, c in p32] + [(x_tensor(x), dev(c), "bf16") for x, c in p16]
    out = km.kmeans_solve_batch(items, m_max=10, tol=1e-6)
    for (X, C0, prec), b in zip(items, out):
        _same(_solo(km, X, C0, m_max=10, tol=1e-6, prec=prec), b)


def test_two_engines_concurrently():
    """Two engines on their own streams (one restricted to part of the
    device) stepped without blocking: every result equals its solo solve."""
    km = _lib()
    ps = _problems([(4000, 16, 20), (3000, 3, 40), (5000, 64, 30)], seed0=500)
    pl = _problems([(20000, 64, 256)], seed0=510, bf16=True)
    small = [(x_tensor(x), dev(c)) for x, c in ps]
    large = [(x_tensor(x), dev(c)) for x, c in pl]
    es = km.Engine(m_max=10, tol=1e-6)
    el = km.Engine(m_max=10, tol=1e-6, prec="bf16")
    el.set_share(0.5)
    ts = {es.submit(X, C0): i for i, (X, C0) in enumerate(small)}
    tl = {el.submit(X, C0): i for i, (X, C0) in enumerate(large)}
    gs, gl = {}, {}
    for _ in range(20000):
        es.step(wait=False)
        el.step(wait=False)
        for t, C, rho, res in es.poll():
            gs[ts[t]] = (C, rho, res)
        for t, C, rho, res in el.poll():
            gl[tl[t]] = (C, rho, res)
        if len(gs) == len(small) and len(gl) == len(large):
            break
    es.close()
    el.close()
    assert len(gs) == len(small) and len(gl) == len(large)
    for i, (X, C0) in enumerate(small):
        _same(_solo(km, X, C0, m_max=10, tol=1e-6), gs[i])
    for i, (X, C0) in enumerate(large):
        _same(_solo(km, X, C0, m_max=10, tol=1e-6, prec="bf16"), gl[i])
