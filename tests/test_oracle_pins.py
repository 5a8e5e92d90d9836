"""Pins for the FP64 oracle: facts fixed by the paper or by mathematics.

None of these tests re-types the oracle's own formulas; each checks the
oracle against something independent of it (a brute-force optimum, an exact
dynamic program, a closed form, a library solver, an invariant the paper
proves, or a hand-derived worked example).
"""

import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import kmeans_oracle as ko

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _scatter(points):
    """Within-group scatter sum ||x - mean||^2 (plain Python)."""
    if not points:
        return 0.0
    d = len(points[0])
    n = len(points)
    mean = [sum(p[k] for p in points) / n for k in range(d)]
    return sum(sum((p[k] - mean[k]) ** 2 for k in range(d)) for p in points)


def _brute_force_optimum(X, K):
    """Global minimum of Eq. (1) over all partitions into at most K groups."""
    pts = [tuple(map(float, r)) for r in X]
    best, best_lab = math.inf, None
    for lab in itertools.product(range(K), repeat=len(pts)):
        if lab[0] != 0:        # symmetry: first point in group 0
            continue
        e = sum(_scatter([p for p, l in zip(pts, lab) if l == j]) for j in range(K))
        if e < best:
            best, best_lab = e, lab
    return best, best_lab


def _dp_1d(x, K):
    """Exact 1-D K-means optimum by dynamic programming over sorted data."""
    xs = np.sort(np.asarray(x, dtype=np.float64))
    n = xs.size
    s1 = np.concatenate([[0.0], np.cumsum(xs)])
    s2 = np.concatenate([[0.0], np.cumsum(xs * xs)])

    def cost(i, j):  # scatter of xs[i..j] inclusive, vectorised over i
        cnt = j - i + 1
        sm = s1[j + 1] - s1[i]
        return (s2[j + 1] - s2[i]) - sm * sm / cnt

    INF = math.inf
    dp = np.full((K + 1, n), INF)
    arg = np.zeros((K + 1, n), dtype=np.int64)
    for j in range(n):
        dp[1, j] = cost(np.array([0]), j)[0]
    for k in range(2, K + 1):
        for j in range(n):
            i = np.arange(1, j + 1)
            if i.size == 0:
                continue
            cand = dp[k - 1, i - 1] + cost(i, j)
            b = int(np.argmin(cand))
            dp[k, j] = cand[b]
            arg[k, j] = i[b]
    # recover the segments
    bounds = []
    j, k = n - 1, K
    while k >= 1:
        i = arg[k, j] if k > 1 else 0
        bounds.append((i, j))
        j, k = i - 1, k - 1
    bounds.reverse()
    return dp[K, n - 1], xs, bounds


# ---------------------------------------------------------------------------
# P1 brute force on tiny inputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_brute_force_optimum_bounds_solver(seed):
    rng = np.random.default_rng(seed)
    n, K, d = 7, 3, 2
    X = rng.normal(size=(n, d)) * 3.0
    Estar, lab = _brute_force_optimum(X, K)
    for init_seed in range(4):
        idx = np.random.default_rng(100 + init_seed).choice(n, K, replace=False)
        res = ko.solve(X, X[idx], m_max=3, tol=0.0)
        assert res.status == ko.STATUS_CONVERGED
        assert res.E >= Estar * (1 - 1e-12)
        assert res.E == pytest.approx(ko.energy(X, res.rho, res.C), rel=1e-12)
    # start at the optimal partition's means: returns immediately with E*
    groups = [np.flatnonzero(np.array(lab) == j) for j in range(K)]
    if all(g.size for g in groups):
        C0 = np.stack([X[g].mean(axis=0) for g in groups])
        res = ko.solve(X, C0, m_max=3, tol=0.0)
        assert res.iters == 1
        assert res.E == pytest.approx(Estar, rel=1e-12)


# ---------------------------------------------------------------------------
# P2 exact 1-D optimum by dynamic programming
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_dp_1d_optimum(seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(mu, 1.0, 60) for mu in (-8, -2, 3, 9)])
    K = 4
    Estar, xs, bounds = _dp_1d(x, K)
    X = xs[:, None]
    C0 = np.array([[xs[i:j + 1].mean()] for i, j in bounds])
    res = ko.solve(X, C0, m_max=5, tol=0.0)
    assert res.E == pytest.approx(Estar, rel=1e-10)
    for s in range(5):
        idx = np.random.default_rng(s).choice(x.size, K, replace=False)
        r = ko.solve(X, X[idx], m_max=5, tol=0.0)
        assert r.E >= Estar * (1 - 1e-12)


# ---------------------------------------------------------------------------
# P3 Lloyd decreases the energy (majorisation argument of Sec. 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_lloyd_step_monotone(seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(300, 3)) + rng.integers(0, 4, size=(300, 1)) * 4.0
    C = rng.normal(size=(6, 3)) * 4.0
    for _ in range(10):
        a, Cn, E = ko.g(X, C)
        En = ko.energy(X, ko.assign(X, Cn).rho, Cn)
        assert En <= E * (1 + 1e-14)
        C = Cn


# ---------------------------------------------------------------------------
# P4 safeguarded iteration: accepted energies never increase (Sec. 2.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_accepted_energy_monotone(seed):
    from paper_1805_10638_amd import synth
    X, _ = synth.plain_small(rep=seed, n=2000)
    C0 = synth.init_centroids(X, 10, seed)
    res = ko.solve(X, C0, m_max=10, tol=0.0)
    acc = [r["E_acc"] for r in res.trace if "E_acc" in r]
    assert len(acc) >= 2
    assert all(b <= a * (1 + 1e-13) for a, b in zip(acc, acc[1:]))
    # a rejected candidate never has a lower energy than the previous accepted one
    prev = math.inf
    for r in res.trace:
        if r.get("decision") == "rejected" and r["changed_cand"] > 0:
            assert r["E_cand"] >= prev
        if "E_acc" in r:
            prev = r["E_acc"]


# ---------------------------------------------------------------------------
# P5 m = 0 is Lloyd's algorithm
# ---------------------------------------------------------------------------

def _lloyd_loop(X, C0, tol, max_iter):
    """Lloyd's algorithm written directly from Sec. 1 (assignment then update)."""
    P = ko.assign(X, C0).rho
    C, _ = ko.update(X, P, C0)
    Eprev = math.inf
    for t in range(1, max_iter + 1):
        Pn = ko.assign(X, C).rho
        E = ko.energy(X, Pn, C)
        if np.array_equal(Pn, P):
            return C, Pn, E, t
        if tol > 0 and math.isfinite(Eprev) and Eprev - E <= tol * Eprev:
            return C, Pn, E, t
        P, Eprev = Pn, E
        C, _ = ko.update(X, P, C)
    return C, P, Eprev, max_iter


@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_m0_is_lloyd(tol):
    from paper_1805_10638_amd import synth
    X, _ = synth.plain_small(rep=3, n=3000)
    C0 = synth.init_centroids(X, 10, 7)
    res = ko.solve(X, C0, m_max=0, tol=tol)
    C, P, E, t = _lloyd_loop(X, C0, tol, 500)
    assert res.iters == t
    assert np.array_equal(res.C, C)
    assert np.array_equal(res.rho, P)
    assert res.E == E
    assert res.accepted == 0 and res.rejected == 0


# The classical fixed-m variant (Sec. 2.2 compares it with dynamic m): with m
# held at 0 no difference ever enters the least squares, so the run is Lloyd's
# algorithm whatever m_max is; with m held at 2 the dynamic rule's changes of
# m must not happen.

@pytest.mark.parametrize("tol", [0.0, 1e-4])
def test_fixed_m_zero_is_lloyd(tol):
    from paper_1805_10638_amd import synth
    X, _ = synth.plain_small(rep=0, n=3000)
    C0 = synth.init_centroids(X, 10, 1)   # slow Lloyd run: the energy ratio often exceeds eps2
    res = ko.solve(X, C0, m_max=10, m_init=0, fixed_m=True, tol=tol)
    C, P, E, t = _lloyd_loop(X, C0, tol, 500)
    assert res.iters == t
    assert np.array_equal(res.C, C)
    assert np.array_equal(res.rho, P)
    assert res.E == E
    assert res.accepted == 0 and res.rejected == 0 and res.m_final == 0


def test_fixed_m_keeps_m():
    from paper_1805_10638_amd import synth
    X, _ = synth.plain_small(rep=2, n=3000)
    C0 = synth.init_centroids(X, 10, 3)
    dyn = ko.solve(X, C0, m_max=10, m_init=2, tol=0.0)
    assert {r["m"] for r in dyn.trace if "m" in r} != {2}    # the dynamic rule moves m here
    fix = ko.solve(X, C0, m_max=10, m_init=2, fixed_m=True, tol=0.0)
    assert {r["m"] for r in fix.trace if "m" in r} == {2}
    assert all(r["mt"] == min(2, r["t"]) for r in fix.trace if "mt" in r)


# ---------------------------------------------------------------------------
# P6 exact convergence returns a fixed point of G (Eq. 6)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_fixed_point_at_convergence(seed):
    from paper_1805_10638_amd import synth
    X, _ = synth.plain_small(rep=seed, n=2500)
    C0 = synth.init_centroids(X, 10, seed + 11)
    res = ko.solve(X, C0, m_max=10, tol=0.0)
    assert res.status == ko.STATUS_CONVERGED
    a, Cn, E = ko.g(X, res.C)
    assert np.array_equal(Cn, res.C)
    assert np.array_equal(a.rho, res.rho)
    assert E == res.E


# ---------------------------------------------------------------------------
# P7 Anderson on an affine contraction: Eq. (7)/(8) sign and indexing
# ---------------------------------------------------------------------------

def _affine_run(n, steps, sign, seed=0):
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(n, n))
    A = 0.9 * Q / np.max(np.abs(np.linalg.eigvals(Q)))
    b = rng.normal(size=n)
    xstar = np.linalg.solve(np.eye(n) - A, b)
    x0 = rng.normal(size=n)
    hist = ko.History(n + 2)
    G0 = A @ x0 + b
    hist.push(G0, G0 - x0)
    x = G0
    errs = []
    for t in range(1, steps + 1):
        G = A @ x + b
        hist.push(G, G - x)
        mt = min(n, t)
        if sign < 0:
            x, _, _ = hist.accelerate(mt)
        else:                       # planted mistake: Eq. (8) with "+"
            dF, dG = hist.differences(mt)
            theta = ko.ridge_least_squares(dF, hist.F[-1])
            x = hist.G[-1] + dG @ theta
        errs.append(np.linalg.norm(x - xstar) / np.linalg.norm(xstar))
    return errs


@pytest.mark.parametrize("n", [2, 4, 6])
def test_anderson_affine_exact(n):
    errs = _affine_run(n, n + 2, sign=-1)
    assert errs[-1] < 1e-8
    bad = _affine_run(n, n + 2, sign=+1)
    assert bad[-1] > 1e-3


# ---------------------------------------------------------------------------
# P8 least squares against a library solver (reading R8)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 3, 7])
def test_ridge_ls_matches_lstsq(m):
    rng = np.random.default_rng(m)
    n = 50
    dF = rng.normal(size=(n, m)) * rng.uniform(0.1, 10, size=m)
    F = rng.normal(size=n)
    theta = ko.ridge_least_squares(dF, F, lam=1e-10)
    s = np.linalg.norm(dF, axis=0)
    aug = np.vstack([dF / s, np.sqrt(1e-10) * np.eye(m)])
    rhs = np.concatenate([F, np.zeros(m)])
    y, *_ = np.linalg.lstsq(aug, rhs, rcond=None)
    np.testing.assert_allclose(theta, y / s, rtol=1e-10, atol=0)


def test_ridge_ls_zero_columns_and_zero_rhs():
    dF = np.zeros((5, 2))
    dF[:, 1] = np.arange(5.0)
    th = ko.ridge_least_squares(dF, np.ones(5))
    assert th[0] == 0.0
    assert th[1] == pytest.approx(10.0 / 30.0 / (1 + 1e-10), rel=1e-12)
    assert np.all(ko.ridge_least_squares(dF, np.zeros(5)) == 0.0)


# ---------------------------------------------------------------------------
# P9 the dynamic-m rule as a table (Sec. 2.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("E,E1,E2,m,expect", [
    (90.0, 100.0, 120.0, 3, 3),        # ratio 0.5: neither < 0.02 nor > 0.5
    (89.0, 100.0, 120.0, 3, 4),        # ratio 0.55 > eps2: grow
    (99.9, 100.0, 120.0, 3, 2),        # ratio 0.005 < eps1: shrink
    (101.0, 100.0, 120.0, 3, 2),       # energy increased: shrink
    (50.0, 100.0, 120.0, 10, 10),      # capped at m_max
    (100.0, 100.0, 120.0, 0, 0),       # floored at 0
    (99.0, 100.0, math.inf, 3, 3),     # E^{t-2} not finite: unchanged
    (99.0, 100.0, 100.0, 3, 4),        # den = 0, energy decreased: grow
    (101.0, 100.0, 100.0, 3, 2),       # den = 0, energy increased: shrink
    (100.0, 100.0, 100.0, 3, 3),       # den = num = 0: unchanged
])
def test_dynamic_m_table(E, E1, E2, m, expect):
    assert ko.adjust_m(m, E, E1, E2, m_max=10) == expect


# ---------------------------------------------------------------------------
# P10 energy identity (closed form of the within-cluster scatter)
# ---------------------------------------------------------------------------

def test_energy_identity():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(400, 4)) + 3.0
    rho = rng.integers(0, 7, size=400)
    C, cnt = ko.update(X, rho, np.zeros((7, 4)))
    E = ko.energy(X, rho, C)
    closed = 0.0
    for j in range(7):
        S = X[rho == j]
        if len(S):
            closed += (S * S).sum() - (S.sum(axis=0) ** 2).sum() / len(S)
    assert E == pytest.approx(closed, rel=1e-9)


# ---------------------------------------------------------------------------
# P11 well separated mixture: converges at once to the component means
# ---------------------------------------------------------------------------

def test_separated_mixture():
    rng = np.random.default_rng(9)
    K, d = 6, 3
    centers = rng.uniform(-50, 50, size=(K, d))
    z = rng.integers(0, K, size=600)
    X = centers[z] + 0.01 * rng.normal(size=(600, d))
    first = [int(np.flatnonzero(z == j)[0]) for j in range(K)]
    res = ko.solve(X, X[first], m_max=10, tol=0.0)
    assert res.iters <= 2
    want = np.stack([X[z == j].mean(axis=0) for j in range(K)])
    np.testing.assert_allclose(res.C, want, rtol=0, atol=1e-12)
    assert np.array_equal(res.rho, z)


# ---------------------------------------------------------------------------
# P12 special cases
# ---------------------------------------------------------------------------

def test_k1_global_mean():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(500, 3))
    res = ko.solve(X, X[:1], m_max=10, tol=0.0)
    np.testing.assert_allclose(res.C[0], X.mean(axis=0), rtol=0, atol=1e-14)
    assert res.E == pytest.approx(X.var(axis=0).sum() * 500, rel=1e-12)
    assert not ko.assign(X, res.C).near_tie.any()


def test_k_equals_n():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(20, 2))
    res = ko.solve(X, X.copy(), m_max=10, tol=0.0)
    assert res.E == 0.0 and res.iters == 1
    assert np.array_equal(res.rho, np.arange(20))


def test_exact_tie_lowest_index_and_flag():
    X = np.array([[0.5], [0.25], [2.25]])
    C = np.array([[0.0], [1.0], [3.0]])
    a = ko.assign(X, C)
    assert a.rho.tolist() == [0, 0, 2]
    assert a.near_tie.tolist() == [True, False, False]
    # duplicated centroids: d2 == d1 at every row
    a = ko.assign(X, np.array([[1.0], [1.0]]))
    assert a.rho.tolist() == [0, 0, 0] and a.near_tie.all()


def test_empty_cluster_keeps_centroid():
    X = np.array([[0.0], [1.0], [2.0]])
    C = np.array([[1.0], [100.0]])
    a, Cn, E = ko.g(X, C)
    assert a.rho.tolist() == [0, 0, 0]
    assert Cn.tolist() == [[1.0], [100.0]]
    assert E == 2.0


def test_near_tie_threshold():
    # d1 = 1, d2 = 1 + 5e-7 -> relative gap 5e-7 < 1e-6: near tie
    X = np.array([[0.0]])
    C = np.array([[1.0], [-math.sqrt(1 + 5e-7)]])
    assert ko.assign(X, C).near_tie[0]
    C = np.array([[1.0], [-math.sqrt(1 + 3e-6)]])
    assert not ko.assign(X, C).near_tie[0]


def test_duplicate_points():
    X = np.repeat(np.array([[1.0, 2.0], [5.0, 5.0]]), 50, axis=0)
    res = ko.solve(X, X[[0, 1]], m_max=10, tol=0.0)   # both seeds from group 0
    # one centroid takes group 0, the other stays empty or moves: energy finite
    assert math.isfinite(res.E)
    res = ko.solve(X, X[[0, 60]], m_max=10, tol=0.0)
    assert res.E == 0.0 and res.iters == 1


# ---------------------------------------------------------------------------
# Hand-derived worked example (tests/golden/tiny_1d.json)
# ---------------------------------------------------------------------------

def _frac(s):
    return float(Fraction(s))


def test_golden_tiny_1d():
    with open(os.path.join(GOLDEN, "tiny_1d.json")) as f:
        g = json.load(f)
    X = np.array(g["X"], dtype=np.float64)
    C0 = np.array(g["C0"], dtype=np.float64)
    res = ko.solve(X, C0, m_max=g["m_max"], tol=0.0)
    exp = g["expected"]
    assert res.iters == exp["iters"]
    assert res.rejected == exp["rejected"] and res.accepted == exp["accepted"]
    assert res.assign_passes == exp["assign_passes"]
    assert res.rho.tolist() == exp["rho"]
    np.testing.assert_allclose(res.C.ravel(), [_frac(v) for v in exp["C"]], rtol=1e-15)
    assert res.E == pytest.approx(_frac(exp["E"]), rel=1e-15)
    # first iteration values
    t1 = res.trace[0]
    assert t1["E_cand"] == pytest.approx(_frac(exp["E1"]), rel=1e-14)
    assert t1["theta"][0] == pytest.approx(_frac(exp["theta1"]), rel=1e-9)
    # the literal reading of Algorithm 1 returns the accelerated iterate
    lit = ko.solve(X, C0, m_max=g["m_max"], tol=0.0, literal_return=True)
    np.testing.assert_allclose(lit.C.ravel(), [_frac(v) for v in exp["literal_C"]], rtol=1e-9)
    assert lit.iters == exp["iters"] and lit.rejected == 0


def test_golden_tol_reject_1d():
    """Stopping rule on the accepted energy after a rejection (reading R3):
    tests/golden/tol_reject_1d.json, derived by hand in exact rationals."""
    with open(os.path.join(GOLDEN, "tol_reject_1d.json")) as f:
        g = json.load(f)
    X = np.array(g["X"], dtype=np.float64)
    C0 = np.array(g["C0"], dtype=np.float64)
    exp = g["expected"]
    res = ko.solve(X, C0, m_max=g["m_max"], tol=g["tol"])
    assert res.status == ko.STATUS_CONVERGED
    assert res.iters == exp["iters"]
    assert (res.accepted, res.rejected, res.assign_passes) == (exp["accepted"], exp["rejected"],
                                                               exp["assign_passes"])
    assert res.m_final == exp["m_final"]
    assert res.rho.tolist() == exp["rho"]
    assert [r["decision"] for r in res.trace] == exp["decisions"]
    assert [r["E_cand"] for r in res.trace] == pytest.approx([_frac(v) for v in exp["E_cand"]], rel=1e-11)
    assert res.trace[1]["E_fb"] == _frac(exp["E_fb_t2"])
    assert [r["theta"][0] for r in res.trace[:2]] == pytest.approx([_frac(v) for v in exp["theta"]], rel=1e-9)
    assert res.trace[-1]["stop"] == "tol"
    np.testing.assert_allclose(res.C.ravel(), [_frac(v) for v in exp["C"]], rtol=1e-12)
    assert res.E == pytest.approx(_frac(exp["E"]), rel=1e-11)
    z = exp["tol0"]
    r0 = ko.solve(X, C0, m_max=g["m_max"], tol=0.0)
    assert r0.iters == z["iters"] and r0.rho.tolist() == z["rho"]
    np.testing.assert_allclose(r0.C.ravel(), [_frac(v) for v in z["C"]], rtol=1e-15)
    assert r0.E == _frac(z["E"])


# ---------------------------------------------------------------------------
# Bound-based assignment (Hamerly's lower bound, Sec. 3)
# ---------------------------------------------------------------------------

def _true_labels_and_second(X, C):
    """Brute force: every distance written out, lowest index on ties."""
    n, k = X.shape[0], C.shape[0]
    D = np.empty((n, k))
    for j in range(k):
        D[:, j] = np.sqrt(((X - C[j]) ** 2).sum(axis=1))
    rho = np.argmin(D, axis=1)
    D2 = D.copy()
    D2[np.arange(n), rho] = np.inf
    return rho, D2.min(axis=1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bounded_assignment_walk(seed):
    """Along a walk of centroid sets with shrinking and growing steps the
    bounded assignment gives the brute-force labels, every bound stays below
    the true distance to every other centroid, and small steps keep most
    rows while large ones keep few."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(600, 3)) * 3.0
    C = X[rng.choice(600, 7, replace=False)].copy()
    rho, second = _true_labels_and_second(X, C)
    lb = second.copy()
    kept_frac = []
    for scale in (1e-3, 1e-2, 0.1, 1e-3, 1.0, 3.0, 1e-4, 1e-2):
        Cn = C + rng.normal(size=C.shape) * scale
        a, lbn, kept = ko.assign_bounded(X, Cn, C, rho, lb)
        r_true, s_true = _true_labels_and_second(X, Cn)
        assert np.array_equal(a.rho, r_true)
        assert np.all(lbn <= s_true * (1 + 1e-12))
        kept_frac.append(kept.mean())
        C, rho, lb = Cn, a.rho, lbn
    assert kept_frac[0] > 0.9 and kept_frac[6] > 0.9
    assert kept_frac[5] < 0.5


def test_bounded_assignment_other_centroid_moves_in():
    """One sample at 0 labelled with c_0 = 0.1 (bound 0.9 from c_1 = 1.0).
    c_1 moves to 0.05: the largest shift of another centroid (0.95) exceeds
    the bound, so the row is assigned in full and takes c_1.  Subtracting the
    row's own centroid shift (0) instead would keep the stale label."""
    X = np.array([[0.0]])
    C_ref = np.array([[0.1], [1.0]])
    a, lb, kept = ko.assign_bounded(X, np.array([[0.1], [0.05]]), C_ref, np.array([0]), np.array([0.9]))
    assert not kept[0]
    assert a.rho.tolist() == [1]
    assert lb[0] == pytest.approx(0.1)


def test_bounded_assignment_own_centroid_moves_most():
    """c_0 (the row's own centroid) moves by 0.5, the others stay: the shift
    subtracted from the bound is the largest among the OTHER centroids (0),
    so the row is kept with its bound 0.9; subtracting the overall largest
    shift (0.5) would give 0.4 < 0.6 and force a full assignment."""
    X = np.array([[0.0]])
    C_ref = np.array([[0.1], [1.0], [2.0]])
    Cn = np.array([[0.6], [1.0], [2.0]])
    a, lb, kept = ko.assign_bounded(X, Cn, C_ref, np.array([0]), np.array([0.9]))
    assert kept[0]
    assert a.rho.tolist() == [0]
    assert lb[0] == pytest.approx(0.9)


def test_bounded_assignment_static_centroids_keep_all_but_near_ties():
    """Centroids that do not move and exact bounds: every row is kept except
    those within the near-tie margin, which are assigned in full."""
    X = np.array([[0.0], [0.5], [0.5 + 1e-9], [2.0]])
    C = np.array([[0.0], [1.0], [2.5]])
    rho, second = _true_labels_and_second(X, C)
    a, lb, kept = ko.assign_bounded(X, C, C, rho, second)
    assert kept.tolist() == [True, False, False, True]
    assert np.array_equal(a.rho, rho)
    assert a.near_tie.tolist() == [False, True, True, False]
