"""Plain FP64 CPU reference for Anderson-accelerated Lloyd K-Means.

TEST INFRASTRUCTURE ONLY.  This module is the correctness oracle: it may be
imported by the test-suite, by the smoke check and by the CPU-baseline leg of
the benchmark, and by nothing else.  The GPU library never calls it, and it
shares no code with the GPU library (the only common dependency is the seeded
input generator module, which holds none of the method's arithmetic).

Everything here is written for clarity, not speed: float64 NumPy, direct
differences for distances, no blocking or fusion beyond what the definitions
state.  Inputs are the stored float32/bfloat16 values, upcast exactly.

Paper: Zhang, Yao, Peng, Yu, Deng, "Fast K-Means Clustering with Anderson
Acceleration" (arXiv 1805.10638).

  * energy                  -- Sec. 1, Eq. (1)
  * assignment step         -- Sec. 1, Eq. (3)
  * update step             -- Sec. 1, Eq. (4)
  * fixed-point map G       -- Sec. 2.1, Eq. (6)
  * least-squares problem   -- Sec. 2.1, Eq. (7)
  * accelerated iterate     -- Sec. 2.1, Eq. (8) and Algorithm 1
  * energy safeguard        -- Sec. 2.1 (revert to the Lloyd iterate)
  * dynamic m               -- Sec. 2.2, Algorithm 1
  * default parameters      -- Sec. 3 (eps1=0.02, eps2=0.5, m initialised to 2)
  * bound-based assignment  -- Sec. 3 (the experiments run the assignment
                               step with Hamerly's lower-bound method)

Readings of points the paper leaves open (each is listed with its reason in
the design notes of the repository):
  R1  P^0 is the assignment of C^0 (computed inside G(C^0)).
  R2  An accelerated iterate whose assignment equals the previous one is not
      returned; the fall-back Lloyd iterate is taken instead, and the run ends
      when that fall-back reproduces the previous assignment (Sec. 2.1, last
      paragraph).  ``literal_return=True`` returns at the first equal
      assignment instead (Algorithm 1 as printed).
  R3  Optional stopping rule: stop after the accept/reject decision when the
      relative decrease of the accepted energy is at most ``tol``.
  R4  The accelerated iterate is G^t - sum_j theta_j (G^{t-j+1} - G^{t-j})
      (the sign of Algorithm 1; the only one consistent with Eq. (7)).
  R5  The m-rule is skipped while E^{t-2} is not finite and is evaluated in
      cross-multiplied form  num < eps1*den / num > eps2*den  with
      num = E^{t-1} - E^t (E^t of the candidate), den = E^{t-2} - E^{t-1}.
  R6  The fall-back iterate at iteration t is G^{t-1} = Update(P^{t-1}).
  R7  A candidate that already is the Lloyd iterate (no column used in the
      least-squares problem) is never "reverted" to itself.
  R8  Least squares by normal equations on norm-scaled columns with ridge
      1e-10 and a Cholesky factorisation; zero columns are dropped.
  R9  An empty cluster keeps its input centroid.
  R10 argmin ties go to the lowest index.
  R11 Near tie: (d2 - d1) < 1e-6 * d2 on float64 direct-difference
      distances (d1, d2 the smallest and second smallest); d2 = 0 counts.
  R12 m starts at min(2, m_max); the history keeps the last m_max + 1
      (G, F) pairs and is not reset when an iterate is rejected.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EPS1 = 0.02          # Sec. 3
EPS2 = 0.5           # Sec. 3
M_INIT = 2           # Sec. 3
RIDGE = 1e-10        # reading R8
NEAR_TIE_REL = 1e-6  # reading R11

STATUS_CONVERGED = 0
STATUS_NOT_CONVERGED = 1
STATUS_NONFINITE = -5


def _f64(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Lloyd primitives (Sec. 1)
# ---------------------------------------------------------------------------

def squared_distances(X, C) -> np.ndarray:
    """D[i, j] = sum_k (X[i,k] - C[j,k])^2 in float64 by direct differences."""
    X = _f64(X)
    C = _f64(C)
    diff = X[:, None, :] - C[None, :, :]
    return np.einsum("ijk,ijk->ij", diff, diff)


@dataclass
class Assignment:
    rho: np.ndarray        # int64 labels (Eq. 3), lowest index on ties (R10)
    d1: np.ndarray         # smallest squared distance per row
    d2: np.ndarray         # second smallest (inf when K == 1)
    near_tie: np.ndarray   # bool, reading R11


def assign(X, C, rows_per_chunk: int | None = None) -> Assignment:
    """Assignment step, Eq. (3): rho_i = argmin_j ||x_i - c_j||."""
    X = _f64(X)
    C = _f64(C)
    n, k = X.shape[0], C.shape[0]
    if rows_per_chunk is None:
        rows_per_chunk = max(1, (1 << 22) // max(1, k * X.shape[1]))
    rho = np.empty(n, dtype=np.int64)
    d1 = np.empty(n)
    d2 = np.full(n, np.inf)
    for s in range(0, n, rows_per_chunk):
        D = squared_distances(X[s:s + rows_per_chunk], C)
        r = np.argmin(D, axis=1)          # first minimum: lowest index
        rho[s:s + len(r)] = r
        best = D[np.arange(len(r)), r]
        d1[s:s + len(r)] = best
        if k > 1:
            D[np.arange(len(r)), r] = np.inf
            d2[s:s + len(r)] = D.min(axis=1)
    near = (d2 - d1) < NEAR_TIE_REL * d2
    near |= (d2 == 0.0)
    return Assignment(rho, d1, d2, near)


def assign_bounded(X, C, C_ref, rho_ref, lb_ref):
    """Assignment step with one lower bound per sample (Hamerly's method, the
    assignment the paper's experiments use, Sec. 3).

    ``lb_ref[i]`` is a lower bound of the distance from x_i to every centroid
    of ``C_ref`` other than its label ``rho_ref[i]``.  When the centroids move
    to C, each distance to a centroid j changes by at most
    delta_j = ||C_j - C_ref_j|| (triangle inequality), so
    lp_i = lb_ref[i] - max_{j != rho_ref[i]} delta_j bounds the distance from
    x_i to every other centroid of C.  If the distance d1 to C[rho_ref[i]]
    satisfies d1^2 (1 + 2.1e-6) < lp_i^2, the label is unchanged (and the row
    is not a near tie, R11); otherwise the row is assigned in full.  The new
    bound is lp_i for kept rows and the second smallest distance for the
    others.

    Returns (Assignment, lb_new, kept) where the Assignment is the one of
    assign(X, C) (labels identical; d1, d2 and near ties of the full rows,
    d2 = lp^2 and no near tie for kept rows)."""
    X = _f64(X)
    C = _f64(C)
    C_ref = _f64(C_ref)
    rho_ref = np.asarray(rho_ref)
    lb_ref = _f64(lb_ref)
    n, k = X.shape[0], C.shape[0]
    delta = np.sqrt(((C - C_ref) ** 2).sum(axis=1))
    if k > 1:
        order = np.argsort(-delta, kind="stable")
        excl = np.where(rho_ref == order[0], delta[order[1]], delta[order[0]])
    else:
        excl = np.zeros(n)
    lp = lb_ref - excl
    diff = X - C[rho_ref]
    d1 = np.einsum("ij,ij->i", diff, diff)
    kept = (lp > 0) & (d1 * (1.0 + 2.1e-6) < lp * lp)
    rest = np.flatnonzero(~kept)
    full = assign(X[rest], C)
    rho = rho_ref.astype(np.int64).copy()
    rho[rest] = full.rho
    out_d1 = d1.copy()
    out_d1[rest] = full.d1
    out_d2 = np.where(kept, lp * lp, np.inf)
    out_d2[rest] = full.d2
    near = np.zeros(n, dtype=bool)
    near[rest] = full.near_tie
    lb_new = np.where(kept, lp, 0.0)
    lb_new[rest] = np.sqrt(full.d2)
    return Assignment(rho, out_d1, out_d2, near), lb_new, kept


def energy(X, rho, C) -> float:
    """Eq. (1) evaluated with a given assignment: sum_i ||x_i - c_{rho_i}||^2.

    Row terms are formed by direct differences; their total is the correctly
    rounded sum (math.fsum)."""
    X = _f64(X)
    C = _f64(C)
    diff = X - C[np.asarray(rho)]
    return math.fsum(np.einsum("ij,ij->i", diff, diff).tolist())


def update(X, rho, C):
    """Update step, Eq. (4): c_j = mean of the samples assigned to j.

    An empty cluster keeps its input centroid (R9).  Returns (C_new, counts)."""
    X = _f64(X)
    C = _f64(C)
    k, d = C.shape
    rho = np.asarray(rho)
    counts = np.bincount(rho, minlength=k)
    sums = np.empty((k, d))
    for col in range(d):
        sums[:, col] = np.bincount(rho, weights=X[:, col], minlength=k)
    Cn = C.copy()
    nz = counts > 0
    Cn[nz] = sums[nz] / counts[nz, None]
    return Cn, counts


def g(X, C):
    """The fixed-point map of Eq. (6): G(C) = Update(Assign(C)).

    Returns (assignment, G(C), E(C)) where E(C) uses the assignment of C."""
    a = assign(X, C)
    Cn, _ = update(X, a.rho, C)
    return a, Cn, energy(X, a.rho, C)


# ---------------------------------------------------------------------------
# Anderson acceleration (Sec. 2.1)
# ---------------------------------------------------------------------------

def ridge_least_squares(dF: np.ndarray, F: np.ndarray, lam: float = RIDGE) -> np.ndarray:
    """theta = argmin ||F - dF theta||^2 (Eq. 7), reading R8.

    dF has one column per difference F^{t-j+1} - F^{t-j}.  Columns are scaled
    to unit norm, the normal equations get a ridge ``lam`` and are solved by
    Cholesky; the scaling is undone afterwards.  Zero columns get theta = 0."""
    dF = _f64(dF)
    F = _f64(F)
    m = dF.shape[1]
    theta = np.zeros(m)
    if m == 0:
        return theta
    gram = dF.T @ dF                       # m inner products per new column
    rhs = dF.T @ F
    s = np.sqrt(np.diag(gram))
    keep = np.flatnonzero(s > 0.0)
    if keep.size == 0:
        return theta
    sk = s[keep]
    A = gram[np.ix_(keep, keep)] / np.outer(sk, sk) + lam * np.eye(keep.size)
    b = rhs[keep] / sk
    L = np.linalg.cholesky(A)
    y = _back_substitute(L.T, _forward_substitute(L, b))
    theta[keep] = y / sk
    return theta


def _forward_substitute(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    n = b.size
    y = np.zeros(n)
    for i in range(n):
        y[i] = (b[i] - L[i, :i] @ y[:i]) / L[i, i]
    return y


def _back_substitute(U: np.ndarray, y: np.ndarray) -> np.ndarray:
    n = y.size
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - U[i, i + 1:] @ x[i + 1:]) / U[i, i]
    return x


class History:
    """The last ``capacity`` pairs (G^s, F^s) as flat float64 vectors."""

    def __init__(self, capacity: int):
        self.capacity = max(1, capacity)
        self.G: list[np.ndarray] = []
        self.F: list[np.ndarray] = []

    def push(self, G, F) -> None:
        self.G.append(_f64(G).ravel().copy())
        self.F.append(_f64(F).ravel().copy())
        if len(self.G) > self.capacity:
            self.G.pop(0)
            self.F.pop(0)

    def differences(self, mt: int):
        """Columns j=1..mt of F^{t-j+1}-F^{t-j} and G^{t-j+1}-G^{t-j}."""
        dF = np.stack([self.F[-j] - self.F[-j - 1] for j in range(1, mt + 1)], axis=1) \
            if mt > 0 else np.zeros((self.F[-1].size, 0))
        dG = np.stack([self.G[-j] - self.G[-j - 1] for j in range(1, mt + 1)], axis=1) \
            if mt > 0 else np.zeros((self.G[-1].size, 0))
        return dF, dG

    def accelerate(self, mt: int, lam: float = RIDGE):
        """Eq. (7) then the accelerated iterate (R4): returns (x_next, theta, used)
        where ``used`` counts the columns that entered the least squares."""
        G, F = self.G[-1], self.F[-1]
        dF, dG = self.differences(mt)
        theta = ridge_least_squares(dF, F, lam)
        used = int(np.count_nonzero(np.linalg.norm(dF, axis=0) > 0.0)) if mt > 0 else 0
        x = G - dG @ theta if mt > 0 else G.copy()
        return x, theta, used


# ---------------------------------------------------------------------------
# Dynamic m (Sec. 2.2)
# ---------------------------------------------------------------------------

def adjust_m(m: int, E: float, E1: float, E2: float, m_max: int,
             eps1: float = EPS1, eps2: float = EPS2) -> int:
    """Ratio rule of Sec. 2.2 with reading R5.

    r = (E^{t-1} - E^t) / (E^{t-2} - E^{t-1});  r < eps1 shrinks m,
    r > eps2 grows m, otherwise m is kept.  Skipped while E^{t-2} is inf."""
    if not math.isfinite(E2):
        return m
    num = E1 - E
    den = E2 - E1
    if num < eps1 * den:
        return max(m - 1, 0)
    if num > eps2 * den:
        return min(m + 1, m_max)
    return m


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    C: np.ndarray
    rho: np.ndarray
    E: float
    iters: int
    status: int
    accepted: int = 0
    rejected: int = 0
    assign_passes: int = 0
    m_final: int = 0
    trace: list = field(default_factory=list)


def solve(X, C0, m_max: int = 10, tol: float = 1e-6, max_iter: int = 500,
          eps1: float = EPS1, eps2: float = EPS2, m_init: int = M_INIT,
          fixed_m: bool = False, literal_return: bool = False,
          replay=None, stored=None, lam: float = RIDGE, stored_cand=None) -> SolveResult:
    """Anderson-accelerated Lloyd iteration with dynamic m (Algorithm 1).

    ``replay(t)`` may return a centroid array that replaces the candidate
    C^t at the start of iteration t (used to follow another implementation's
    iterates step by step); returning None keeps the oracle's own candidate.
    ``stored(C)`` maps the fall-back iterate to the values another
    implementation stores for it (e.g. float32 rounding) when replaying;
    by default the fall-back is the float64 G^{t-1} itself.  ``stored_cand(C)``
    does the same for every candidate C^t (C^1 = G^0 and each accelerated
    iterate), so that an implementation which stores its iterates in float32
    can be followed end to end without replaying its candidates; by default
    candidates stay float64.  Neither hook changes any arithmetic of the
    method, only the values an iterate is stored as.
    """
    X = _f64(X)
    C0 = _f64(C0)
    k, d = C0.shape
    m = min(m_init, m_max)

    # Initialisation: C^1 = G(C^0), F^0 = C^1 - C^0, E^0 = +inf  (R1)
    a0 = assign(X, C0)
    P_prev = a0.rho
    G_prev, _ = update(X, P_prev, C0)
    hist = History(m_max + 1)
    hist.push(G_prev, G_prev - C0)
    C = G_prev.copy() if stored_cand is None else _f64(stored_cand(G_prev)).reshape(k, d)
    C_is_lloyd = True
    E1 = math.inf        # E^{t-1}
    E2 = math.inf        # E^{t-2}
    C_acc, passes = C0, 1
    accepted = rejected = 0
    trace = []

    def finish(P, Cr, E, t, status):
        return SolveResult(Cr.copy(), P.copy(), E, t, status, accepted, rejected,
                           passes, m, trace)

    for t in range(1, max_iter + 1):
        if replay is not None:
            Cr = replay(t)
            if Cr is not None:
                C = _f64(Cr).reshape(k, d).copy()
        rec = {"t": t}

        a = assign(X, C)
        passes += 1
        P = a.rho
        E = energy(X, P, C)
        rec.update(E_cand=E, changed_cand=int(np.count_nonzero(P != P_prev)),
                   cand_is_lloyd=C_is_lloyd, cand_near_ties=int(a.near_tie.sum()))
        if not math.isfinite(E):
            trace.append(rec)
            return finish(P, C, E, t, STATUS_NONFINITE)
        same = bool(np.array_equal(P, P_prev))
        if same and (C_is_lloyd or literal_return):
            rec.update(decision="converged", E_acc=E, m=m)
            trace.append(rec)
            return finish(P, C, E, t, STATUS_CONVERGED)

        if not fixed_m:
            m = adjust_m(m, E, E1, E2, m_max, eps1, eps2)
        rec["m"] = m

        if not C_is_lloyd and (same or E >= E1):
            # Revert to the Lloyd iterate (Sec. 2.1 safeguard; R2, R6)
            C = G_prev.copy() if stored is None else _f64(stored(G_prev)).reshape(k, d)
            a = assign(X, C)
            passes += 1
            P = a.rho
            E = energy(X, P, C)
            rejected += 1
            rec.update(decision="rejected", E_fb=E,
                       changed_fb=int(np.count_nonzero(P != P_prev)))
            if not math.isfinite(E):
                trace.append(rec)
                return finish(P, C, E, t, STATUS_NONFINITE)
            if np.array_equal(P, P_prev):
                rec.update(E_acc=E, stop="fixed_point")
                trace.append(rec)
                return finish(P, C, E, t, STATUS_CONVERGED)
        else:
            if not C_is_lloyd:
                accepted += 1
            rec["decision"] = "accepted" if not C_is_lloyd else "lloyd"
        rec["E_acc"] = E

        if tol > 0 and math.isfinite(E1) and (E1 - E) <= tol * E1:   # R3
            rec["stop"] = "tol"
            trace.append(rec)
            return finish(P, C, E, t, STATUS_CONVERGED)

        # Anderson step
        G, _ = update(X, P, C)
        F = G - C
        hist.push(G, F)
        mt = min(m, t)
        x_next, theta, used = hist.accelerate(mt, lam)
        rec.update(mt=mt, used=used, theta=theta.tolist(), G=G.copy(),
                   C_next=x_next.reshape(k, d).copy())
        trace.append(rec)

        E2, E1 = E1, E
        P_prev, G_prev, C_acc = P, G, C
        C = x_next.reshape(k, d) if stored_cand is None else _f64(stored_cand(x_next.reshape(k, d))).reshape(k, d)
        C_is_lloyd = used == 0

    return finish(P_prev, C_acc, E1, max_iter, STATUS_NOT_CONVERGED)


def lloyd(X, C0, tol: float = 1e-6, max_iter: int = 500) -> SolveResult:
    """Plain Lloyd: Algorithm 1 with the history disabled (m_max = 0)."""
    return solve(X, C0, m_max=0, tol=tol, max_iter=max_iter)
