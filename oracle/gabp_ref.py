"""FP64 reference (oracle) for the GaBP SVM solver -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy code.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path never does.  It shares no code with the HIP library.

Paper: Bickson, Yom-Tov, Dolev, "A Gaussian Belief Propagation Solver for
Large Scale Support Vector Machines" (arXiv 0810.1648).

What is computed, with the passage each step follows:

* The SVM dual (section "Classification Using Support Vector Machines",
  eqs. dual/cons1/cons2): maximise sum(h) - 1/2 h'Dh with
  D_ij = y_i y_j K(x_i, x_j).
* The constraints are dropped (section "Proposed Solution of SVM Solver
  Based on GaBP"): the method solves the linear system A h = 1 whose
  solution is the mean of p(h) ~ exp(-1/2 h'Ah + h'1).
* Bias by augmentation with the constant lambda = 1/N (same section); in
  feature space this adds lambda^2 to every kernel entry (reading C2 in the
  design notes).
* The diagonal of D is weighted to make it diagonally dominant (subsection
  "GaBP Algorithm Convergence"; the 2-norm soft margin adds 1/C).
* GaBP: Algorithm 1 (per-message exclusion sums) and Algorithm 2
  (broadcast aggregates, each outgoing message = aggregate minus the
  recipient's own term), in synchronous rounds (section "Experimental
  Results": synchronous communication rounds).

Parity unpinned: none -- every function below is pinned by a test in
tests/test_oracle_pins.py against closed forms, LAPACK, brute force or an
invariant.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

# --------------------------------------------------------------------------
# System construction
# --------------------------------------------------------------------------

DIAG_NONE = "none"
DIAG_SOFTMARGIN = "softmargin"
DIAG_DOMINANT_ROW = "dominant_row"
DIAG_DOMINANT_UNIFORM = "dominant_uniform"


def rbf_augmented_kernel(X, gamma: float, lam: float, chunk: int = 64) -> np.ndarray:
    """K'_ij = exp(-gamma ||x_i - x_j||^2) + lam^2, in FP64.

    The RBF kernel is the one used in every experiment (section
    "Experimental Results"); the lam^2 term is the bias augmentation of
    section "Proposed Solution of SVM Solver Based on GaBP" read in feature
    space.  Distances are direct differences (no Gram expansion).
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    K = np.empty((n, n))
    for i0 in range(0, n, chunk):
        d2 = ((X[i0:i0 + chunk, None, :] - X[None, :, :]) ** 2).sum(axis=-1)
        K[i0:i0 + chunk] = np.exp(-gamma * d2)
    return K + lam * lam


def signed_matrix(K: np.ndarray, y) -> np.ndarray:
    """D_ij = y_i y_j K_ij (eq. dual)."""
    y = np.asarray(y, dtype=np.float64)
    return y[:, None] * y[None, :] * K


def weight_diagonal(D: np.ndarray, C: float, mode: str = DIAG_DOMINANT_ROW,
                    delta: float = 0.1) -> np.ndarray:
    """Return A = D with its diagonal weighted (subsection "GaBP Algorithm
    Convergence").

    none:             A_ii = D_ii
    softmargin:       A_ii = D_ii + 1/C   (2-norm soft margin)
    dominant_row:     A_ii = max(D_ii + 1/C, (1 + delta) r_i),
                      r_i = sum_{j != i} |D_ij|
    dominant_uniform: one shift w = max_i (max(D_ii + 1/C, (1+delta) r_i) - D_ii)
                      added to every diagonal entry.
    """
    A = np.array(D, dtype=np.float64, copy=True)
    d = np.diag(D).copy()
    r = np.abs(D).sum(axis=1) - np.abs(d)
    if mode == DIAG_NONE:
        new = d
    elif mode == DIAG_SOFTMARGIN:
        new = d + 1.0 / C
    elif mode == DIAG_DOMINANT_ROW:
        new = np.maximum(d + 1.0 / C, (1.0 + delta) * r)
    elif mode == DIAG_DOMINANT_UNIFORM:
        w = np.max(np.maximum(d + 1.0 / C, (1.0 + delta) * r) - d)
        new = d + w
    else:
        raise ValueError(mode)
    A[np.diag_indices_from(A)] = new
    return A


def svm_system(X, y, gamma: float, C: float, lam: float,
               mode: str = DIAG_DOMINANT_ROW, delta: float = 0.1):
    """A = weighted(Y K' Y) and b = 1: the linear system GaBP solves."""
    K = rbf_augmented_kernel(X, gamma, lam)
    A = weight_diagonal(signed_matrix(K, y), C, mode, delta)
    return A, np.ones(A.shape[0])


# --------------------------------------------------------------------------
# Sparsified kernel (closing discussion: sparsify the kernel matrix to reach
# millions of points; not the paper's experiments)
# --------------------------------------------------------------------------


def sparse_threshold_d2(gamma: float, tau: float) -> float:
    """exp(-gamma d^2) >= tau  <=>  d^2 <= -ln(tau) / gamma."""
    return -np.log(tau) / gamma


def pair_sq_distances(X, chunk: int = 64) -> np.ndarray:
    """||x_i - x_j||^2 in FP64 by direct differences."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    D2 = np.empty((n, n))
    for i0 in range(0, n, chunk):
        D2[i0:i0 + chunk] = ((X[i0:i0 + chunk, None, :] - X[None, :, :]) ** 2).sum(axis=-1)
    return D2


def sparse_rbf_augmented_kernel(X, gamma: float, lam: float, tau: float) -> np.ndarray:
    """Thresholded kernel: K'_ij = exp(-gamma d^2) + lam^2 for the pairs with
    exp(-gamma d^2) >= tau (d^2 <= -ln(tau)/gamma), 0 for the other pairs
    i != j; the diagonal keeps 1 + lam^2.  The graph of the GaBP messages is
    the set of kept pairs."""
    D2 = pair_sq_distances(X)
    keep = D2 <= sparse_threshold_d2(gamma, tau)
    np.fill_diagonal(keep, True)
    return np.where(keep, np.exp(-gamma * D2) + lam * lam, 0.0)


def sparse_edges(X, gamma: float, tau: float) -> np.ndarray:
    """Kept pairs (i, j), i < j, in lexicographic order (int64, shape E x 2)."""
    D2 = pair_sq_distances(X)
    iu, ju = np.nonzero(np.triu(D2 <= sparse_threshold_d2(gamma, tau), k=1))
    return np.stack([iu, ju], axis=1).astype(np.int64)


def sparse_svm_system(X, y, gamma: float, C: float, lam: float, tau: float,
                      mode: str = DIAG_DOMINANT_ROW, delta: float = 0.1):
    """A = weighted(Y K'_sparse Y), b = 1 (the diagonal rule sees the sparse
    row sums)."""
    K = sparse_rbf_augmented_kernel(X, gamma, lam, tau)
    A = weight_diagonal(signed_matrix(K, y), C, mode, delta)
    return A, np.ones(A.shape[0])


def sparse_tau_with_gap(X, gamma: float, mean_degree: float, rel_gap: float = 1e-3):
    """A threshold tau for about `mean_degree` kept neighbours per point whose
    distance cut d2* sits in a gap of the pair distances: no pair has
    |d^2 - d2*| <= rel_gap d2*, so any distance computation accurate to
    better than that keeps the same pairs.  Returns (tau, d2*)."""
    D2 = pair_sq_distances(X)
    n = D2.shape[0]
    v = np.sort(D2[np.triu_indices(n, k=1)])
    k0 = int(min(len(v) - 2, max(1, mean_degree * n / 2)))
    for step in range(len(v)):
        for k in (k0 + step, k0 - step):
            if 1 <= k < len(v) - 1:
                lo, hi = v[k], v[k + 1]
                mid = 0.5 * (lo + hi)
                if mid > 0 and (mid - lo) > rel_gap * mid and (hi - mid) > rel_gap * mid:
                    return float(np.exp(-gamma * mid)), float(mid)
    raise ValueError("no gap found")


# --------------------------------------------------------------------------
# Algorithm 1: GaBP with per-message exclusion sums (tiny N only)
# --------------------------------------------------------------------------

def gabp_algorithm1(A, b, sweeps: int):
    """Algorithm 1, synchronous schedule.  Returns the list of marginal
    means after each sweep 1..sweeps (step 4 "Infer").

    Messages are kept in the paper's mean/precision form: P[k, i] and
    M[k, i] are the precision and mean of the message k -> i.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    nbr = [[k for k in range(n) if k != i and A[k, i] != 0.0] for i in range(n)]
    Pii = np.diag(A).copy()                 # scalar fixes, step 1
    mu_ii = b / Pii
    P = np.zeros((n, n))
    M = np.zeros((n, n))
    out = []
    for _ in range(sweeps):
        Pn = np.zeros((n, n))
        Mn = np.zeros((n, n))
        for i in range(n):
            for j in nbr[i]:
                excl = [k for k in nbr[i] if k != j]
                prec = Pii[i] + sum(P[k, i] for k in excl)
                info = Pii[i] * mu_ii[i] + sum(P[k, i] * M[k, i] for k in excl)
                Pn[i, j] = -A[i, j] ** 2 / prec
                Mn[i, j] = info / A[i, j]
        P, M = Pn, Mn
        mu = np.array([(Pii[i] * mu_ii[i] + sum(P[k, i] * M[k, i] for k in nbr[i]))
                       / (Pii[i] + sum(P[k, i] for k in nbr[i])) for i in range(n)])
        out.append(mu)
    return out


# --------------------------------------------------------------------------
# Algorithm 2 in the paper's mean form (small N)
# --------------------------------------------------------------------------

def gabp_algorithm2_mean_form(A, b, sweeps: int):
    """Algorithm 2 exactly as printed: broadcast P~_i, mu~_i, then every
    internal scalar from the aggregate minus the recipient's own term,
    P_ij = -A_ij^2 / (P~_i - P_ji), mu_ij = (P~_i mu~_i - P_ji mu_ji) / A_ij.
    Requires A_ij != 0 wherever messages flow (dense positive kernels).
    Returns the marginal means after each sweep.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    off = ~np.eye(n, dtype=bool) & (A != 0.0)
    Pii = np.diag(A).copy()
    mu_ii = b / Pii
    P = np.zeros((n, n))                    # P[k, i]: k -> i
    M = np.zeros((n, n))
    out = []
    for _ in range(sweeps):
        Pt = Pii + P.sum(axis=0)
        mut = (Pii * mu_ii + (P * M).sum(axis=0)) / Pt
        Pn = np.zeros((n, n))
        Mn = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                if off[i, j]:
                    Pn[i, j] = -A[i, j] ** 2 / (Pt[i] - P[j, i])
                    Mn[i, j] = (Pt[i] * mut[i] - P[j, i] * M[j, i]) / A[i, j]
        P, M = Pn, Mn
        Pt = Pii + P.sum(axis=0)
        out.append((Pii * mu_ii + (P * M).sum(axis=0)) / Pt)
    return out


# --------------------------------------------------------------------------
# Algorithm 2 in information form: the oracle used for parity
# --------------------------------------------------------------------------

CONVERGED = "converged"
NOT_CONVERGED = "not_converged"
DIVERGED = "diverged"
STAGNATED = "stagnated"


@dataclass
class GabpResult:
    alpha: np.ndarray          # marginal means after the last sweep
    ptilde: np.ndarray         # aggregate precisions P~ after the last sweep
    sweeps: int                # completed sweeps
    status: str
    deltas: list               # ||alpha^t - alpha^(t-1)||_inf, t = 1..sweeps
    trajectory: list | None    # alpha^0, alpha^1, ... if requested


def gabp_solve(A, b, max_sweeps: int = 1000, tol_abs: float = 0.0,
               tol_rel: float = 1e-12, keep_trajectory: bool = False) -> GabpResult:
    """Synchronous Algorithm 2 with messages stored in information form.

    State: P[i, j] = precision of the message i -> j and
    E[i, j] = P_ij mu_ij (its information).  Aggregates (step 2
    "broadcast"): P~_j = A_jj + sum_i P_ij, S_j = b_j + sum_i E_ij, so that
    mu~_j = S_j / P~_j.  Internal scalars from the aggregate minus the
    recipient's own term: with Q_ij = P~_i - P_ji,
        P_ij <- -A_ij^2 / Q_ij,     E_ij <- -A_ij (S_i - E_ji) / Q_ij,
    which is Algorithm 2's mu_ij multiplied by P_ij.  Sweep 0 is the
    aggregate of all-zero messages; alpha^t = S^t / P~^t (step 4 "Infer").

    Stops when ||alpha^t - alpha^(t-1)||_inf <= tol_abs + tol_rel
    ||alpha^t||_inf (step 3 "Check", tested on alpha), after max_sweeps
    (not converged), or when some Q_ij <= 0, P~ <= 0 or a value is not
    finite (diverged: no valid Gaussian message exists).
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    off = ~np.eye(n, dtype=bool)
    Aoff = np.where(off, A, 0.0)
    A2 = Aoff * Aoff
    P = np.zeros((n, n))
    E = np.zeros((n, n))
    Pt = np.diag(A).copy()
    S = b.copy()
    alpha = S / Pt
    traj = [alpha.copy()] if keep_trajectory else None
    deltas = []
    status = NOT_CONVERGED
    t = 0
    for t in range(1, max_sweeps + 1):
        Q = Pt[:, None] - P.T                       # Q[i, j] = P~_i - P_ji
        Qok = np.where(off, Q, 1.0)
        if not (np.all(np.isfinite(Qok)) and np.all(Qok > 0.0)):
            status = DIVERGED
            t -= 1
            break
        Pn = np.where(off, -A2 / Qok, 0.0)
        En = np.where(off, -Aoff * (S[:, None] - E.T) / Qok, 0.0)
        P, E = Pn, En
        Pt = np.diag(A) + P.sum(axis=0)
        S = b + E.sum(axis=0)
        if not (np.all(np.isfinite(Pt)) and np.all(Pt > 0.0) and np.all(np.isfinite(S))):
            status = DIVERGED
            break
        new = S / Pt
        d = float(np.max(np.abs(new - alpha)))
        alpha = new
        deltas.append(d)
        if keep_trajectory:
            traj.append(alpha.copy())
        if d <= tol_abs + tol_rel * float(np.max(np.abs(alpha))):
            status = CONVERGED
            break
    return GabpResult(alpha, Pt, t, status, deltas, traj)


def svm_alpha_labels_folded(Kp, y, C, mode=DIAG_DOMINANT_ROW, delta=0.1, **kw):
    """Solve (K' + W) g = y and return alpha = y * g.

    Because A = Y (K' + W) Y and Y^2 = I, GaBP on (K' + W, b = y) produces
    the iterates of GaBP on (A, b = 1) up to exact sign flips; this routine
    exists so a test can check that identity bitwise.
    """
    W = weight_diagonal(Kp, C, mode, delta)
    y = np.asarray(y, dtype=np.float64)
    r = gabp_solve(W, y, **kw)
    r.alpha = y * r.alpha
    if r.trajectory is not None:
        r.trajectory = [y * a for a in r.trajectory]
    return r


# --------------------------------------------------------------------------
# Stateless (truncated) messages: no per-edge state, only aggregate history
# --------------------------------------------------------------------------

def gabp_solve_stateless(A, b, depth: int, sweeps: int):
    """Synchronous GaBP where each sweep's messages are rebuilt from the
    history of aggregates instead of stored messages.

    The message i -> j at sweep t depends on the stored state only through
    the reverse message j -> i at sweep t-1, which in turn depends on
    i -> j at t-2, and so on down to the all-zero messages of sweep 0.
    Unrolling `depth` levels and replacing the message at level t-depth by
    zero reproduces the stored recursion exactly while t <= depth.
    Returns the list alpha^1 .. alpha^sweeps.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    off = ~np.eye(n, dtype=bool)
    Aoff = np.where(off, A, 0.0)
    hist_P = [np.diag(A).copy()]            # P~^0, P~^1, ...
    hist_S = [b.copy()]
    out = []
    for t in range(1, sweeps + 1):
        lo = max(1, t - depth + 1)           # first sweep rebuilt from zero state
        # level s: messages of sweep s, computed from sweep s-1 aggregates and
        # the reverse messages of sweep s-1 (zero at the start of the chain)
        P = np.zeros((n, n))
        E = np.zeros((n, n))
        for s in range(lo, t + 1):
            Pt, S = hist_P[s - 1], hist_S[s - 1]
            Q = np.where(off, Pt[:, None] - P.T, 1.0)
            Pn = np.where(off, -Aoff * Aoff / Q, 0.0)
            En = np.where(off, -Aoff * (S[:, None] - E.T) / Q, 0.0)
            P, E = Pn, En
        hist_P.append(np.diag(A) + P.sum(axis=0))
        hist_S.append(b + E.sum(axis=0))
        out.append(hist_S[-1] / hist_P[-1])
    return out


# --------------------------------------------------------------------------
# Grouped (block Gauss-Seidel) schedule
# --------------------------------------------------------------------------
#
# Algorithm 2 leaves the message schedule open, and the section on
# asynchronous settings reports faster convergence when messages do not wait
# for a global round.  The deterministic schedule used here splits the nodes
# into ordered groups; a sweep visits the groups in order, and the visit of
# group g recomputes every message INTO a node of g from the current
# aggregates and reverse messages (messages inside g see each other's
# previous values), then refreshes the aggregates of g.  One group is the
# synchronous schedule.


def gabp_solve_grouped(A, b, groups, max_sweeps: int = 1000, tol_abs: float = 0.0,
                       tol_rel: float = 1e-12, keep_trajectory: bool = False) -> GabpResult:
    """Grouped schedule with stored messages (information form).  `groups`
    is a list of index arrays partitioning 0..n-1, visited in list order.
    Stop rule and failure flags as gabp_solve, tested after each sweep."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    off = ~np.eye(n, dtype=bool)
    Aoff = np.where(off, A, 0.0)
    A2 = Aoff * Aoff
    P = np.zeros((n, n))          # P[i, j]: message i -> j
    E = np.zeros((n, n))
    Pt = np.diag(A).copy()
    S = b.copy()
    alpha = S / Pt
    traj = [alpha.copy()] if keep_trajectory else None
    deltas = []
    status = NOT_CONVERGED
    t = 0
    for t in range(1, max_sweeps + 1):
        bad = False
        for g in groups:
            g = np.asarray(g)
            # Q[i, j] = P~_i - P_ji for the targets j in g
            Q = Pt[:, None] - P[g, :].T
            Qok = np.where(off[:, g], Q, 1.0)
            if not (np.all(np.isfinite(Qok)) and np.all(Qok > 0.0)):
                bad = True
                break
            Pn = np.where(off[:, g], -A2[:, g] / Qok, 0.0)
            En = np.where(off[:, g], -Aoff[:, g] * (S[:, None] - E[g, :].T) / Qok, 0.0)
            P[:, g] = Pn
            E[:, g] = En
            Pt[g] = np.diag(A)[g] + P[:, g].sum(axis=0)
            S[g] = b[g] + E[:, g].sum(axis=0)
        if bad:
            status = DIVERGED
            t -= 1
            break
        if not (np.all(np.isfinite(Pt)) and np.all(Pt > 0.0) and np.all(np.isfinite(S))):
            status = DIVERGED
            break
        new = S / Pt
        d = float(np.max(np.abs(new - alpha)))
        alpha = new
        deltas.append(d)
        if keep_trajectory:
            traj.append(alpha.copy())
        if d <= tol_abs + tol_rel * float(np.max(np.abs(alpha))):
            status = CONVERGED
            break
    return GabpResult(alpha, Pt, t, status, deltas, traj)


def gabp_solve_grouped_stateless(A, b, groups, depth: int, sweeps: int):
    """Grouped schedule where each message is rebuilt from the history of
    aggregates instead of stored messages.

    Visits are numbered tau = t G + g (sweep t, group g).  The message s -> d
    computed at visit tau uses the aggregates of s as they stand at tau
    (version = number of visits of s's group before tau) and the reverse
    message d -> s as last computed, i.e. at the latest visit of s's group
    strictly before tau (none: zero).  Following that chain `depth` levels
    and replacing the next reverse message by zero gives the rebuilt
    message; it equals the stored schedule while the chain reaches the zero
    start.  Returns alpha after each of the `sweeps` sweeps."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    G = len(groups)
    grp = np.empty(n, dtype=np.int64)
    for k, g in enumerate(groups):
        grp[np.asarray(g)] = k
    def visits_before(gs, tau):
        # visits u G + gs < tau, u >= 0
        return np.where(tau > gs, (tau - gs + G - 1) // G, 0)

    def last_visit_before(gs, tau):
        v = visits_before(gs, tau)
        return np.where(v > 0, (v - 1) * G + gs, -1)

    # hist_P[k, v], hist_S[k, v]: aggregates of node k at its version v
    hist_P = np.zeros((n, sweeps + 1))
    hist_S = np.zeros((n, sweeps + 1))
    hist_P[:, 0] = np.diag(A)
    hist_S[:, 0] = b

    out = []
    for t in range(sweeps):
        for gi, g in enumerate(groups):
            g = np.asarray(g)
            tau0 = t * G + gi
            # chains for all (source s, target d in g), s != d
            S_idx, D_idx = np.meshgrid(np.arange(n), g, indexing="ij")
            mask = S_idx != D_idx
            src, dst = S_idx[mask], D_idx[mask]
            a = A[src, dst]
            # walk the chain down: level k message goes from x_k to y_k at visit tau_k
            taus, xs, ys = [np.full(src.shape, tau0)], [src], [dst]
            for k in range(1, depth):
                tau_prev = taus[-1]
                x_prev, y_prev = xs[-1], ys[-1]
                # reverse of (x -> y) at tau: (y -> x) at the last visit of grp[x] before tau
                taus.append(np.where(tau_prev >= 0, last_visit_before(grp[x_prev], tau_prev), -1))
                xs.append(y_prev)
                ys.append(x_prev)
            # deepest level's reverse message is zero; undefined visits give zero messages
            Pm = np.zeros(src.shape)
            Em = np.zeros(src.shape)
            for k in range(depth - 1, -1, -1):
                tau_k, x_k = taus[k], xs[k]
                live = tau_k >= 0
                v = np.where(live, visits_before(grp[x_k], np.maximum(tau_k, 0)), 0)
                Pv, Sv = hist_P[x_k, v], hist_S[x_k, v]
                Q = Pv - Pm
                Pn = np.where(live, -a * a / np.where(live, Q, 1.0), 0.0)
                En = np.where(live, -a * (Sv - Em) / np.where(live, Q, 1.0), 0.0)
                Pm, Em = Pn, En
            Pin = np.zeros((n, len(g)))
            Ein = np.zeros((n, len(g)))
            Pin[mask] = Pm
            Ein[mask] = Em
            newP = np.diag(A)[g] + Pin.sum(axis=0)
            newS = b[g] + Ein.sum(axis=0)
            hist_P[g, t + 1] = newP
            hist_S[g, t + 1] = newS
        out.append(hist_S[:, t + 1] / hist_P[:, t + 1])
    return out


# --------------------------------------------------------------------------
# Closed forms, library solves and bounds used as pins
# --------------------------------------------------------------------------

def first_sweep(A, b):
    """Aggregates after one sweep from zero messages:
    P~^1_j = A_jj - sum_{i != j} A_ij^2 / A_ii,
    S^1_j = b_j - sum_{i != j} A_ij b_i / A_ii."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.diag(A)
    Aoff = A - np.diag(d)
    Pt = d - (Aoff ** 2 / d[:, None]).sum(axis=0)
    S = b - (Aoff * (b / d)[:, None]).sum(axis=0)
    return Pt, S


def cholesky_solve(A, b):
    """alpha* = A^-1 b through LAPACK's Cholesky factorisation."""
    L = np.linalg.cholesky(np.asarray(A, dtype=np.float64))
    z = np.linalg.solve(L, np.asarray(b, dtype=np.float64))
    return np.linalg.solve(L.T, z)


def cg_solve(matvec, b, tol: float = 1e-13, max_iter: int = 10000):
    """Plain conjugate gradients for an SPD operator."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    bn = np.sqrt(b @ b)
    for _ in range(max_iter):
        Ap = matvec(p)
        a = rr / (p @ Ap)
        x += a * p
        r -= a * Ap
        rn = r @ r
        if np.sqrt(rn) <= tol * bn:
            break
        p = r + (rn / rr) * p
        rr = rn
    return x


def pcg_solve(matvec, b, diag, tol: float = 1e-13, max_iter: int = 1000, log=None):
    """Conjugate gradients with the Jacobi preconditioner (textbook PCG) for
    an SPD operator given as a function; `diag` is the operator's diagonal.
    Stops when the recursive residual satisfies ||r||_2 <= tol ||b||_2.
    Returns (x, iterations)."""
    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / np.asarray(diag, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    bn = np.sqrt(b @ b)
    it = 0
    for it in range(1, max_iter + 1):
        q = matvec(p)
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        rn = np.sqrt(r @ r)
        if log is not None:
            log(it, rn / bn)
        if rn <= tol * bn:
            break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it


def varah_bound(A, alpha, b):
    """||alpha - A^-1 b||_inf <= ||b - A alpha||_inf / min_i (|A_ii| - r_i)
    for a strictly diagonally dominant A (Varah's bound)."""
    A = np.asarray(A, dtype=np.float64)
    d = np.abs(np.diag(A))
    r = np.abs(A).sum(axis=1) - d
    gap = np.min(d - r)
    if gap <= 0:
        return np.inf
    return float(np.max(np.abs(np.asarray(b) - A @ alpha)) / gap)


def message_contraction(A, sweeps: int):
    """Largest factor |A_ij| / Q_ij with which a reverse message enters the
    next message (Algorithm 2 in information form, Q_ij = P~_i - P_ji), per
    sweep 1 .. sweeps.  The precisions do not depend on b, so only they are
    iterated; sweep t uses the aggregates of sweep t-1 (sweep 0: zero
    messages).  Returns a list of floats (inf once some Q_ij <= 0)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    off = ~np.eye(n, dtype=bool)
    Aoff = np.where(off, A, 0.0)
    P = np.zeros((n, n))
    Pt = np.diag(A).copy()
    out = []
    for _ in range(sweeps):
        Q = np.where(off, Pt[:, None] - P.T, 1.0)
        if not np.all(Q > 0.0):
            out.append(np.inf)
            break
        out.append(float(np.max(np.abs(Aoff) / Q)) if n > 1 else 0.0)
        P = np.where(off, -Aoff * Aoff / Q, 0.0)
        Pt = np.diag(A) + P.sum(axis=0)
    return out


def contraction_bound(A):
    """A-priori bound on message_contraction over every sweep (not in the
    paper; it decides how many levels the stateless form unrolls).

    Messages stay non-positive while every Q > 0, so Q_ij >= P~_i and
    P~_i >= A_ii - sum_k A_ik^2 / min_k P~_k >= A_ii - c_i / m with
    c_i = max_k |A_ik| * sum_{k != i} |A_ik| and m a lower bound of the
    previous aggregates.  m* = min_i of the larger root of m^2 - A_ii m + c_i
    is such a bound for every sweep when every lo_i = A_ii - c_i / m* is at
    least m* (induction from P~^0 = A_ii).  Then |A_ij| / Q_ij <=
    max_k |A_ik| / lo_i.  Returns (m*, rho), rho = inf when the bound fails.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    off = ~np.eye(n, dtype=bool)
    absoff = np.where(off, np.abs(A), 0.0)
    d = np.diag(A)
    rowmax = absoff.max(axis=1) if n > 1 else np.zeros(n)
    c = rowmax * absoff.sum(axis=1)
    disc = d * d - 4.0 * c
    if np.any(disc < 0.0) or np.any(d <= 0.0):
        return 0.0, np.inf
    mstar = float(np.min(0.5 * (d + np.sqrt(disc))))
    lo = d - c / mstar
    if np.any(lo < mstar * (1.0 - 1e-12)):
        return mstar, np.inf
    return mstar, float(np.max(rowmax / lo))


def box_qp_bruteforce(A, C: float):
    """max 1'h - 1/2 h'Ah s.t. 0 <= h <= C, by enumerating the 3^N
    active sets (lower bound, upper bound, free) and keeping the KKT point
    (eqs. dual and cons1, without cons2, which the bias augmentation
    removes).  For SPD A the KKT point is the unique optimum."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    one = np.ones(n)
    best = None
    for state in itertools.product((0, 1, 2), repeat=n):
        state = np.array(state)
        lo, hi, fr = state == 0, state == 1, state == 2
        h = np.zeros(n)
        h[hi] = C
        if fr.any():
            rhs = one[fr] - A[np.ix_(fr, ~fr)] @ h[~fr]
            h[fr] = np.linalg.solve(A[np.ix_(fr, fr)], rhs)
            if np.any(h[fr] < -1e-12) or np.any(h[fr] > C + 1e-12):
                continue
        g = one - A @ h
        if np.any(g[lo] > 1e-10) or np.any(g[hi] < -1e-10):
            continue
        val = one @ h - 0.5 * h @ A @ h
        if best is None or val > best[1]:
            best = (h, val)
    return best[0]


def box_qp_projected_gauss_seidel(A, C: float, tol: float = 1e-15, max_iter: int = 100000):
    """max 1'h - 1/2 h'Ah s.t. 0 <= h <= C by projected Gauss-Seidel
    (coordinate ascent: h_i <- clip((1 - sum_{j != i} A_ij h_j) / A_ii, 0, C)
    in index order), which converges to the unique optimum for SPD A.  For
    sizes beyond the brute force."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    h = np.zeros(n)
    d = np.diag(A)
    for _ in range(max_iter):
        old = h.copy()
        for i in range(n):
            g = 1.0 - A[i] @ h + d[i] * h[i]
            h[i] = min(max(g / d[i], 0.0), C)
        if np.max(np.abs(h - old)) <= tol * max(np.max(np.abs(h)), 1e-300):
            break
    return h


def gabp_solve_box(A, b, C: float, max_sweeps: int = 1000, tol_abs: float = 0.0,
                   tol_rel: float = 1e-12, keep_trajectory: bool = False) -> GabpResult:
    """Algorithm 2 (information form, synchronous) with the box constraint
    0 <= h <= C (eq. cons1) restored, which the paper drops: after every
    aggregate step (and for the initial aggregates) the belief mean
    S_i / P~_i is clipped to [0, C] and the node broadcasts S_i = P~_i times
    the clipped mean, so the next messages see the projected mean.  Not the
    paper's method; its fixed point is compared with the box QP."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    off = ~np.eye(n, dtype=bool)
    Aoff = np.where(off, A, 0.0)
    A2 = Aoff * Aoff
    P = np.zeros((n, n))
    E = np.zeros((n, n))
    Pt = np.diag(A).copy()
    alpha = np.clip(b / Pt, 0.0, C)
    S = Pt * alpha
    traj = [alpha.copy()] if keep_trajectory else None
    deltas = []
    status = NOT_CONVERGED
    t = 0
    for t in range(1, max_sweeps + 1):
        Q = Pt[:, None] - P.T
        Qok = np.where(off, Q, 1.0)
        if not (np.all(np.isfinite(Qok)) and np.all(Qok > 0.0)):
            status = DIVERGED
            t -= 1
            break
        Pn = np.where(off, -A2 / Qok, 0.0)
        En = np.where(off, -Aoff * (S[:, None] - E.T) / Qok, 0.0)
        P, E = Pn, En
        Pt = np.diag(A) + P.sum(axis=0)
        S = b + E.sum(axis=0)
        if not (np.all(np.isfinite(Pt)) and np.all(Pt > 0.0) and np.all(np.isfinite(S))):
            status = DIVERGED
            break
        new = np.clip(S / Pt, 0.0, C)
        S = Pt * new
        d = float(np.max(np.abs(new - alpha)))
        alpha = new
        deltas.append(d)
        if keep_trajectory:
            traj.append(alpha.copy())
        if d <= tol_abs + tol_rel * float(np.max(np.abs(alpha))):
            status = CONVERGED
            break
    return GabpResult(alpha, Pt, t, status, deltas, traj)


def decision_function(Xtr, y, alpha, Xq, gamma: float, lam: float):
    """f(x) = sum_i alpha_i y_i (K(x_i, x) + lam^2) (section "Classification
    Using Support Vector Machines": the sign of f classifies x, with the bias
    carried by the augmentation)."""
    Xtr = np.asarray(Xtr, dtype=np.float64)
    Xq = np.asarray(Xq, dtype=np.float64)
    w = np.asarray(alpha, dtype=np.float64) * np.asarray(y, dtype=np.float64)
    f = np.empty(Xq.shape[0])
    for q in range(Xq.shape[0]):
        d2 = ((Xtr - Xq[q]) ** 2).sum(axis=1)
        f[q] = w @ (np.exp(-gamma * d2) + lam * lam)
    return f


def krr_dual_closed_form(K, y, lam_ridge: float):
    """Kernel ridge regression dual optimum alpha = 2 lam (K + lam I)^-1 y
    (section "Kernel Ridge Regression problem")."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    return 2.0 * lam_ridge * np.linalg.solve(K + lam_ridge * np.eye(n), np.asarray(y, dtype=np.float64))
