"""Pins of the FP64 oracle against things other than itself.

Every check compares the oracle with a closed form, LAPACK, brute force, a
hand-derived example or an exact invariant, chosen so that a dropped term,
a wrong sign, a swapped index or a transposed operand fails at least one.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import gabp_ref as R
from paper_0810_1648_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- kernel --

def test_kernel_closed_form_points():
    X = np.array([[0.0, 0.0], [1.0, 1.0], [3.0, -1.0]], dtype=np.float32)
    g, lam = 0.3, 0.25
    K = R.rbf_augmented_kernel(X, g, lam)
    assert K[0, 0] == pytest.approx(1.0 + lam * lam, abs=0)
    assert K[0, 1] == pytest.approx(np.exp(-g * 2.0) + lam * lam, rel=1e-15)
    assert K[1, 2] == pytest.approx(np.exp(-g * (4.0 + 4.0)) + lam * lam, rel=1e-15)
    assert np.array_equal(K, K.T)


def test_c_kernel_row_closed_form(oracle_c):
    X = np.array([[0.0, 0.0], [1.0, 1.0], [3.0, -1.0]], dtype=np.float32)
    row = oracle_c.kernel_row(X, 0.3, 0.25, 1)
    expect = [np.exp(-0.6) + 0.0625, 1.0625, np.exp(-0.3 * 8.0) + 0.0625]
    np.testing.assert_allclose(row, expect, rtol=1e-15)


def test_diagonal_rules_closed_form():
    D = np.array([[1.0, -0.9, 0.6], [-0.9, 1.0, 0.8], [0.6, 0.8, 1.0]])
    # row sums of |off-diagonal|: r = (1.5, 1.7, 1.4)
    A = R.weight_diagonal(D, 10.0, R.DIAG_DOMINANT_ROW, 0.1)
    np.testing.assert_allclose(np.diag(A), [1.65, 1.87, 1.54], rtol=1e-15)
    A = R.weight_diagonal(D, 0.5, R.DIAG_DOMINANT_ROW, 0.1)
    np.testing.assert_allclose(np.diag(A), [3.0, 3.0, 3.0], rtol=1e-15)
    A = R.weight_diagonal(D, 10.0, R.DIAG_SOFTMARGIN, 0.1)
    np.testing.assert_allclose(np.diag(A), [1.1, 1.1, 1.1], rtol=1e-15)
    A = R.weight_diagonal(D, 10.0, R.DIAG_DOMINANT_UNIFORM, 0.1)
    np.testing.assert_allclose(np.diag(A), [1.87, 1.87, 1.87], rtol=1e-15)
    A = R.weight_diagonal(D, 10.0, R.DIAG_NONE, 0.1)
    np.testing.assert_allclose(np.diag(A), [1.0, 1.0, 1.0], rtol=0)
    assert A[0, 1] == -0.9 and A[2, 1] == 0.8


# ----------------------------------------------------- worked example ----

def _load_chain3():
    rows = {}
    A = b = None
    with open(os.path.join(GOLDEN, "chain3.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "A":
                A = np.array([float(v) for v in tok[1:]]).reshape(3, 3)
            elif tok[0] == "b":
                b = np.array([float(v) for v in tok[1:]])
            else:
                vals = [float(Fraction(v)) for v in tok[1:]]
                rows[int(tok[0])] = (np.array(vals[:3]), np.array(vals[3:]))
    return A, b, rows


def test_chain3_worked_example_numpy():
    A, b, rows = _load_chain3()
    for t, (alpha, pt) in rows.items():
        r = R.gabp_solve(A, b, max_sweeps=t, tol_rel=0.0)
        assert r.sweeps == t or r.status == R.CONVERGED
        np.testing.assert_allclose(r.alpha, alpha, rtol=1e-15)
        np.testing.assert_allclose(r.ptilde, pt, rtol=1e-15)


def test_chain3_worked_example_c(oracle_c):
    A, b, rows = _load_chain3()
    for t, (alpha, pt) in rows.items():
        r = oracle_c.matrix_solve(A, b, max_sweeps=t, tol_rel=0.0)
        np.testing.assert_allclose(r["alpha"], alpha, rtol=1e-15)
        np.testing.assert_allclose(r["ptilde"], pt, rtol=1e-15)


# ------------------------------------------------- algorithm identities --

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_algorithm1_equals_algorithm2(seed):
    """The broadcast rewrite (aggregate minus own term) reproduces the
    per-message exclusion sums of Algorithm 1 sweep by sweep."""
    wl = inputs.make_workload("tiny", n=14, seed=seed)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    a1 = R.gabp_algorithm1(A, b, 8)
    a2 = R.gabp_algorithm2_mean_form(A, b, 8)
    info = R.gabp_solve(A, b, max_sweeps=8, tol_rel=0.0, keep_trajectory=True)
    for t in range(8):
        assert _rel(a2[t], a1[t]) < 1e-13
        assert _rel(info.trajectory[t + 1], a1[t]) < 1e-13


def test_algorithm1_equals_information_form_signed_matrix():
    A = inputs.random_spd_dominant(9, seed=5, margin=0.3)
    b = np.linspace(-1.0, 2.0, 9)
    a1 = R.gabp_algorithm1(A, b, 6)
    info = R.gabp_solve(A, b, max_sweeps=6, tol_rel=0.0, keep_trajectory=True)
    for t in range(6):
        assert _rel(info.trajectory[t + 1], a1[t]) < 1e-13


def test_single_node():
    r = R.gabp_solve(np.array([[2.5]]), np.array([1.0]), max_sweeps=3)
    assert r.alpha[0] == 1.0 / 2.5
    assert r.status == R.CONVERGED


def test_two_nodes_exact_after_one_sweep(oracle_c):
    a11, a12, a22 = 3.0, -1.25, 2.0
    A = np.array([[a11, a12], [a12, a22]])
    b = np.ones(2)
    exact = np.array([(a22 - a12), (a11 - a12)]) / (a11 * a22 - a12 ** 2)
    for res in (R.gabp_solve(A, b, max_sweeps=1, tol_rel=0.0).alpha,
                oracle_c.matrix_solve(A, b, max_sweeps=1, tol_rel=0.0)["alpha"]):
        np.testing.assert_allclose(res, exact, rtol=1e-15)
    r = R.gabp_solve(A, b, max_sweeps=5, tol_rel=0.0, keep_trajectory=True)
    for t in range(1, len(r.trajectory)):
        np.testing.assert_allclose(r.trajectory[t], exact, rtol=1e-15)


def test_first_sweep_closed_form():
    """first_sweep (aggregates after one sweep from zero messages) against
    the hand-worked chain: P~^1 = (15/4, 7/2, 15/4), S^1 = alpha^1 P~^1 =
    (3/4, 1/2, 3/4); then the sweep itself agrees with it on a dense system."""
    A, b, rows = _load_chain3()
    pt, sv = R.first_sweep(A, b)
    np.testing.assert_array_equal(pt, [15 / 4, 7 / 2, 15 / 4])
    np.testing.assert_array_equal(sv, [3 / 4, 1 / 2, 3 / 4])
    np.testing.assert_allclose(sv / pt, rows[1][0], rtol=1e-15)
    A = inputs.random_spd_dominant(12, seed=3)
    b = np.cos(np.arange(12.0))
    pt, sv = R.first_sweep(A, b)
    r = R.gabp_solve(A, b, max_sweeps=1, tol_rel=0.0)
    np.testing.assert_allclose(r.ptilde, pt, rtol=1e-14)
    np.testing.assert_allclose(r.alpha, sv / pt, rtol=1e-14)


@pytest.mark.parametrize("n", [5, 9, 17])
def test_tree_exactness_means_and_precisions(n, oracle_c):
    """On a tree (chain) GaBP is exact after diameter sweeps, for the means
    and for the marginal precisions 1/(A^-1)_ii."""
    A = inputs.chain_matrix(n, seed=n)
    b = np.sin(np.arange(n) + 1.0)
    inv = np.linalg.inv(A)
    r = R.gabp_solve(A, b, max_sweeps=n - 1, tol_rel=0.0)
    np.testing.assert_allclose(r.alpha, inv @ b, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r.ptilde, 1.0 / np.diag(inv), rtol=1e-12)
    c = oracle_c.matrix_solve(A, b, max_sweeps=n - 1, tol_rel=0.0)
    np.testing.assert_allclose(c["alpha"], inv @ b, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(c["ptilde"], 1.0 / np.diag(inv), rtol=1e-12)


# --------------------------------------------------- converged solution --

def test_tiny_workload_fixed_point_is_cholesky(oracle_c):
    wl = inputs.make_workload("tiny")
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    r = R.gabp_solve(A, b, tol_rel=1e-13)
    assert r.status == R.CONVERGED
    assert _rel(r.alpha, exact) < 1e-10
    c = oracle_c.svm_solve(wl.X, wl.y, wl.gamma, wl.C, wl.lam, tol_rel=1e-13)
    assert c["status"] == "converged"
    assert _rel(c["alpha"], exact) < 1e-10
    np.testing.assert_allclose(c["adiag"], np.diag(A), rtol=1e-14)
    # the tiny workload's own stopping rule (absolute 1e-8 on the change)
    r8 = oracle_c.svm_solve(wl.X, wl.y, wl.gamma, wl.C, wl.lam, tol_abs=1e-8, tol_rel=0.0)
    assert r8["status"] == "converged" and np.max(np.abs(r8["alpha"] - exact)) < 1e-7


def test_letter_shape_fixed_point_cg_and_cholesky(oracle_c):
    wl = inputs.make_workload("letter", n=1200)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    cg = R.cg_solve(lambda v: A @ v, b, tol=1e-14)
    assert _rel(cg, exact) < 1e-11
    c = oracle_c.svm_solve(wl.X, wl.y, wl.gamma, wl.C, wl.lam, tol_rel=1e-13)
    assert c["status"] == "converged"
    assert _rel(c["alpha"], exact) < 1e-10


def test_varah_bound_closed_forms():
    """Hand-worked values of varah_bound: (i) A = [[4, 1], [1, 3]], b = 1,
    alpha = 0: residual 1, smallest dominance gap min(4 - 1, 3 - 1) = 2, so
    the bound is 1/2 (the true error is ||A^-1 1||_inf = 3/11); (ii) a
    uniform diagonal d I, where the bound is an equality: |b_i - d a_i| / d =
    |a_i - b_i / d|; (iii) no strict dominance: no bound (+inf)."""
    A = np.array([[4.0, 1.0], [1.0, 3.0]])
    assert R.varah_bound(A, np.zeros(2), np.ones(2)) == 0.5
    assert np.max(np.abs(np.linalg.solve(A, np.ones(2)))) == pytest.approx(3 / 11, rel=1e-15)
    d = 2.5
    a = np.array([0.1, -0.3, 0.7])
    b = np.array([1.0, 2.0, -1.0])
    err = np.max(np.abs(a - b / d))
    assert R.varah_bound(d * np.eye(3), a, b) == pytest.approx(err, rel=1e-15)
    assert R.varah_bound(np.array([[1.0, 1.0], [1.0, 3.0]]), np.zeros(2), np.ones(2)) == np.inf


def test_varah_bound_holds_along_trajectory():
    wl = inputs.make_workload("tiny", n=300)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    r = R.gabp_solve(A, b, max_sweeps=40, tol_rel=0.0, keep_trajectory=True)
    for a in r.trajectory[1:]:
        assert np.max(np.abs(a - exact)) <= R.varah_bound(A, a, b) * (1 + 1e-9) + 1e-15


def test_residual_rows_vanish_at_exact_solution(oracle_c):
    wl = inputs.make_workload("letter", n=700)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    rows = np.array([0, 5, 333, 699])
    res, ad = oracle_c.residual_rows(wl.X, wl.y, wl.gamma, wl.C, wl.lam, exact, rows)
    assert np.max(np.abs(res)) < 1e-10
    np.testing.assert_allclose(ad, np.diag(A)[rows], rtol=1e-14)


# ------------------------------------------------------------ invariants --

def test_label_sign_equivariance_is_bitwise():
    """GaBP on (Y K' Y + W, 1) equals y * GaBP on (K' + W, y) exactly."""
    wl = inputs.make_workload("tiny", n=200, seed=7)
    K = R.rbf_augmented_kernel(wl.X, wl.gamma, wl.lam)
    A = R.weight_diagonal(R.signed_matrix(K, wl.y), wl.C)
    lit = R.gabp_solve(A, np.ones(wl.N), max_sweeps=25, tol_rel=0.0, keep_trajectory=True)
    fold = R.svm_alpha_labels_folded(K, wl.y, wl.C, max_sweeps=25, tol_rel=0.0, keep_trajectory=True)
    for a, c in zip(lit.trajectory, fold.trajectory):
        assert np.array_equal(a, c)


def test_permutation_equivariance():
    wl = inputs.make_workload("tiny", n=150, seed=11)
    perm = np.random.default_rng(0).permutation(wl.N)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    Ap, bp = R.svm_system(wl.X[perm], wl.y[perm], wl.gamma, wl.C, wl.lam)
    r = R.gabp_solve(A, b, max_sweeps=30, tol_rel=0.0)
    rp = R.gabp_solve(Ap, bp, max_sweeps=30, tol_rel=0.0)
    assert _rel(rp.alpha, r.alpha[perm]) < 1e-12


def test_kernel_ridge_regression_closed_form():
    """With a uniform ridge on K', GaBP's y * alpha times 2 lam_r is the
    KRR dual optimum 2 lam_r (K' + lam_r I)^-1 y."""
    wl = inputs.make_workload("tiny", n=120, seed=3)
    K = R.rbf_augmented_kernel(wl.X, wl.gamma, wl.lam)
    lam_r = 1.2 * float(np.max(K.sum(axis=1)))
    A = R.signed_matrix(K, wl.y) + lam_r * np.eye(wl.N)
    r = R.gabp_solve(A, np.ones(wl.N), tol_rel=1e-14)
    krr = R.krr_dual_closed_form(K, wl.y, lam_r)
    assert _rel(2.0 * lam_r * wl.y.astype(np.float64) * r.alpha, krr) < 1e-10


@pytest.mark.parametrize("seed", range(6))
def test_box_qp_bruteforce_matches_interior_solution(seed):
    wl = inputs.make_workload("tiny", n=7, seed=100 + seed)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    r = R.gabp_solve(A, b, tol_rel=1e-14)
    qp = R.box_qp_bruteforce(A, wl.C)
    if np.all(r.alpha > 0) and np.all(r.alpha < wl.C):
        np.testing.assert_allclose(qp, r.alpha, rtol=1e-9, atol=1e-12)
    else:
        # the unconstrained optimum is infeasible: the QP value must then be
        # no better than the unconstrained one
        f = lambda h: h.sum() - 0.5 * h @ A @ h  # noqa: E731
        assert f(qp) <= f(r.alpha) + 1e-12


def test_decision_function_identity_on_training_points():
    """At the fixed point (K' + W)(y*alpha) = y, so on a training point
    f(x_i) = y_i (1 - w_i alpha_i), w_i being the diagonal weight."""
    wl = inputs.make_workload("tiny", n=160, seed=2)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    alpha = R.cholesky_solve(A, b)
    f = R.decision_function(wl.X, wl.y, alpha, wl.X, wl.gamma, wl.lam)
    w = np.diag(A) - (1.0 + wl.lam ** 2)
    np.testing.assert_allclose(f, wl.y.astype(np.float64) * (1.0 - w * alpha), rtol=1e-9, atol=1e-12)
    assert np.mean(np.sign(f) == wl.y) > 0.9


# ------------------------------------------------------------ divergence --

def test_equicorrelated_divergence_and_dominant_convergence(oracle_c):
    """diag 2, off-diagonal 0.5, N = 10 is SPD (lambda_min = 1.5) but has no
    real message fixed point: by symmetry P = -1/4 / (2 + 8 P) has a negative
    discriminant.  Sweep 1 gives P = -1/8, P~ = 2 - 9/8 = 7/8; sweep 2 gives
    P = -1/4 / (7/8 + 1/8) = -1/4 and P~ = 2 - 9/4 = -1/4 <= 0: both oracles
    report divergence at sweep 2."""
    A = inputs.equicorrelated(10, diag=2.0, off=0.5)
    assert np.min(np.linalg.eigvalsh(A)) == pytest.approx(1.5)
    r1 = R.gabp_solve(A, np.ones(10), max_sweeps=1, tol_rel=0.0)
    np.testing.assert_allclose(r1.ptilde, 7 / 8, rtol=1e-15)
    r = R.gabp_solve(A, np.ones(10), max_sweeps=200)
    assert r.status == R.DIVERGED and r.sweeps == 2
    np.testing.assert_allclose(r.ptilde, -1 / 4, rtol=1e-14)
    c = oracle_c.matrix_solve(A, np.ones(10), max_sweeps=200)
    assert c["status"] == "diverged" and c["sweeps"] == 2
    A5 = inputs.equicorrelated(10, diag=5.0, off=0.5)
    exact = np.linalg.solve(A5, np.ones(10))
    r5 = R.gabp_solve(A5, np.ones(10), tol_rel=1e-15, max_sweeps=500)
    assert _rel(r5.alpha, exact) < 1e-13


def test_softmargin_only_diverges_on_dense_rbf():
    wl = inputs.make_workload("tiny")
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam, mode=R.DIAG_SOFTMARGIN)
    r = R.gabp_solve(A, b, max_sweeps=600, tol_abs=1e-8, tol_rel=0.0)
    assert r.status != R.CONVERGED


# ------------------------------------------------------------- stateless --

def test_stateless_exact_while_within_depth_and_bounded_after():
    wl = inputs.make_workload("tiny", n=220, seed=4)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    ref = R.gabp_solve(A, b, max_sweeps=20, tol_rel=0.0, keep_trajectory=True)
    for depth in (3, 6):
        st = R.gabp_solve_stateless(A, b, depth=depth, sweeps=20)
        for t in range(1, depth + 1):
            assert np.array_equal(st[t - 1], ref.trajectory[t])
        errs = [_rel(st[t - 1], ref.trajectory[t]) for t in range(depth + 1, 21)]
        assert max(errs) > 0.0
    # deeper unrolling is closer to the stored recursion
    e3 = _rel(R.gabp_solve_stateless(A, b, 3, 20)[-1], ref.trajectory[20])
    e6 = _rel(R.gabp_solve_stateless(A, b, 6, 20)[-1], ref.trajectory[20])
    assert e6 < e3


def test_message_contraction_closed_forms():
    # two nodes: Q_12 = P~_1 - P_21 = A_11 at every sweep
    a, c, o = 3.0, 5.0, -1.5
    tr = R.message_contraction(np.array([[a, o], [o, c]]), 6)
    assert tr == [max(abs(o) / a, abs(o) / c)] * 6
    # 3-node chain (a tree): sweep 1 divides by the diagonal, from sweep 2 on
    # the cavity precisions of the leaves' neighbours exclude the leaf
    a, b, c, o1, o2 = 2.0, 3.0, 2.5, 0.8, -1.1
    A = np.array([[a, o1, 0.0], [o1, b, o2], [0.0, o2, c]])
    tr = R.message_contraction(A, 5)
    s1 = max(abs(o1) / a, abs(o1) / b, abs(o2) / b, abs(o2) / c)
    s2 = max(abs(o1) / a, abs(o1) / (b - o2 * o2 / c), abs(o2) / (b - o1 * o1 / a), abs(o2) / c)
    assert tr[0] == pytest.approx(s1, rel=1e-15)
    for v in tr[1:]:
        assert v == pytest.approx(s2, rel=1e-15)


def test_contraction_bound_closed_forms():
    # no couplings: nothing is passed on
    assert R.contraction_bound(np.diag([1.0, 2.0, 3.0]))[1] == 0.0
    # two nodes [[a, o], [o, c]]: c_i = o^2, m* = min larger roots, lo_i = A_ii - o^2 / m*
    a, c, o = 3.0, 5.0, 1.0
    m = min((a + np.sqrt(a * a - 4 * o * o)) / 2, (c + np.sqrt(c * c - 4 * o * o)) / 2)
    mstar, rho = R.contraction_bound(np.array([[a, o], [o, c]]))
    assert mstar == pytest.approx(m, rel=1e-15)
    assert rho == pytest.approx(max(o / (a - o * o / m), o / (c - o * o / m)), rel=1e-15)
    # no real root: no bound
    assert R.contraction_bound(np.array([[1.0, 0.9], [0.9, 1.0]]))[1] == np.inf


@pytest.mark.parametrize("case", range(6))
def test_contraction_bound_holds_along_trajectory(case):
    if case < 3:
        A = inputs.random_spd_dominant(60 + 20 * case, seed=80 + case, margin=[0.1, 0.5, 2.0][case])
    else:
        X, y = inputs.blobs(150, 8, 90 + case)
        A, _ = R.svm_system(X, y, [2e-3, 1.0 / 8, 1.0][case - 3], 1.0, 1.0 / 150)
    mstar, rho = R.contraction_bound(A)
    tr = R.message_contraction(A, 40)
    assert np.isfinite(rho) and np.all(np.isfinite(tr))
    assert max(tr) <= rho * (1 + 1e-12), (max(tr), rho)
    # the bound is useful: within a small factor of what the sweeps reach
    assert rho <= 2.0 * max(tr)


# ------------------------------------------------- grouped (Gauss-Seidel) schedule --

def _tiny_system(n=120, seed=3):
    wl = inputs.make_workload("tiny", n=n, seed=seed)
    return R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)


def test_grouped_with_one_group_is_the_synchronous_schedule():
    A, b = _tiny_system()
    n = len(b)
    r1 = R.gabp_solve(A, b, max_sweeps=8, tol_rel=0.0, keep_trajectory=True)
    r2 = R.gabp_solve_grouped(A, b, [np.arange(n)], max_sweeps=8, tol_rel=0.0, keep_trajectory=True)
    for x, y in zip(r1.trajectory, r2.trajectory):
        assert _rel(y, x) <= 1e-15
    s1 = R.gabp_solve_stateless(A, b, 3, 8)
    s2 = R.gabp_solve_grouped_stateless(A, b, [np.arange(n)], 3, 8)
    for x, y in zip(s1, s2):
        assert _rel(y, x) <= 1e-15


def test_grouped_two_nodes_exact_after_one_sweep():
    A = np.array([[3.0, -1.2], [-1.2, 2.0]])
    b = np.array([1.0, 1.0])
    r = R.gabp_solve_grouped(A, b, [np.array([0]), np.array([1])], max_sweeps=1, tol_rel=0.0)
    np.testing.assert_allclose(r.alpha, np.linalg.solve(A, b), rtol=1e-15)


def test_grouped_serial_chain_first_sweep_is_forward_elimination():
    # serial order on a chain: after one sweep the last node holds the exact
    # solution and the exact marginal precision (Gaussian elimination)
    A = inputs.chain_matrix(6, seed=31)
    b = np.linspace(1.0, 2.0, 6)
    r = R.gabp_solve_grouped(A, b, [np.array([k]) for k in range(6)], max_sweeps=1, tol_rel=0.0)
    x = np.linalg.solve(A, b)
    assert r.alpha[5] == pytest.approx(x[5], rel=1e-14)
    assert r.ptilde[5] == pytest.approx(1.0 / np.linalg.inv(A)[5, 5], rel=1e-14)
    # three nodes, written out
    a00, a11, a22, a01, a12 = 2.0, 3.0, 2.5, 0.8, -1.1
    A3 = np.array([[a00, a01, 0.0], [a01, a11, a12], [0.0, a12, a22]])
    b3 = np.array([1.0, 2.0, 3.0])
    r3 = R.gabp_solve_grouped(A3, b3, [np.array([0]), np.array([1]), np.array([2])], max_sweeps=1, tol_rel=0.0)
    p0 = a00 - a01 ** 2 / a11
    s0 = b3[0] - a01 * b3[1] / a11
    p1 = a11 - a01 ** 2 / a00 - a12 ** 2 / a22
    s1 = b3[1] - a01 * b3[0] / a00 - a12 * b3[2] / a22
    q12 = a11 - a01 ** 2 / a00
    p2 = a22 - a12 ** 2 / q12
    s2 = b3[2] - a12 * (b3[1] - a01 * b3[0] / a00) / q12
    np.testing.assert_allclose(r3.ptilde, [p0, p1, p2], rtol=1e-15)
    np.testing.assert_allclose(r3.alpha, [s0 / p0, s1 / p1, s2 / p2], rtol=1e-15)
    assert r3.alpha[2] == pytest.approx(np.linalg.solve(A3, b3)[2], rel=1e-14)


@pytest.mark.parametrize("G", [2, 4, 7])
def test_grouped_fixed_point_is_cholesky_and_comes_sooner(G):
    A, b = _tiny_system(n=300, seed=5)
    groups = np.array_split(np.arange(300), G)
    r = R.gabp_solve_grouped(A, b, groups, max_sweeps=400, tol_rel=1e-13)
    sync = R.gabp_solve(A, b, max_sweeps=400, tol_rel=1e-13)
    assert r.status == R.CONVERGED and sync.status == R.CONVERGED
    assert _rel(r.alpha, R.cholesky_solve(A, b)) <= 1e-10
    assert 3 * r.sweeps <= sync.sweeps, (r.sweeps, sync.sweeps)


def test_grouped_stateless_equals_stored_while_the_chain_reaches_the_start():
    A, b = _tiny_system()
    groups = np.array_split(np.arange(len(b)), 4)
    ref = R.gabp_solve_grouped(A, b, groups, max_sweeps=6, tol_rel=0.0, keep_trajectory=True)
    errs = {}
    for depth in (3, 6, 13):
        st = R.gabp_solve_grouped_stateless(A, b, groups, depth, 6)
        e = [_rel(st[t - 1], ref.trajectory[t]) for t in range(1, 7)]
        # each level reaches back half a sweep: exact through sweep depth // 2
        assert max(e[:depth // 2]) <= 1e-14, (depth, e)
        errs[depth] = e[-1]
    assert errs[3] > errs[6] > errs[13] and errs[13] <= 1e-14


# ------------------------------------------------------------ sparsified kernel --

def test_sparse_kernel_limits():
    X, y = inputs.blobs(60, 5, 61)
    A_dense, b = R.svm_system(X, y, 0.2, 1.0, 1.0 / 60)
    # a threshold below every kernel value keeps every pair: the dense system
    D2 = R.pair_sq_distances(X)
    tau_all = 0.5 * float(np.exp(-0.2 * D2.max()))
    A_sp, _ = R.sparse_svm_system(X, y, 0.2, 1.0, 1.0 / 60, tau_all)
    np.testing.assert_array_equal(A_sp, A_dense)
    # a cut below the smallest distance keeps no pair: diagonal system
    off = D2[~np.eye(60, dtype=bool)]
    tau_none = float(np.exp(-0.2 * 0.5 * off.min()))
    A0, b0 = R.sparse_svm_system(X, y, 0.2, 1.0, 1.0 / 60, tau_none)
    assert np.count_nonzero(A0 - np.diag(np.diag(A0))) == 0
    np.testing.assert_allclose(np.diag(A0), 1.0 + (1.0 / 60) ** 2 + 1.0, rtol=1e-15)
    assert len(R.sparse_edges(X, 0.2, tau_none)) == 0


def test_sparse_edges_brute_force():
    X, _ = inputs.blobs(30, 4, 62)
    gamma, tau = 0.3, 0.05
    cut = -np.log(tau) / gamma
    want = []
    for i in range(30):
        for j in range(i + 1, 30):
            d2 = sum((float(X[i, k]) - float(X[j, k])) ** 2 for k in range(4))
            if d2 <= cut:
                want.append((i, j))
    got = [tuple(e) for e in R.sparse_edges(X, gamma, tau)]
    assert got == want and 0 < len(want) < 30 * 29 // 2


def test_sparse_separated_clusters_decouple():
    # two clusters far apart and a cut between the intra- and inter-cluster
    # distances: the system is block diagonal and each block solves alone
    rng = np.random.default_rng(63)
    Xa = rng.standard_normal((40, 3))
    Xb = rng.standard_normal((35, 3)) + 50.0
    X = np.vstack([Xa, Xb]).astype(np.float32)
    y = np.where(rng.random(75) < 0.5, 1.0, -1.0).astype(np.float32)
    gamma, lam, tau = 0.05, 1.0 / 75, 1e-6
    A, b = R.sparse_svm_system(X, y, gamma, 1.0, lam, tau)
    assert np.count_nonzero(A[:40, 40:]) == 0
    full = R.cholesky_solve(A, b)
    Aa, ba = R.sparse_svm_system(X[:40], y[:40], gamma, 1.0, lam, tau)
    Ab, bb = R.sparse_svm_system(X[40:], y[40:], gamma, 1.0, lam, tau)
    np.testing.assert_allclose(full[:40], R.cholesky_solve(Aa, ba), rtol=1e-12)
    np.testing.assert_allclose(full[40:], R.cholesky_solve(Ab, bb), rtol=1e-12)
    r = R.gabp_solve(A, b, max_sweeps=500, tol_rel=1e-13)
    assert r.status == R.CONVERGED and _rel(r.alpha, full) <= 1e-10


def test_sparse_threshold_gap():
    X, _ = inputs.blobs(200, 6, 64)
    tau, cut = R.sparse_tau_with_gap(X, 0.1, mean_degree=12)
    D2 = R.pair_sq_distances(X)[np.triu_indices(200, k=1)]
    assert np.min(np.abs(D2 - cut)) > 1e-3 * cut
    assert tau == pytest.approx(np.exp(-0.1 * cut), rel=1e-15)
    deg = 2 * np.count_nonzero(D2 <= cut) / 200
    assert 6 <= deg <= 24


# ----------------------------------------------------------- box-projected sweep --

def _obj(A, h):
    return float(np.sum(h) - 0.5 * h @ A @ h)


def test_box_projection_with_a_loose_box_is_plain_gabp():
    # a dominant matrix with non-positive couplings keeps every iterate
    # positive, so a box above the solution never clips
    A = -np.abs(inputs.random_spd_dominant(150, seed=9, margin=0.5))
    A[np.diag_indices(150)] *= -1.0
    b = np.ones(150)
    r = R.gabp_solve(A, b, max_sweeps=12, tol_rel=0.0, keep_trajectory=True)
    C = 10.0 * float(np.max(np.abs(R.cholesky_solve(A, b))))
    rb = R.gabp_solve_box(A, b, C, max_sweeps=12, tol_rel=0.0, keep_trajectory=True)
    # while no mean leaves the box the sweeps agree up to the rounding of
    # S = P~ (S / P~)
    checked = 0
    for t in range(13):
        if not np.all(r.trajectory[t] > 0.0):
            break
        assert _rel(rb.trajectory[t], r.trajectory[t]) <= 1e-13
        checked += 1
    assert checked == 13


@pytest.mark.parametrize("case", range(12))
def test_box_projected_fixed_point_is_the_box_qp_optimum(case):
    # brute force over the 3^N active sets (N = 7) pins the projected sweep
    rng = np.random.default_rng(200 + case)
    X, y = inputs.blobs(7, 3, 300 + case)
    C = float(rng.choice([0.05, 0.2, 1.0]))
    A, b = R.svm_system(X, y, 0.5, C, 1.0 / 7)
    h = R.box_qp_bruteforce(A, C)
    r = R.gabp_solve_box(A, b, C, max_sweeps=2000, tol_rel=1e-14)
    assert r.status == R.CONVERGED
    np.testing.assert_allclose(r.alpha, h, rtol=0, atol=1e-12 * max(1.0, float(np.max(h))))
    assert abs(_obj(A, r.alpha) - _obj(A, h)) <= 1e-12 * abs(_obj(A, h))


def test_projected_gauss_seidel_pins():
    # against brute force on small systems, and the KKT conditions at size
    for case in range(4):
        X, y = inputs.blobs(8, 3, 400 + case)
        A, _ = R.svm_system(X, y, 0.5, 0.1, 1.0 / 8)
        np.testing.assert_allclose(R.box_qp_projected_gauss_seidel(A, 0.1), R.box_qp_bruteforce(A, 0.1),
                                   atol=1e-12)
    X, y = inputs.blobs(300, 5, 410)
    A, _ = R.svm_system(X, y, 0.2, 0.01, 1.0 / 300)
    h = R.box_qp_projected_gauss_seidel(A, 0.01)
    g = 1.0 - A @ h
    lo, hi = h <= 0.0, h >= 0.01
    fr = ~(lo | hi)
    assert hi.sum() > 0 and fr.sum() > 0
    assert np.max(np.abs(g[fr])) <= 1e-10 and np.all(g[lo] <= 1e-10) and np.all(g[hi] >= -1e-10)
    r = R.gabp_solve_box(A, np.ones(300), 0.01, max_sweeps=2000, tol_rel=1e-14)
    assert r.status == R.CONVERGED and np.max(np.abs(r.alpha - h)) <= 1e-12


# ------------------------------------------------ matrix-free and stateless C forms --

def test_c_matvec_is_the_dense_product(oracle_c):
    """The matrix-free product (rows rebuilt from the features) equals A v
    with A built densely by the NumPy oracle, and its diagonal is A's."""
    for name, n in (("letter", 700), ("covertype", 900), ("tiny", 333)):
        wl = inputs.make_workload(name, n=n)
        A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam, delta=wl.delta)
        v = np.random.default_rng(n).standard_normal(n)
        out, ad = oracle_c.svm_matvec(wl.X, wl.y, wl.gamma, wl.C, wl.lam, v, delta=wl.delta, want_diag=True)
        ref = A @ v
        assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(A) @ np.abs(v))
        np.testing.assert_allclose(ad, np.diag(A), rtol=1e-14)


@pytest.mark.parametrize("name,n", [("letter", 1500), ("covertype", 2000), ("tiny", 500)])
def test_pcg_reference_is_cholesky(oracle_c, name, n):
    """The reference solution of the large workloads (Jacobi-preconditioned
    CG on the matrix-free product) against LAPACK Cholesky."""
    wl = inputs.make_workload(name, n=n)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam, delta=wl.delta)
    exact = R.cholesky_solve(A, b)
    mv = lambda v: oracle_c.svm_matvec(wl.X, wl.y, wl.gamma, wl.C, wl.lam, v, delta=wl.delta)  # noqa: E731
    x, it = R.pcg_solve(mv, b, np.diag(A), tol=1e-13)
    assert it < 60
    assert _rel(x, exact) <= 1e-12
    # the same on the dense matrix, and plain CG agrees
    x2, _ = R.pcg_solve(lambda v: A @ v, b, np.diag(A), tol=1e-13)
    assert _rel(x2, exact) <= 1e-12
    assert _rel(R.cg_solve(lambda v: A @ v, b, tol=1e-14), exact) <= 1e-11


def test_pcg_closed_form_two_by_two():
    """CG solves an n x n SPD system in at most n steps: A = [[4, 1], [1, 3]],
    b = 1 gives (2/11, 3/11) after two iterations."""
    A = np.array([[4.0, 1.0], [1.0, 3.0]])
    x, it = R.pcg_solve(lambda v: A @ v, np.ones(2), np.diag(A), tol=1e-15)
    assert it <= 2
    np.testing.assert_allclose(x, [2 / 11, 3 / 11], rtol=1e-15)


@pytest.mark.parametrize("depth", [1, 3, 5])
def test_c_stateless_equals_stored_while_within_depth(oracle_c, depth):
    """The C oracle's stateless form reproduces its stored-message sweep bit
    for bit while t <= depth (the chain reaches the zero messages of sweep
    0), and the NumPy oracle's stateless form after that."""
    wl = inputs.make_workload("tiny", n=260, seed=7)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    T = depth + 4
    c = oracle_c.stateless_matrix(A, b, depth, T)
    assert c["status"] == "converged"
    py = R.gabp_solve_stateless(A, b, depth, T)
    for t in range(1, T + 1):
        if t <= depth:
            stored = oracle_c.matrix_solve(A, b, max_sweeps=t, tol_rel=0.0)["alpha"]
            assert np.array_equal(c["trajectory"][t - 1], stored), t
        assert _rel(c["trajectory"][t - 1], py[t - 1]) <= 1e-13


def test_c_stateless_rows_are_the_sweep_of_the_features(oracle_c):
    """One stateless sweep for listed rows, each row of A rebuilt from the
    features, equals the explicit-matrix form: sweep 1 against the first-
    sweep closed form, sweep 2 (history P~^0, P~^1) against the trajectory."""
    wl = inputs.make_workload("covertype", n=600, seed=11)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    ad = np.diag(A).copy()
    pt1, s1 = R.first_sweep(A, b)
    rows = np.array([0, 7, 255, 256, 599])
    r1 = oracle_c.stateless_rows(wl.X, wl.y, wl.gamma, wl.lam, ad, ad[None, :], b[None, :], 1, 3, rows)
    assert r1["status"] == "converged"
    np.testing.assert_allclose(r1["P"], pt1[rows], rtol=1e-13)
    np.testing.assert_allclose(r1["S"], s1[rows], rtol=1e-12)
    r2 = oracle_c.stateless_rows(wl.X, wl.y, wl.gamma, wl.lam, ad, np.stack([ad, pt1]), np.stack([b, s1]),
                                 2, 3, rows)
    ref = oracle_c.stateless_matrix(A, b, 3, 2)["trajectory"][1]
    np.testing.assert_allclose(r2["S"] / r2["P"], ref[rows], rtol=1e-12)
