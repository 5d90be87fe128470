"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance for FP64 and FP32 results (stated as a number):
    ||alpha - alpha_ref||_inf <= 1e-5 * ||alpha_ref||_inf,
at convergence and for each of the first 20 sweeps.  The MIXED path is
reported per result and held to the bounds derived for its Gram: the
default three-term BF16 split (BF16x6) reaches the same 1e-5; the two-term
split (BF16x3) and a single BF16 product perturb the features by about
2^-17 and 2^-9 relative, and are held to 1e-4 and 1e-2 (their measured
errors are about 2e-5 and 2e-3).
"""
import numpy as np
import pytest

from oracle import gabp_ref as R
from paper_0810_1648_amd import gabp, inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _rel(a, ref):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(ref))) / np.max(np.abs(ref)))


def run(torch, wl, device=True, **kw):
    params = dict(gamma=wl.gamma, C=wl.C, lambda_aug=wl.lam, diag_delta=wl.delta,
                  precision=wl.precision, tol_abs=wl.tol_abs, tol_rel=wl.tol_rel)
    params.update(kw)
    print(f"[case] {wl.name} N={wl.N} m={wl.m} {params}", flush=True)
    s = gabp.GabpSVM(**params)
    if device:
        X = torch.from_numpy(wl.X).cuda()
        y = torch.from_numpy(wl.y).cuda()
        st = s.solve(X, y)
        torch.cuda.synchronize()
    else:
        st = s.solve(wl.X, wl.y)
    return s, st


def oracle_traj(wl, sweeps):
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam, delta=wl.delta)
    r = R.gabp_solve(A, b, max_sweeps=sweeps, tol_rel=0.0, keep_trajectory=True)
    return A, r


# ------------------------------------------------------- converged results --

def test_fp64_tiny_workload_matches_oracle(torch, oracle_c):
    wl = inputs.make_workload("tiny")
    s, st = run(torch, wl)
    ref = oracle_c.svm_solve(wl.X, wl.y, wl.gamma, wl.C, wl.lam, tol_abs=wl.tol_abs, tol_rel=0.0)
    assert st == gabp.OK and s.reason() == "converged"
    # the stop rule fires at the oracle's sweep: the oracle's changes around
    # it are far from the threshold compared with the FP64 rounding
    # differences (about 1e-13 relative), so the sweep count is exact
    d = ref["deltas"]
    assert d[-1] <= wl.tol_abs < d[-2] and min(wl.tol_abs - d[-1], d[-2] - wl.tol_abs) > 1e-6 * wl.tol_abs
    assert s.sweeps() == ref["sweeps"]
    np.testing.assert_allclose(s.trace(), d, rtol=0, atol=1e-12)
    err = _rel(s.alpha(), ref["alpha"])
    print(f"fp64 tiny: sweeps {s.sweeps()} (oracle {ref['sweeps']}), rel err {err:.2e}")
    assert err <= TOL
    np.testing.assert_allclose(s.adiag(), ref["adiag"], rtol=1e-12)
    np.testing.assert_allclose(s.ptilde(), ref["ptilde"], rtol=1e-9)


@pytest.mark.parametrize("n", [255, 256, 257, 1100])
def test_fp32_letter_shape_matches_cholesky(torch, n):
    wl = inputs.make_workload("letter", n=n)
    s, st = run(torch, wl, precision="fp32")
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    err = _rel(s.alpha(), exact)
    print(f"fp32 letter N={n}: status {st} reason {s.reason()} sweeps {s.sweeps()} rel err {err:.2e}")
    assert st == gabp.OK
    assert err <= TOL
    np.testing.assert_allclose(s.adiag(), np.diag(A), rtol=2e-6)


@pytest.mark.parametrize("gram,bound", [("bf16x6", TOL), ("bf16x3", 1e-4), ("bf16", 1e-2)])
def test_mixed_covertype_shape(torch, gram, bound):
    wl = inputs.make_workload("covertype", n=1500)
    s, st = run(torch, wl, precision="mixed", gram=gram)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    err = _rel(s.alpha(), exact)
    print(f"mixed/{gram} covertype N=1500: status {st} sweeps {s.sweeps()} rel err vs FP64 {err:.2e}")
    assert st == gabp.OK
    assert err <= bound


# ---------------------------------------------------- sweep-by-sweep parity --

@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_first_twenty_sweeps(torch, prec):
    wl = inputs.make_workload("tiny", n=700, seed=9)
    A, ref = oracle_traj(wl, 20)
    for t in (1, 2, 3, 5, 8, 13, 20):
        s, st = run(torch, wl, precision=prec, max_sweeps=t, tol_abs=0.0,
                    tol_rel=0.0, stagnation_window=0)
        assert st == gabp.E_NOT_CONVERGED and s.sweeps() == t
        err = _rel(s.alpha(), ref.trajectory[t])
        assert err <= TOL, (prec, t, err)
        s.close()


def test_max_sweeps_one_is_first_sweep_closed_form(torch):
    wl = inputs.make_workload("tiny", n=300, seed=3)
    s, st = run(torch, wl, max_sweeps=1, tol_abs=0.0, tol_rel=0.0)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    n = wl.N
    pt, sv = R.first_sweep(A, b)
    assert st == gabp.E_NOT_CONVERGED and s.reason() == "max_sweeps" and s.sweeps() == 1
    np.testing.assert_allclose(s.alpha(), sv / pt, rtol=1e-12)
    np.testing.assert_allclose(s.ptilde(), pt, rtol=1e-12)
    assert n == len(s.alpha())


# ------------------------------------------------- chosen matrices (K' given) --

def run_kernel(torch, K, y=None, **kw):
    n = K.shape[0]
    y = np.ones(n, np.float32) if y is None else y
    params = dict(kernel="precomputed", precision="fp64", diag_mode="none", tol_rel=1e-14,
                  stagnation_window=0)
    params.update(kw)
    print(f"[case] kernel N={n} {params}", flush=True)
    s = gabp.GabpSVM(**params)
    st = s.solve_kernel(torch.from_numpy(np.ascontiguousarray(K)).cuda(), torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    return s, st


@pytest.mark.parametrize("n", [17, 300])
def test_tree_exact_means_and_precisions(torch, n):
    A = inputs.chain_matrix(n, seed=n)
    inv = np.linalg.inv(A)
    s, st = run_kernel(torch, A, max_sweeps=n - 1, tol_rel=0.0)
    np.testing.assert_allclose(s.alpha(), inv @ np.ones(n), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(s.ptilde(), 1.0 / np.diag(inv), rtol=1e-11)


def test_two_nodes_exact(torch):
    A = np.array([[3.0, -1.25], [-1.25, 2.0]])
    s, st = run_kernel(torch, A, max_sweeps=1, tol_rel=0.0)
    exact = np.array([2.0 + 1.25, 3.0 + 1.25]) / (6.0 - 1.25 ** 2)
    np.testing.assert_allclose(s.alpha(), exact, rtol=1e-15)


def test_single_point(torch):
    s, st = run_kernel(torch, np.array([[2.5]]))
    assert st == gabp.OK
    assert s.alpha()[0] == 1.0 / 2.5


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_equicorrelated_diverges(torch, prec):
    """No real message fixed point: the aggregate precision reaches -1/4 at
    sweep 2 (hand-derived; both oracles report divergence there), so the
    solver must flag divergence at that sweep in every precision."""
    A = inputs.equicorrelated(10, 2.0, 0.5)
    ref = R.gabp_solve(A, np.ones(10), max_sweeps=200)
    assert ref.status == R.DIVERGED and ref.sweeps == 2
    s, st = run_kernel(torch, A, precision=prec, max_sweeps=200, tol_rel=1e-12)
    print(f"equicorrelated {prec}: status {st} reason {s.reason()} sweeps {s.sweeps()}")
    assert st == gabp.E_DIVERGED and s.reason() == "diverged" and s.sweeps() == ref.sweeps
    if prec != "fp64":
        return
    s2, st2 = run_kernel(torch, inputs.equicorrelated(10, 5.0, 0.5), max_sweeps=500)
    np.testing.assert_allclose(s2.alpha(), np.linalg.solve(inputs.equicorrelated(10, 5.0, 0.5), np.ones(10)),
                               rtol=1e-13)


def test_signed_kernel_matrix_fp32(torch):
    A = inputs.random_spd_dominant(600, seed=2, margin=0.2)
    s, st = run_kernel(torch, A, precision="fp32", tol_rel=1e-7, stagnation_window=10)
    assert st == gabp.OK
    assert _rel(s.alpha(), np.linalg.solve(A, np.ones(600))) <= TOL


# --------------------------------------------------------------- behaviour --

def test_invalid_inputs_rejected(torch):
    wl = inputs.make_workload("tiny", n=64)
    X = wl.X.copy()
    X[3, 1] = np.nan
    for dev in (False, True):
        s = gabp.GabpSVM(gamma=wl.gamma)
        with pytest.raises(gabp.GabpError) as e:
            if dev:
                s.solve(torch.from_numpy(X).cuda(), torch.from_numpy(wl.y).cuda())
            else:
                s.solve(X, wl.y)
        assert e.value.status == gabp.E_INVALID
        y = wl.y.copy()
        y[0] = 0.0
        with pytest.raises(gabp.GabpError):
            if dev:
                s.solve(torch.from_numpy(wl.X).cuda(), torch.from_numpy(y).cuda())
            else:
                s.solve(wl.X, y)


def test_host_device_inputs_and_polling_are_bitwise_identical(torch):
    wl = inputs.make_workload("letter", n=900)
    a, _ = run(torch, wl, precision="fp32", device=True, check_every=8)
    b, _ = run(torch, wl, precision="fp32", device=False, check_every=1)
    c, _ = run(torch, wl, precision="fp32", device=True, check_every=5)
    assert np.array_equal(a.alpha(), b.alpha()) and np.array_equal(a.alpha(), c.alpha())
    assert a.sweeps() == b.sweeps() == c.sweeps()


def test_kernel_entries_match_oracle(torch, oracle_c):
    wl = inputs.make_workload("letter", n=700)
    rng = np.random.default_rng(0)
    rows = rng.integers(0, wl.N, 200)
    cols = (rows + 1 + rng.integers(0, wl.N - 1, 200)) % wl.N
    ref = np.array([oracle_c.kernel_row(wl.X, wl.gamma, wl.lam, int(i))[j] for i, j in zip(rows, cols)])
    for prec, gram, bound in (("fp64", "auto", 1e-13), ("fp32", "auto", 2e-6), ("mixed", "bf16x6", 2e-6),
                              ("mixed", "bf16x3", 1e-4), ("mixed", "bf16", 2e-2)):
        s, _ = run(torch, wl, precision=prec, gram=gram, max_sweeps=1)
        got = s.kernel_entries(rows, cols)
        err = float(np.max(np.abs(got - ref) / ref))
        print(f"K' entries {prec}/{gram}: max rel err {err:.2e}")
        assert err <= bound


def test_predict_matches_oracle_decision_function(torch):
    wl = inputs.make_workload("tiny", n=400, seed=8)
    s, st = run(torch, wl, precision="fp64")
    Xq = inputs.blobs(50, wl.m, 77)[0]
    f = s.predict(Xq)
    ref = R.decision_function(wl.X, wl.y, s.alpha(), Xq, wl.gamma, wl.lam)
    np.testing.assert_allclose(f, ref, rtol=1e-10, atol=1e-12)
    fd = s.predict(torch.from_numpy(Xq).cuda()).cpu().numpy()
    np.testing.assert_allclose(fd, f, rtol=0, atol=0)
    # bias query: lambda^2 sum alpha y
    assert s.bias() == pytest.approx(wl.lam ** 2 * float(np.sum(s.alpha() * wl.y)), rel=1e-12)


def test_box_clip_and_sv_mask(torch):
    wl = inputs.make_workload("tiny", n=300, seed=12)
    s, _ = run(torch, wl, box_mode="clip_output", C=0.05, sv_tau=0.0)
    a = s.alpha()
    assert a.min() >= 0.0 and a.max() <= 0.05
    assert s.sv_count() == int(np.sum(a > 0.0)) and np.array_equal(s.sv_mask(), a > 0.0)


# ------------------------------------------- K' recomputed / stateless edges --

def test_recompute_matches_materialised(torch):
    # FP32 Gram: both forms compute K' by the same formula (row sums equal to
    # rounding order); BF16 splits: the recomputed bands take the exponent
    # straight from the Gram of augmented rows, the plane forms the distance
    # on the VALU, each within FP32 rounding of the kernel value
    for prec, n, rtol in (("fp32", 900, 1e-12), ("mixed", 700, 1e-6)):
        wl = inputs.make_workload("covertype", n=n, seed=21)
        a, _ = run(torch, wl, precision=prec, kstore="materialise", edge_state="stored")
        b, _ = run(torch, wl, precision=prec, kstore="recompute", edge_state="stored")
        assert b.plan()["kstore"] == gabp.KSTORE["recompute"]
        np.testing.assert_allclose(b.adiag(), a.adiag(), rtol=rtol)
        err = _rel(b.alpha(), a.alpha())
        print(f"recompute vs materialise {prec}: rel diff {err:.2e}, sweeps {b.sweeps()} vs {a.sweeps()}")
        assert err <= 1e-6


def _chunk_rule(prec, levels, ser):
    # the synchronous stateless sweeps that run over 2 x 2 chunks of tiles:
    # FP32 partial sums (FP32, or MIXED with series reciprocals) and a
    # recursion small enough for the chunk's sums
    fp32_partials = prec == "fp32" or (prec == "mixed" and ser > 0)
    return fp32_partials and (levels == 1 or (levels == 2 and ser > 0) or (levels == 3 and ser == 3))


@pytest.mark.parametrize("prec,n,depth,gamma", [("mixed", 200, 3, None), ("mixed", 700, 3, None),
                                                ("fp32", 1100, 2, None), ("mixed", 1500, 1, None),
                                                ("fp32", 900, 1, None), ("fp32", 2900, 3, None),
                                                ("mixed", 1500, 3, 2.0), ("fp32", 1100, 3, 2.0)])
def test_chunked_sweep_matches_oracle_trajectory(torch, prec, n, depth, gamma):
    # one to twelve blocks (odd and even counts, a ragged last block): the
    # sweep over 2 x 2 tile chunks (asked for at these sizes, which take
    # single tiles by default) follows the oracle's stateless recursion sweep
    # by sweep; gamma = 2 makes the system contract enough for series form 3
    # at three levels
    wl = inputs.make_workload("covertype", n=n, seed=31)
    g = wl.gamma if gamma is None else gamma
    A, b = R.svm_system(wl.X, wl.y, g, wl.C, wl.lam, delta=wl.delta)
    ref = R.gabp_solve_stateless(A, b, depth=depth, sweeps=12)
    for t in (1, depth, depth + 1, 12):
        s, st = run(torch, wl, precision=prec, edge_state="stateless", kstore="materialise", stateless_depth=depth,
                    max_sweeps=t, tol_abs=0.0, tol_rel=0.0, stagnation_window=0, tile_chunk=2, gamma=g)
        p = s.plan()
        assert p["tile_chunk"] == (2 if _chunk_rule(prec, depth, p["series_reciprocal"]) else 1), p
        # a strongly contracting system can reach its FP32 fixed point (no
        # change at all) before sweep t, which stops the solve there
        assert s.sweeps() == t or (s.sweeps() < t and s.reason() == "converged"), (s.sweeps(), t, s.reason())
        err = _rel(s.alpha(), ref[s.sweeps() - 1])
        assert err <= TOL, (prec, n, depth, t, p["tile_chunk"], err)
    print(f"{prec} n={n} depth={depth}: series form {p['series_reciprocal']}, tile chunk {p['tile_chunk']}")
    if gamma is not None:
        assert p["series_reciprocal"] == 3 and p["tile_chunk"] == 2, p


@pytest.mark.parametrize("prec,depth", [("fp32", 1), ("fp32", 2), ("mixed", 2)])
def test_chunked_sweep_on_a_given_matrix(torch, prec, depth):
    # a given dense system (no RBF; three blocks) through the sweep over
    # 2 x 2 tile chunks: the oracle's truncated stateless recursion, and the
    # same result as single tiles up to the order of the FP32 sums
    A = inputs.random_spd_dominant(700, seed=41, margin=0.5)
    ref = R.gabp_solve_stateless(A, np.ones(700), depth=depth, sweeps=10)
    got = {}
    for tc in (1, 2):
        s, st = run_kernel(torch, A, precision=prec, edge_state="stateless", stateless_depth=depth,
                           kstore="materialise", max_sweeps=10, tol_rel=0.0, tile_chunk=tc)
        p = s.plan()
        # a short recursion may reach its FP32 fixed point (no change at all)
        # before the tenth sweep, which stops the solve there
        assert 5 <= s.sweeps() <= 10
        want = 2 if (tc == 2 and _chunk_rule(prec, depth, p["series_reciprocal"])) else 1
        assert p["tile_chunk"] == want, p
        got[tc] = s.alpha()
        err = _rel(got[tc], ref[s.sweeps() - 1])
        print(f"{prec} depth {depth} tile_chunk {p['tile_chunk']}: rel err {err:.2e}")
        assert err <= TOL, (prec, depth, tc, err)
    assert _rel(got[2], got[1]) <= 1e-6
    if depth == 1:
        assert p["tile_chunk"] == 2


def test_chunking_only_where_the_rule_allows(torch):
    # FP64 plans, stored pair records, the grouped schedule and deeper
    # recursions keep one tile per workgroup even when chunks are asked for;
    # a plan that allows chunks takes them by default only from 4,096 chunks
    # on (not at 900 points), and never with tile_chunk = 1
    wl = inputs.make_workload("covertype", n=900, seed=32)
    for kw in (dict(precision="fp64", edge_state="stateless", stateless_depth=2, tile_chunk=2),
               dict(precision="mixed", edge_state="stored", tile_chunk=2),
               dict(precision="mixed", edge_state="stateless", stateless_depth=2, schedule="grouped", tile_chunk=2),
               dict(precision="mixed", edge_state="stateless", stateless_depth=4, tile_chunk=2),
               dict(precision="fp32", edge_state="stateless", stateless_depth=1),
               dict(precision="fp32", edge_state="stateless", stateless_depth=1, tile_chunk=1)):
        s, st = run(torch, wl, kstore="materialise", **kw)
        assert s.plan()["tile_chunk"] == 1, (kw, s.plan())
    s, st = run(torch, wl, kstore="materialise", precision="fp32", edge_state="stateless", stateless_depth=1,
                tile_chunk=2)
    assert s.plan()["tile_chunk"] == 2, s.plan()


@pytest.mark.parametrize("depth", [1, 3, 6])
def test_stateless_matches_oracle_truncated_recursion(torch, depth):
    wl = inputs.make_workload("tiny", n=600, seed=13)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    ref = R.gabp_solve_stateless(A, b, depth=depth, sweeps=12)
    for t in (1, depth, depth + 1, 12):
        for kstore in ("materialise", "recompute"):
            s, st = run(torch, wl, precision="fp64" if kstore == "materialise" else "mixed",
                        edge_state="stateless", kstore=kstore, stateless_depth=depth, max_sweeps=t,
                        tol_abs=0.0, tol_rel=0.0, stagnation_window=0)
            assert s.plan()["edge_state"] == gabp.EDGE["stateless"] and s.sweeps() == t
            err = _rel(s.alpha(), ref[t - 1])
            assert err <= TOL, (depth, t, kstore, err)


def test_stateless_auto_depth_converges_to_solution(torch):
    wl = inputs.make_workload("covertype", n=2600, seed=5)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    for prec, kstore in (("fp32", "materialise"), ("mixed", "materialise"), ("mixed", "recompute"),
                         ("fp32", "recompute")):
        s, st = run(torch, wl, precision=prec, edge_state="stateless", kstore=kstore)
        plan = s.plan()
        err = _rel(s.alpha(), exact)
        print(f"stateless {prec}/{kstore}: depth {plan['stateless_depth']} rho {plan['stateless_rho']:.3e} "
              f"sweeps {s.sweeps()} reason {s.reason()} rel err {err:.2e}")
        assert st == gabp.OK and err <= TOL


def test_plan_follows_memory_budget(torch):
    wl = inputs.make_workload("letter", n=1800)
    s, _ = run(torch, wl, precision="fp32", hbm_budget_bytes=int(42e6))
    p = s.plan()
    assert p["kstore"] == gabp.KSTORE["recompute"] or p["edge_state"] == gabp.EDGE["stateless"]
    assert p["device_bytes"] <= 42e6
    s2 = gabp.GabpSVM(gamma=wl.gamma, precision="fp32", hbm_budget_bytes=1000)
    with pytest.raises(gabp.GabpError) as e:
        s2.solve(wl.X, wl.y)
    assert e.value.status == gabp.E_NOMEM
    s3 = gabp.GabpSVM(gamma=wl.gamma, precision="fp64", kstore="recompute")
    with pytest.raises(gabp.GabpError) as e:
        s3.solve(wl.X, wl.y)
    assert e.value.status == gabp.E_INVALID


# (N, gamma, precision, series form): wide RBFs give row sums ~ N and a
# contraction rho ~ 1/N; FP32 messages (FP32, MIXED) take the one-term top
# level while rho^4 is below 2^-24 (form 1), with 1/P~ alone at the lower
# levels when rho^3 is too and a middle level exists (form 3), and the
# two-term one up to rho^6 (form 2); FP64 needs rho^5 below 2^-52 for any
# series (rr = 1.25 rho throughout)
SERIES_CASES = [(1500, 2e-3, "fp32", 3), (1500, 2e-3, "mixed", 3), (1500, 5e-3, "mixed", 3),
                (1500, 2e-2, "fp32", 1), (1500, 2e-2, "mixed", 1), (600, 0.05, "fp32", 2),
                (600, 0.05, "mixed", 2), (2000, 2e-3, "fp64", 2)]


@pytest.mark.parametrize("n,gamma,prec,form", SERIES_CASES)
def test_stateless_series_reciprocals_match_oracle(torch, n, gamma, prec, form):
    """The sweeps with series reciprocals follow the oracle's truncated
    recursion (exact reciprocals) at the chosen depth: the series error is
    below the arithmetic's precision by the plan's rule."""
    X, y = inputs.blobs(n, 8, 71)
    wl = inputs.Workload("blobs-wide", X, y, gamma=gamma, C=1.0, lam=1.0 / n, precision=prec, tol_rel=0.0)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    tol = 1e-11 if prec == "fp64" else TOL
    print(f"[case] series n={n} gamma={gamma} {prec}", flush=True)
    for t in (1, 2, 3, 6):
        s, st = run(torch, wl, precision=prec, edge_state="stateless", kstore="materialise",
                    max_sweeps=t, tol_abs=0.0, tol_rel=0.0, stagnation_window=0)
        p = s.plan()
        assert p["series_reciprocal"] == form, p
        ref = R.gabp_solve_stateless(A, b, depth=p["stateless_depth"], sweeps=t)[-1]
        err = _rel(s.alpha(), ref)
        assert err <= tol, (prec, t, p["stateless_depth"], err)
    exact = R.cholesky_solve(A, b)
    s, st = run(torch, wl, precision=prec, edge_state="stateless", tol_rel=1e-9)
    err = _rel(s.alpha(), exact)
    print(f"series stateless {prec}: depth {s.plan()['stateless_depth']} form {s.plan()['series_reciprocal']} "
          f"rho {s.plan()['stateless_rho']:.2e} sweeps {s.sweeps()} rel err vs Cholesky {err:.2e}")
    # the stop rule (change below 1e-9 relative) bounds the distance left
    assert st == gabp.OK and err <= (1e-8 if prec == "fp64" else TOL)


@pytest.mark.parametrize("gamma", [2e-3, 1.0 / 8, 1.0])
def test_contraction_bound_matches_oracle(torch, gamma):
    """The plan's contraction bound (computed on the device from the weighted
    diagonal, the row maxima and the row sums of K') equals the oracle's
    bound on the same system, and bounds the contraction the sweeps reach."""
    X, y = inputs.blobs(700, 8, 93)
    wl = inputs.Workload("blobs-rho", X, y, gamma=gamma, C=1.0, lam=1.0 / 700, precision="fp64",
                         tol_rel=1e-9)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    mstar, rho_ref = R.contraction_bound(A)
    reached = max(R.message_contraction(A, 30))
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        s, st = run(torch, wl, precision=prec, kstore="materialise")
        rho = s.plan()["stateless_rho"]
        print(f"gamma {gamma} {prec}: rho {rho:.6e} oracle {rho_ref:.6e} reached {reached:.6e}")
        assert abs(rho - rho_ref) <= tol * rho_ref
        assert reached <= rho * (1 + 1e-9)


# --------------------------------------------------- decision function (MFMA) --

@pytest.mark.parametrize("prec,gram,m,bound", [
    ("fp32", "auto", 54, TOL), ("mixed", "bf16x6", 54, TOL), ("mixed", "bf16x6", 10, TOL),
    ("fp32", "auto", 130, TOL), ("mixed", "bf16x3", 20, 1e-4), ("mixed", "bf16", 130, 1e-2),
    ("fp64", "auto", 54, 1e-10)])
def test_predict_matches_oracle_on_held_out_points(torch, prec, gram, m, bound):
    """f(x_q) on held-out points against the oracle's decision function with
    the same alpha: |f - f_ref| <= bound * sum_i |alpha_i| (every K' entry is
    at most 1 + lambda^2, so this is the kernel's relative accuracy).  N and
    the query count are ragged against the 32-row blocks and the 128-query
    workgroups; m = 10, 20, 54, 130 cover register-held query fragments of
    32, 64 and 128 features and the reloading form beyond."""
    X, y, Xt, yt = inputs.covertype_like(1100, m, 51 + m, n_test=1000)
    wl = inputs.Workload("covertype-holdout", X, y, gamma=27.0 / m, C=1.0, lam=1.0 / 1100,
                         precision=prec, tol_rel=1e-9)
    s, st = run(torch, wl, gram=gram)
    assert st == gabp.OK
    alpha = s.alpha()
    f = s.predict(Xt)
    ref = R.decision_function(wl.X, wl.y, alpha, Xt, wl.gamma, wl.lam)
    scale = float(np.sum(np.abs(alpha)))
    err = float(np.max(np.abs(f - ref))) / scale
    acc = np.mean(np.where(f >= 0, 1.0, -1.0) == yt)
    print(f"predict {prec}/{gram} m={m}: max |f - f_ref| / sum|alpha| = {err:.2e}; "
          f"held-out accuracy {acc:.3f}")
    assert err <= bound
    if bound <= 1e-4:
        # labels agree wherever the oracle's f is farther from 0 than twice
        # the bound (for the single-product Gram, 1e-2 of sum |alpha| exceeds
        # every |f|, so the labels are not decided by the bound there)
        sure = np.abs(ref) > 2 * bound * scale
        assert sure.sum() >= 100
        assert np.array_equal(np.sign(f[sure]), np.sign(ref[sure]))
    fd = s.predict(torch.from_numpy(Xt).cuda()).cpu().numpy()
    assert np.array_equal(fd, f)
    # one query, and the last partial workgroup alone
    assert np.array_equal(s.predict(Xt[5:6]), f[5:6])
    assert np.array_equal(s.predict(Xt[-7:]), f[-7:])


def test_predict_box_clip_uses_clipped_alpha(torch):
    wl = inputs.make_workload("covertype", n=900, seed=23)
    s, st = run(torch, wl, precision="mixed", box_mode="clip_output", C=0.002)
    a = s.alpha()
    assert a.max() <= 0.002 and a.min() >= 0.0
    Xq = inputs.make_workload("covertype", n=300, seed=24).X
    f = s.predict(Xq)
    ref = R.decision_function(wl.X, wl.y, a, Xq, wl.gamma, wl.lam)
    assert float(np.max(np.abs(f - ref))) <= TOL * float(np.sum(np.abs(a)))


# ------------------------------------------------ grouped (Gauss-Seidel) schedule --

def _block_groups(n, G):
    """The library's groups: 256-point block I belongs to group I G / NB."""
    NB = (n + 255) // 256
    G = min(G, NB)
    blk = np.arange(n) // 256
    gid = blk * G // NB
    return [np.nonzero(gid == g)[0] for g in range(G)]


@pytest.mark.parametrize("prec,edge,G", [("fp64", "stored", 3), ("fp64", "stateless", 2), ("fp32", "stored", 5),
                                         ("fp32", "stateless", 3), ("mixed", "stateless", 5), ("mixed", "stored", 2)])
def test_grouped_schedule_matches_oracle_sweep_by_sweep(torch, prec, edge, G):
    """Each sweep of the grouped schedule against the oracle's grouped
    schedule (stored messages, or the same chains rebuilt from the aggregate
    history at the plan's depth); N = 1100 spans five blocks with a ragged
    last one, so groups of one, two and uneven block counts occur."""
    wl = inputs.make_workload("covertype", n=1100, seed=41)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    groups = _block_groups(1100, G)
    depth = 3 if edge == "stateless" else 0
    ref_stored = R.gabp_solve_grouped(A, b, groups, max_sweeps=8, tol_rel=0.0, keep_trajectory=True)
    ref_sl = R.gabp_solve_grouped_stateless(A, b, groups, depth, 8) if depth else None
    for t in (1, 2, 3, 5, 8):
        kw = dict(precision=prec, edge_state=edge, kstore="materialise", schedule="grouped", sched_groups=G,
                  max_sweeps=t, tol_abs=0.0, tol_rel=0.0, stagnation_window=0)
        if depth:
            kw["stateless_depth"] = depth
        s, st = run(torch, wl, **kw)
        assert s.sweeps() == t and s.plan()["sched_groups"] == G
        ref = ref_sl[t - 1] if depth else ref_stored.trajectory[t]
        err = _rel(s.alpha(), ref)
        tol = 1e-12 if prec == "fp64" else TOL
        assert err <= tol, (prec, edge, G, t, err)


@pytest.mark.parametrize("prec,kstore", [("fp64", "materialise"), ("fp32", "materialise"), ("mixed", "materialise"),
                                         ("mixed", "recompute"), ("fp32", "recompute")])
def test_grouped_schedule_converges_to_the_solution_in_fewer_sweeps(torch, prec, kstore):
    wl = inputs.make_workload("covertype", n=2600, seed=43)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    exact = R.cholesky_solve(A, b)
    out = {}
    for sched in ("sync", "grouped"):
        s, st = run(torch, wl, precision=prec, kstore=kstore, schedule=sched, tol_rel=1e-9)
        assert st == gabp.OK
        out[sched] = (s.sweeps(), _rel(s.alpha(), exact), s.plan())
    print(f"{prec}/{kstore}: sync {out['sync'][:2]}, grouped {out['grouped'][:2]} "
          f"(edge {out['grouped'][2]['edge_state']}, depth {out['grouped'][2]['stateless_depth']})")
    assert out["grouped"][1] <= TOL
    assert 3 * out["grouped"][0] <= out["sync"][0]


# ------------------------------------------------------- box-projected variant --

def _box_case(name, seed, q):
    wl = inputs.make_workload(name, n=1100, seed=seed)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    C = float(np.quantile(R.cholesky_solve(A, b), q))
    return wl, A, b, C


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_box_projected_sweeps_match_oracle(torch, prec):
    """The projected sweep (belief means clipped to [0, C] every sweep)
    against the oracle's projected sweep, sweep by sweep; the tiny workload
    has negative unconstrained alphas, so both bounds bind."""
    wl, _, _, C = _box_case("tiny", 52, 0.9)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, C, wl.lam)     # C also enters the diagonal
    ref = R.gabp_solve_box(A, b, C, max_sweeps=8, tol_rel=0.0, keep_trajectory=True)
    for t in (1, 2, 3, 5, 8):
        s, st = run(torch, wl, precision=prec, C=C, box_mode="project", edge_state="stored",
                    max_sweeps=t, tol_abs=0.0, tol_rel=0.0, stagnation_window=0)
        err = _rel(s.alpha(), ref.trajectory[t])
        assert err <= (1e-12 if prec == "fp64" else TOL), (prec, t, err)
        a = s.alpha()
        assert a.min() >= 0.0 and a.max() <= C


@pytest.mark.parametrize("name,seed,q,kw", [
    ("tiny", 52, 0.9, dict(precision="fp64")),
    ("covertype", 51, 0.8, dict(precision="mixed")),
    ("covertype", 51, 0.8, dict(precision="mixed", schedule="grouped")),
    ("covertype", 51, 0.8, dict(precision="fp32", edge_state="stateless"))])
def test_box_projected_solution_is_the_qp_optimum(torch, name, seed, q, kw):
    """At convergence the projected sweep gives the optimum of the
    box-constrained dual QP (projected Gauss-Seidel oracle), in every form:
    stored or stateless edges, synchronous or grouped schedule."""
    wl, _, _, C = _box_case(name, seed, q)
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, C, wl.lam)
    h = R.box_qp_projected_gauss_seidel(A, C)
    s, st = run(torch, wl, C=C, box_mode="project", tol_rel=1e-10, **kw)
    err = float(np.max(np.abs(s.alpha() - h)) / np.max(h))
    n_lo, n_hi = int(np.sum(h <= 0.0)), int(np.sum(h >= C))
    print(f"box {name} {kw}: {s.sweeps()} sweeps, at 0: {n_lo}, at C: {n_hi}, rel err vs QP {err:.2e}")
    assert st == gabp.OK and err <= TOL and n_lo + n_hi > 0


@pytest.mark.parametrize("edge", ["stored", "stateless"])
def test_repeated_solves_on_one_handle_reuse_buffers(torch, edge):
    """A handle keeps its device buffers between solves and reuses them when
    they are large enough: the same problem twice, a smaller one after it and
    the larger one again all give bitwise the alpha of a fresh handle."""
    X1, y1 = inputs.blobs(1100, 16, 501)
    X2, y2 = inputs.blobs(600, 16, 502)
    kw = dict(gamma=1.0 / 16, C=1.0, precision="mixed", tol_rel=1e-7, edge_state=edge, kstore="materialise")
    print(f"[case] repeated solves, {edge} edges", flush=True)

    def fresh(X, y):
        s = gabp.GabpSVM(**kw)
        assert s.solve(X, y) == gabp.OK
        a = s.alpha()
        s.close()
        return a

    ref1, ref2 = fresh(X1, y1), fresh(X2, y2)
    s = gabp.GabpSVM(**kw)
    held = []
    for X, y, ref in ((X1, y1, ref1), (X1, y1, ref1), (X2, y2, ref2), (X1, y1, ref1)):
        assert s.solve(X, y) == gabp.OK
        assert np.array_equal(s.alpha(), ref)
        held.append(s.plan()["device_bytes"])
    s.close()
    # the second solve of the same shape holds what the first held
    assert held[1] == held[0]


# --------------------------------------------------- residual certificate --

@pytest.mark.parametrize("prec,kstore,n", [("fp64", "materialise", 700), ("fp32", "materialise", 1100),
                                           ("mixed", "materialise", 2600), ("mixed", "recompute", 2600),
                                           ("fp32", "recompute", 257)])
def test_residual_certificate_matches_oracle(torch, oracle_c, prec, kstore, n):
    """GABP_Q_RESIDUAL_BOUND against the oracle over every row: the device
    forms ||1 - A alpha||_inf with its own K' (FP64 entries in the FP64 path,
    FP32 otherwise), so the two residuals differ by at most the K' rounding
    times sum_j |A_ij alpha_j|; the dominance gap min_i (A_ii - r_i) likewise;
    and the bound certifies the distance to the exact solution (Cholesky)."""
    wl = inputs.make_workload("covertype" if prec != "fp64" else "tiny", n=n, seed=31)
    s, st = run(torch, wl, precision=prec, kstore=kstore, tol_rel=1e-9, tol_abs=0.0,
                edge_state="stored" if kstore == "materialise" else "auto")
    assert st == gabp.OK
    a = s.alpha()
    c = s.residual_bound()
    A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam)
    res, _ = oracle_c.residual_rows(wl.X, wl.y, wl.gamma, wl.C, wl.lam, a, np.arange(wl.N))
    absrow = np.abs(A) @ np.abs(a)                 # sum_j |A_ij alpha_j|
    off = np.abs(A - np.diag(np.diag(A))).sum(axis=1)
    gap_ref = float(np.min(np.diag(A) - off))
    eps = 1e-13 if prec == "fp64" else 4e-6        # K' entry accuracy of the path
    print(f"certificate {prec}/{kstore} N={n}: device residual {c['residual_inf']:.3e} "
          f"(oracle {np.max(np.abs(res)):.3e}), gap {c['gap']:.6g} (oracle {gap_ref:.6g}), bound {c['bound']:.3e}")
    assert abs(c["residual_inf"] - np.max(np.abs(res))) <= eps * float(np.max(absrow)) + 1e-15
    assert abs(c["gap"] - gap_ref) <= eps * float(np.max(np.diag(A)))
    assert c["bound"] == pytest.approx(c["residual_inf"] / c["gap"], rel=1e-15)
    exact = R.cholesky_solve(A, b)
    err = float(np.max(np.abs(a - exact)))
    # Varah on the oracle's system, with the device residual standing in for
    # the oracle's up to the same K' rounding
    assert err <= (c["residual_inf"] + eps * float(np.max(absrow))) / gap_ref * (1 + 1e-9)
    # the query is formed once per solve and repeats exactly
    assert s.residual_bound() == c


def test_residual_certificate_refused_for_sparse(torch):
    wl = inputs.make_workload("large", n=3000)
    s, st = run(torch, wl, kernel="rbf_sparse", sparse_tau=0.3)
    assert st == gabp.OK
    with pytest.raises(gabp.GabpError) as e:
        s.residual_bound()
    assert e.value.status == gabp.E_STATE


# ------------------------------------------- plans without a truncation bound --

def test_stateless_without_bound_is_refused(torch):
    """The soft-margin diagonal alone (K'_ii + 1/C) leaves the dense RBF
    system far from dominant: no contraction bound exists.  AUTO without room
    for the stored records (a 20 MB budget: the K' plane of 1,800 points is
    9.4 MB, the four record planes 38 MB) must fail with GABP_E_NOMEM, an
    explicit stateless plan with an automatic depth with GABP_E_INVALID; an
    explicit depth runs the truncated recursion and the plan flags it."""
    wl = inputs.make_workload("letter", n=1800)
    kw = dict(precision="fp32", diag_mode="softmargin", max_sweeps=5)
    s0, _ = run(torch, wl, **kw)
    assert s0.plan()["edge_state"] == gabp.EDGE["stored"]       # AUTO with room: stored records
    assert not (1.25 * s0.plan()["stateless_rho"] < 1.0)        # no bound at all
    with pytest.raises(gabp.GabpError) as e:
        run(torch, wl, hbm_budget_bytes=int(20e6), **kw)
    assert e.value.status == gabp.E_NOMEM and "truncation bound" in str(e.value)
    with pytest.raises(gabp.GabpError) as e:
        run(torch, wl, edge_state="stateless", **kw)
    assert e.value.status == gabp.E_INVALID
    s, st = run(torch, wl, edge_state="stateless", stateless_depth=3, **kw)
    assert s.plan()["stateless_depth"] == 3 and s.plan()["stateless_bounded"] == 0


def test_stateless_depth_flag_follows_the_bound(torch):
    """A bounded contraction that needs more than 8 levels for the message
    precision (two blobs, gamma = 1/16, MIXED: rho about 0.09): AUTO keeps the
    stored records, an explicit stateless plan takes 8 levels and is flagged
    as truncated; the benchmark-shaped dominant system reaches its bound."""
    X, y = inputs.blobs(1100, 16, 501)
    wl = inputs.Workload("blobs", X, y, gamma=1.0 / 16, C=1.0, lam=1.0 / 1100, precision="mixed")
    a, _ = run(torch, wl)
    rho = a.plan()["stateless_rho"]
    assert 0.0 < 1.25 * rho < 1.0 and a.plan()["edge_state"] == gabp.EDGE["stored"]
    b, st = run(torch, wl, edge_state="stateless")
    assert st == gabp.OK and b.plan()["stateless_depth"] == 8 and b.plan()["stateless_bounded"] == 0
    # 10 MB: the stateless form fits (K' plane 3.9 MB), the records never do
    # (four planes 15.7 MB)
    with pytest.raises(gabp.GabpError) as e:
        run(torch, wl, hbm_budget_bytes=int(10e6))
    assert e.value.status == gabp.E_NOMEM
    wl2 = inputs.make_workload("covertype", n=2000)
    s2, _ = run(torch, wl2, edge_state="stateless")
    assert s2.plan()["stateless_bounded"] == 1 and s2.plan()["stateless_depth"] <= 8
