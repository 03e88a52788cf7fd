"""Pins of the oracle's (r, c)-ANN query (Alg. 6) and of the PAA projection of
DET-ONLY (Sec. 6.1) against what the paper and the mathematics fix: brute
force where the radius admits everything, the empty answer where it admits
nothing, Theorem 1's success probability measured empirically, the relation
the paper states between Alg. 6 and one round of Alg. 7, and segment means
computed directly.  Planted mistakes (on the CPU) are each caught."""
import math

import numpy as np
import pytest

import synth
from oracle import detlsh_oracle as O
from test_oracle_pins import brute_ids, check_lb_invariant, make_problem


def nearest(X, q):
    ids, d = brute_ids(X, q, 1)
    return int(ids[0]), float(d[0])


@pytest.mark.parametrize("kind", ["mixture", "integer"])
@pytest.mark.parametrize("seed", [0, 1])
def test_rc_huge_radius_is_exact_nearest_neighbour(kind, seed):
    X, idx, _ = make_problem(n=1200, seed=seed, kind=kind)
    rng = np.random.default_rng(seed)
    for q in synth.gaussian_mixture(5, X.shape[1], 8, 3.0, 1.0, 500 + seed, rows_seed=900 + seed):
        if kind == "integer":
            q = rng.integers(0, 5, X.shape[1]).astype(np.float64)
        qp = O.project(q[None, :], idx.A)[0]
        res = O.query_rc(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 1e9, 1.5, 0.1)
        assert res.cond == 1 and res.stop_tree == 1 and res.S.size == X.shape[0]
        assert (res.id, pytest.approx(res.dist)) == nearest(X, q)


def test_rc_zero_radius_returns_nothing_or_the_query_itself():
    X, idx, _ = make_problem(n=2000, d=24, K=8, N_r=64, frac=0.1, seed=3)
    need = O.n_stop(X.shape[0], 1, 0.1)
    rng = np.random.default_rng(3)
    # a query not in D: S holds the points sharing a cell with it, none at distance 0
    q = X[7].astype(np.float64) + rng.normal(0, 0.05, X.shape[1])
    qp = O.project(q[None, :], idx.A)[0]
    res = O.query_rc(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 0.0, 1.5, 0.1)
    assert res.S.size < need
    assert res.id == -1 and math.isinf(res.dist) and res.cond == 0
    # the query is a data point: its own cell admits it at distance 0 (condition 2)
    q = X[11].astype(np.float64)
    qp = O.project(q[None, :], idx.A)[0]
    res = O.query_rc(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 0.0, 1.5, 0.1)
    assert res.cond == 2 and res.dist == 0.0
    assert res.id == min(np.flatnonzero((X == X[11]).all(1)))


def test_rc_theorem_one_success_rate():
    """Theorem 1: with r the exact nearest-neighbour distance, Alg. 6 returns a
    point within c*r with probability at least 1/2 - 1/e."""
    ok = trials = 0
    for seed in range(12):
        X, idx, _ = make_problem(n=1500, d=32, L=4, K=16, N_r=64, frac=0.1, seed=seed)
        Qs = synth.gaussian_mixture(15, X.shape[1], 8, 3.0, 1.0, 500 + seed, rows_seed=700 + seed)
        for q in Qs:
            _, r = nearest(X, q)
            qp = O.project(q[None, :], idx.A)[0]
            res = O.query_rc(X, q, qp, idx.codes, idx.B, idx.L, idx.K, r, 1.5, 0.1)
            trials += 1
            ok += res.id >= 0 and res.dist <= 1.5 * r * (1 + 1e-12)
    rate = ok / trials
    print(f"Theorem 1 empirical success rate {rate:.3f} over {trials} trials (bound 0.1321)")
    assert rate >= 0.5 - 1 / math.e


@pytest.mark.parametrize("c", [1.5, 2.0])
def test_rc_is_the_first_round_of_the_printed_ladder(c):
    """Alg. 7's loop body is Alg. 6 with k points (Sec. 4.3): from r_min = r,
    Alg. 7 with k = 1 stops in its first round exactly when Alg. 6 answers, with
    the same candidate set and point; when Alg. 6 answers nothing, Alg. 7 goes on."""
    X, idx, _ = make_problem(n=1500, d=24, K=8, N_r=32, frac=0.1, seed=5)
    Qs = synth.gaussian_mixture(12, X.shape[1], 8, 3.0, 1.0, 505, rows_seed=805)
    answered = empty = 0
    for q in Qs:
        qp = O.project(q[None, :], idx.A)[0]
        _, nn = nearest(X, q)
        for r in (0.3 * nn, nn, 2.0 * nn):
            rc = O.query_rc(X, q, qp, idx.codes, idx.B, idx.L, idx.K, r, c, 0.1)
            fx = O.query_fixed(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 1, 0.1, c, r)
            if rc.id >= 0:
                answered += 1
                assert fx.rounds == 1 and fx.ids[0] == rc.id and np.array_equal(fx.S, rc.S)
                assert fx.stop_cond == rc.cond
            else:
                empty += 1
                assert fx.rounds >= 2
    assert answered and empty


def test_paa_rows_are_segment_means():
    for d, K in [(128, 16), (96, 16), (100, 16), (960, 16), (37, 4)]:
        A = O.paa_matrix(d, K)
        w = d // K
        assert A.shape == (K, d)
        np.testing.assert_allclose(A.sum(1), 1.0)
        X = np.random.default_rng(d).normal(size=(50, d))
        direct = X[:, :K * w].reshape(50, K, w).mean(-1)
        np.testing.assert_allclose(O.project(X, A), direct, rtol=1e-12, atol=1e-12)
    with pytest.raises(ValueError):
        O.paa_matrix(8, 16)


def test_det_only_bounds_and_brute_force():
    """DET-ONLY (one space, PAA means) keeps the lower-bound invariant and, with
    beta = 1, returns exact brute force."""
    X = synth.gaussian_mixture(1200, 64, 8, 3.0, 1.0, 901)
    A = O.paa_matrix(64, 16)
    sample = synth.sample_ids(1200, 240, 902)
    idx = O.build_index(X, A, sample, 1, 16, 64)
    Qs = synth.gaussian_mixture(6, 64, 8, 3.0, 1.0, 901, rows_seed=903)
    check_lb_invariant(X, Qs, idx)
    for q in Qs:
        qp = O.project(q[None, :], A)[0]
        res = O.query_magic(X, q, qp, idx.codes, idx.B, 1, 16, 10, 1.0)
        ids, d = brute_ids(X, q, 10)
        assert np.array_equal(res.ids, ids)
        np.testing.assert_allclose(res.dists, d, rtol=1e-12)


# --------------------------------------------------------------------------
# planted mistakes
# --------------------------------------------------------------------------

def test_planted_first_admitted_instead_of_nearest_is_caught(monkeypatch):
    def first_not_nearest(ids, d2, k):
        return np.asarray(ids)[:k], np.asarray(d2)[:k]
    monkeypatch.setattr(O, "top_k", first_not_nearest)
    with pytest.raises(AssertionError):
        test_rc_huge_radius_is_exact_nearest_neighbour("mixture", 0)


def test_planted_paa_window_off_by_one_is_caught(monkeypatch):
    def paa_shifted(d, K):
        w = d // K
        A = np.zeros((K, d))
        for j in range(K):
            A[j, j * w + 1:(j + 1) * w + 1] = 1.0 / w
        return A
    monkeypatch.setattr(O, "paa_matrix", paa_shifted)
    with pytest.raises(AssertionError):
        test_paa_rows_are_segment_means()


def test_insert_with_frozen_breakpoints():
    """Inserted points are encoded against the built breakpoints: in any split
    the codes equal one encoding of the union with those breakpoints, the
    breakpoints stay, and the rebuilt trees partition all points."""
    X, idx, _ = make_problem(n=1500, d=24, K=8, N_r=16, frac=0.2, seed=8)
    new = synth.gaussian_mixture(700, X.shape[1], 8, 3.0, 1.0, 508, rows_seed=908)
    one = O.insert(idx, new)
    two = O.insert(O.insert(idx, new[:300]), new[300:])
    assert np.array_equal(one.codes, two.codes) and np.array_equal(one.B, idx.B)
    union = O.encode(O.project(np.concatenate([X, new]), idx.A), idx.B)
    assert np.array_equal(one.codes, union)
    trees = O.build_trees(one.codes, one.L, one.K, one.N_r, 32)
    for leaves in trees:
        ids = np.sort(np.concatenate([lf.ids for lf in leaves]))
        assert np.array_equal(ids, np.arange(len(union)))


def test_planted_insert_with_refreshed_breakpoints_is_caught(monkeypatch):
    real = O.insert

    def refreshed(idx, X_new):
        out = real(idx, X_new)
        B = O.breakpoints_by_sort(O.project(X_new, idx.A), idx.N_r)
        return O.Index(idx.A, B, out.codes, idx.L, idx.K, idx.N_r)
    monkeypatch.setattr(O, "insert", refreshed)
    with pytest.raises(AssertionError):
        test_insert_with_frozen_breakpoints()


# --------------------------------------------------------------------------
# leaf-granularity query (the query-phase optimisation)
# --------------------------------------------------------------------------

def _leaf_case(seed=10, n=1800, max_leaf=16, kind="mixture"):
    X, idx, _ = make_problem(n=n, d=24, L=4, K=8, N_r=32, frac=0.2, seed=seed, kind=kind)
    trees = O.build_trees(idx.codes, idx.L, idx.K, idx.N_r, max_leaf)
    Qs = synth.gaussian_mixture(6, X.shape[1], 8, 3.0, 1.0, 500 + seed, rows_seed=950 + seed)
    return X, idx, trees, Qs


@pytest.mark.parametrize("max_leaf", [4, 16, 64])
def test_leaf_query_magic_radius_and_stop(max_leaf):
    """At the magic radius the admitted leaves of all trees hold N_S points and
    at any smaller radius fewer; the query stops inside one leaf's worth of
    N_S; the leaves taken from the stop tree are a prefix in bound order; the
    answer is brute force over S."""
    X, idx, trees, Qs = _leaf_case(max_leaf=max_leaf)
    N_S = O.n_stop(len(X), 10, 0.1)
    biggest = max(len(lf.ids) for t in trees for lf in t)
    for q in Qs:
        qp = O.project(q[None, :], idx.A)[0]
        res = O.query_magic_leaf(X, q, qp, idx.codes, idx.B, trees, idx.L, idx.K, 10, 0.1)
        lb, leafmin = O.leaf_bounds(qp, trees, idx.B, idx.L, idx.K)
        m = lb.min(axis=1)
        assert (m <= res.thr).sum() >= N_S
        assert (m <= np.nextafter(res.thr, -np.inf)).sum() < N_S
        assert N_S <= len(res.S) < N_S + biggest
        i = res.stop_tree - 1
        taken = np.isin(np.arange(len(X)), res.S)
        new_here = res.first_tree == res.stop_tree
        inside = set(zip(lb[res.S[new_here], i], leafmin[res.S[new_here], i]))
        outside = [(lb[o, i], leafmin[o, i]) for o in np.flatnonzero(~taken) if lb[o, i] <= res.thr
                   and not (lb[o, :i] <= res.thr).any()]
        if inside and outside:
            assert max(inside) < min(outside)
        ids, d = brute_ids(X[res.S], q, 10)
        assert np.array_equal(res.ids, res.S[ids])


def test_leaf_bound_admits_a_superset_and_beta_one_is_brute_force():
    X, idx, trees, Qs = _leaf_case(seed=11)
    for q in Qs[:3]:
        qp = O.project(q[None, :], idx.A)[0]
        lb_leaf, _ = O.leaf_bounds(qp, trees, idx.B, idx.L, idx.K)
        lb_cell = O.lower_bounds(qp, idx.codes, idx.B, idx.L, idx.K)
        assert np.all(lb_leaf <= lb_cell * (1 + 1e-12) + 1e-12)
        res = O.query_magic_leaf(X, q, qp, idx.codes, idx.B, trees, idx.L, idx.K, 10, 1.0)
        ids, d = brute_ids(X, q, 10)
        assert np.array_equal(res.ids, ids)


def test_planted_cell_bound_in_the_leaf_queue_is_caught(monkeypatch):
    """Admitting leaves by a member's cell bound instead of the leaf box bound
    (the relaxation undone in one place) is caught."""
    def cell_queue(qp_i, leaves, B_i, radius2):
        lo, hi = O.region_bounds(B_i)
        out = []
        for lf in leaves:
            c = lf.lo + (lf.hi - lf.lo) // 2
            b = O.node_lb2(qp_i, c, c, B_i)
            if b <= radius2:
                out.append((b, int(lf.ids.min()), lf.ids))
        out.sort(key=lambda e: (e[0], e[1]))
        return [ids for _, _, ids in out]
    monkeypatch.setattr(O, "leaf_queue", cell_queue)
    with pytest.raises(AssertionError):
        test_leaf_query_magic_radius_and_stop(16)
