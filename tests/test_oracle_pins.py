"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each check below ties one oracle function to something other than itself:
closed forms (Lemma 1, Lemma 3 / Eq. 2, the equal-frequency rule of Sec. 4.1),
invariants (lower bounds never exceed the projected distance, monotone
candidate sets, a partition of the points into leaves), brute force on tiny
inputs, the paper's own alternative algorithm (Alg. 1 against the sorted
sample; the printed Alg. 7 loop against the one-shot magic radius; the tree
walk of Alg. 4/5 against the flat predicate) and the paper's success
probability bounds measured empirically.  The last section plants plausible
mistakes into the oracle (on the CPU) and checks that a pin catches each.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.distance import cdist

import synth
from oracle import detlsh_oracle as O


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def make_problem(n=1500, d=24, L=4, K=8, N_r=16, frac=0.2, seed=0, kind="mixture"):
    rng = np.random.default_rng(seed)
    if kind == "integer":                      # many exact distance ties
        X = rng.integers(0, 5, (n, d)).astype(np.float32)
    else:
        X = synth.gaussian_mixture(n, d, 8, 3.0, 1.0, 500 + seed)
    A = synth.projection_matrix(L, K, d, 100 + seed)
    sample = synth.sample_ids(n, max(N_r, int(frac * n)), 200 + seed)
    idx = O.build_index(X, A, sample, L, K, N_r)
    return X, idx, sample


def brute_ids(X, q, k):
    d2 = cdist(np.asarray(q, np.float64)[None, :], np.asarray(X, np.float64),
               metric="sqeuclidean")[0]
    order = sorted(range(len(d2)), key=lambda o: (d2[o], o))[:k]
    return np.array(order), np.sqrt(d2[order])


def chi2_sf_even(x, K):
    """Pr[Y > x] for Y ~ chi^2(K), K even: exp(-x/2) sum_{i<K/2} (x/2)^i / i!
    (the Poisson-sum closed form, independent of scipy)."""
    assert K % 2 == 0
    h = x / 2.0
    term, s = 1.0, 1.0
    for i in range(1, K // 2):
        term *= h / i
        s += term
    return math.exp(-h) * s


def chi2_isf_even(alpha, K):
    lo, hi = 0.0, 1000.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if chi2_sf_even(mid, K) > alpha:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def check_equal_frequency(Ps, B):
    """P8 on a sample without ties."""
    n_s, m = Ps.shape
    N_r = B.shape[1] - 1
    codes = O.encode(Ps, B)
    for e in range(m):
        cnt = np.bincount(codes[:, e].astype(np.int64), minlength=N_r)
        for z in range(1, N_r + 1):                     # 1-indexed region
            want = (z * n_s) // N_r - ((z - 1) * n_s) // N_r
            if z == 1:
                want -= 1
            if z == N_r:
                want += 1
            if cnt[z - 1] != want:
                return False
    return True


def check_lb_invariant(X, Qs, idx):
    """P3: LB_i(q, o)^2 <= ||H_i(q) - H_i(o)||^2 for all q, o, i."""
    P = O.project(X, idx.A)
    for q in Qs:
        qp = O.project(q[None, :], idx.A)[0]
        lb = O.lower_bounds(qp, idx.codes, idx.B, idx.L, idx.K)
        for i in range(idx.L):
            sl = slice(i * idx.K, (i + 1) * idx.K)
            true2 = ((P[:, sl] - qp[sl]) ** 2).sum(axis=1)
            if np.any(lb[:, i] > true2 * (1 + 1e-12) + 1e-12):
                return False
    return True


# --------------------------------------------------------------------------
# P1 / P2: brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["mixture", "integer"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p1_beta_one_is_brute_force(kind, seed):
    """With beta = 1, N_S >= n so S = D and the answer is the exact k-NN."""
    X, idx, _ = make_problem(n=600, seed=seed, kind=kind)
    Q = X[:5] + 0.37
    for q in Q:
        qp = O.project(q[None, :], idx.A)[0]
        r = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, k=10, beta=1.0)
        ids, dist = brute_ids(X, q, 10)
        assert np.array_equal(r.ids, ids)
        np.testing.assert_allclose(r.dists, dist, rtol=1e-12)
        assert len(r.S) == len(X)


def test_p1_single_region_is_brute_force():
    """N_r = 1: every region bound is 0, so every point is a candidate."""
    X, idx, _ = make_problem(n=500, N_r=1, seed=3)
    q = X[7] * 1.01
    qp = O.project(q[None, :], idx.A)[0]
    r = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, k=7, beta=0.05)
    ids, _ = brute_ids(X, q, 7)
    assert np.array_equal(r.ids, ids)
    assert len(r.S) == len(X)


@pytest.mark.parametrize("kind", ["mixture", "integer"])
def test_p2_answer_is_brute_force_over_S(kind):
    X, idx, _ = make_problem(n=1500, seed=4, kind=kind)
    for q in X[:6] + 0.11:
        qp = O.project(q[None, :], idx.A)[0]
        r = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, k=10, beta=0.1)
        sub_ids, sub_d = brute_ids(X[r.S], q, 10)
        assert np.array_equal(r.ids, r.S[sub_ids])
        np.testing.assert_allclose(r.dists, sub_d, rtol=1e-12)
        assert len(r.S) >= O.n_stop(len(X), 10, 0.1)


# --------------------------------------------------------------------------
# P3: lower bound invariant (including out-of-sample and out-of-range points)
# --------------------------------------------------------------------------

def test_p3_lower_bound_never_exceeds_projected_distance():
    X, idx, _ = make_problem(n=1200, frac=0.05, seed=5)
    far = np.vstack([X[:3] * 4.0, -X[3:6] * 3.0])          # outside the sample's range
    Xall = np.vstack([X, far]).astype(np.float32)
    P = O.project(Xall, idx.A)
    idx2 = O.Index(idx.A, idx.B, O.encode(P, idx.B), idx.L, idx.K, idx.N_r)
    Qs = np.vstack([X[10:14] + 0.5, far[:2] * 1.3])
    assert check_lb_invariant(Xall, Qs, idx2)


def test_p3_node_bound_below_member_bounds():
    X, idx, _ = make_problem(n=2000, K=6, N_r=16, seed=6)
    trees = O.build_trees(idx.codes, idx.L, idx.K, idx.N_r, max_leaf=16)
    q = X[3] + 0.9
    qp = O.project(q[None, :], idx.A)[0]
    lb = O.lower_bounds(qp, idx.codes, idx.B, idx.L, idx.K)
    for i, leaves in enumerate(trees):
        sl = slice(i * idx.K, (i + 1) * idx.K)
        for lf in leaves:
            nlb = O.node_lb2(qp[sl], lf.lo, lf.hi, idx.B[sl])
            assert nlb <= lb[lf.ids, i].min() * (1 + 1e-12) + 1e-15


# --------------------------------------------------------------------------
# P4 / P5: Lemma 1 and the E1 probability of Lemma 3
# --------------------------------------------------------------------------

def test_p4_projected_ratio_is_chi2():
    d, K = 32, 16
    rng = np.random.default_rng(11)
    x = rng.standard_normal(d)
    ratios = []
    for seed in range(2500):
        A = synth.projection_matrix(1, K, d, 10_000 + seed)
        p = O.project(x[None, :], A)[0]
        ratios.append((p @ p) / (x @ x))
    assert stats.kstest(ratios, "chi2", args=(K,)).pvalue > 1e-3


def test_p5_event_e1_rate():
    """Pr[min_i ||H_i(o) - H_i(q)|| <= eps s] = 1 - alpha1^L = 1 - 1/e."""
    d, L, K = 32, 4, 16
    eps = O.epsilon(L, K)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(d)
    s = math.sqrt(x @ x)
    trials, hits = 10_000, 0
    for seed in range(trials):
        A = synth.projection_matrix(L, K, d, 50_000 + seed)
        p = O.project(x[None, :], A)[0].reshape(L, K)
        hits += int(np.sqrt((p * p).sum(axis=1)).min() <= eps * s)
    p0 = 1.0 - math.exp(-1.0)
    lo, hi = stats.binom.interval(0.999, trials, p0)
    assert lo <= hits <= hi, (hits / trials, p0)


# --------------------------------------------------------------------------
# P6: Theorem 2 success probability
# --------------------------------------------------------------------------

def test_p6_c2_k_ann_guarantee():
    c, k, beta = 1.5, 10, 0.1
    ok = total = 0
    for seed in range(4):
        X, idx, _ = make_problem(n=2000, d=32, K=16, N_r=64, frac=0.2, seed=20 + seed)
        Q = synth.gaussian_mixture(10, 32, 8, 3.0, 1.0, 500 + 20 + seed, rows_seed=900 + seed)
        for q in Q:
            qp = O.project(q[None, :], idx.A)[0]
            r = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, k, beta)
            _, dstar = brute_ids(X, q, k)
            ok += int(np.all(r.dists <= c * c * dstar * (1 + 1e-12)))
            total += 1
    assert ok / total >= 0.5 - 1.0 / math.e
    assert ok / total >= 0.9          # observed success is far above the bound


# --------------------------------------------------------------------------
# P7: Lemma 3 / Eq. 2 closed forms and the shape of Fig. 4
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L", range(1, 9))
def test_p7_epsilon_and_beta_closed_form(L):
    K, c = 16, 1.5
    eps2 = chi2_isf_even(math.exp(-1.0 / L), K)
    assert O.epsilon(L, K) == pytest.approx(math.sqrt(eps2), rel=1e-9)
    alpha2 = chi2_sf_even(eps2 / (c * c), K)
    assert O.beta_theory(L, K, c) == pytest.approx(2 - 2 * alpha2 ** L, rel=1e-8)


def test_p7_beta_drops_fast_until_four_trees():
    b = [O.beta_theory(L, 16, 1.5) for L in range(1, 9)]
    assert all(x > y for x, y in zip(b, b[1:]))
    assert (b[0] - b[3]) > 3 * (b[3] - b[7])


def test_p7_n_stop():
    assert O.n_stop(1_000_000, 10, 0.1) == 100_010
    assert O.n_stop(10_000_000, 100, 0.05) == 500_100
    assert O.n_stop(10, 3, 0.15) == 5             # ceil(1.5) = 2


# --------------------------------------------------------------------------
# P8 / P11: breakpoints
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_s,N_r", [(1000, 16), (1024, 256), (777, 64), (4096, 256)])
def test_p8_equal_frequency_on_the_sample(n_s, N_r):
    rng = np.random.default_rng(n_s + N_r)
    Ps = rng.standard_normal((n_s, 3)) * [1.0, 10.0, 0.01]
    B = O.breakpoints_by_sort(Ps, N_r)
    assert np.all(np.diff(B, axis=1) >= 0)
    assert np.array_equal(B[:, 0], Ps.min(axis=0))
    assert np.array_equal(B[:, -1], Ps.max(axis=0))
    assert check_equal_frequency(Ps, B)


def test_p8_encode_matches_the_counting_definition():
    rng = np.random.default_rng(3)
    Ps = rng.standard_normal((300, 2))
    B = O.breakpoints_by_sort(Ps, 16)
    vals = np.concatenate([Ps[:, 0], B[0], [-50.0, 50.0]])      # ties with breakpoints
    codes = O.encode(np.stack([vals, vals], 1), np.stack([B[0], B[0]]))[:, 0]
    for v, cde in zip(vals, codes):
        assert cde == sum(1 for z in range(2, 17) if B[0][z - 1] <= v)
    order = np.argsort(vals, kind="stable")
    assert np.all(np.diff(codes[order].astype(int)) >= 0)      # monotone in h


@pytest.mark.parametrize("n_s,N_r", [(512, 16), (1024, 64), (1000, 8), (2048, 256)])
def test_p11_quickselect_rounds_equal_the_sorted_ranks(n_s, N_r):
    rng = np.random.default_rng(n_s * 7 + N_r)
    Ps = rng.standard_normal((n_s, 2))
    np.testing.assert_array_equal(O.breakpoints_by_quickselect(Ps, N_r),
                                  O.breakpoints_by_sort(Ps, N_r))


# --------------------------------------------------------------------------
# P9: monotone candidate sets, tree partition, tree walk equals flat predicate
# --------------------------------------------------------------------------

def test_p9_tree_partition_and_boxes():
    X, idx, _ = make_problem(n=3000, K=8, N_r=16, seed=8)
    bits = 4
    trees = O.build_trees(idx.codes, idx.L, idx.K, idx.N_r, max_leaf=24)
    for i, leaves in enumerate(trees):
        codes_i = idx.codes[:, i * idx.K:(i + 1) * idx.K].astype(int)
        allids = np.concatenate([lf.ids for lf in leaves])
        assert np.array_equal(np.sort(allids), np.arange(len(X)))
        for lf in leaves:
            assert len(lf.ids) <= 24 or np.all(lf.plen == bits)
            assert np.all(codes_i[lf.ids] >= lf.lo) and np.all(codes_i[lf.ids] <= lf.hi)
            assert np.all(lf.plen >= 1)


# A hand-worked DE-Tree (Sec. 4.2, Alg. 3): N_r = 4 (two bits per code), K = 3,
# max_leaf = 3.  Points 0..11 share the root child whose first-bit vector is
# 000 (codes 0 or 1); point 12 (codes 2, 3, 2) is alone in root child 111.
# Worked by hand with "the dimension whose next bit divides the node most
# evenly, ties to the lowest dimension":
#   root child 000, 12 points: next-bit ones 6, 6, 4 -> |2*ones - 12| = 0, 0, 4
#     -> dimension 0 (tie with dimension 1 goes to the lower one)
#   c0 = 0 {0..5}: ones in dimensions 1, 2 = 1, 3 -> gaps 4, 0 -> dimension 2
#     -> {0,1,2} and {3,4,5}, both within max_leaf
#   c0 = 1 {6..11}: ones 5, 1 -> gaps 4, 4 -> tie -> dimension 1
#     -> {11}, and {6..10} (5 points) whose only open dimension is 2
#        -> {7,8,9,10} (every prefix complete: a leaf despite its size), {6}
# Leaves come root child by root child, depth first, 0-branch first.
HAND_CODES = np.array([
    [0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 1], [0, 0, 1], [0, 1, 1],
    [1, 1, 1], [1, 1, 0], [1, 1, 0], [1, 1, 0], [1, 1, 0], [1, 0, 0],
    [2, 3, 2]], dtype=np.uint8)
HAND_LEAVES = [   # (ids, lo codes, hi codes)
    ([0, 1, 2], [0, 0, 0], [0, 1, 0]),
    ([3, 4, 5], [0, 0, 1], [0, 1, 1]),
    ([11], [1, 0, 0], [1, 0, 1]),
    ([7, 8, 9, 10], [1, 1, 0], [1, 1, 0]),
    ([6], [1, 1, 1], [1, 1, 1]),
    ([12], [2, 2, 2], [3, 3, 3]),
]


def hand_tree_matches():
    leaves = O.build_tree(HAND_CODES, N_r=4, max_leaf=3)
    got = [(lf.ids.tolist(), lf.lo.tolist(), lf.hi.tolist()) for lf in leaves]
    return got == HAND_LEAVES


def test_p9_split_on_the_most_even_dimension_hand_worked():
    assert hand_tree_matches()


def test_planted_split_on_least_even_dimension_is_caught(monkeypatch):
    def least_even(open_dims, ones, size):
        gaps = [abs(2 * c - size) for c in ones]
        return open_dims[int(np.argmax(gaps))]
    monkeypatch.setattr(O, "most_even_dimension", least_even)
    assert not hand_tree_matches()


def test_planted_split_tie_to_highest_dimension_is_caught(monkeypatch):
    def highest_on_tie(open_dims, ones, size):
        gaps = [abs(2 * c - size) for c in ones]
        g = min(gaps)
        return [j for j, x in zip(open_dims, gaps) if x == g][-1]
    monkeypatch.setattr(O, "most_even_dimension", highest_on_tie)
    assert not hand_tree_matches()


def test_p9_candidate_sets_grow_with_radius():
    X, idx, _ = make_problem(n=1500, seed=9)
    qp = O.project((X[5] + 0.3)[None, :], idx.A)[0]
    lb = O.lower_bounds(qp, idx.codes, idx.B, idx.L, idx.K)
    for r2 in np.quantile(lb[:, 0], [0.01, 0.05, 0.2]):
        s1 = set(np.flatnonzero(lb[:, 0] <= r2))
        s2 = set(np.flatnonzero(lb[:, 0] <= r2 * 1.5 ** 2))
        assert s1 <= s2


@pytest.mark.parametrize("max_leaf", [4, 32, 10_000])
def test_tree_walk_equals_flat_predicate(max_leaf):
    """Alg. 4/5 over the built tree returns exactly {o : LB_i^2(o) <= r'^2}."""
    X, idx, _ = make_problem(n=1500, K=6, N_r=16, seed=10)
    trees = O.build_trees(idx.codes, idx.L, idx.K, idx.N_r, max_leaf=max_leaf)
    for q in (X[1] + 0.4, X[77] - 0.2):
        qp = O.project(q[None, :], idx.A)[0]
        lb = O.lower_bounds(qp, idx.codes, idx.B, idx.L, idx.K)
        for i in range(idx.L):
            sl = slice(i * idx.K, (i + 1) * idx.K)
            for r2 in np.quantile(lb[:, i], [0.02, 0.1, 0.5]):
                got = O.range_query_tree(trees[i], qp[sl], idx.codes[:, sl], idx.B[sl], r2)
                assert np.array_equal(got, np.flatnonzero(lb[:, i] <= r2))


# --------------------------------------------------------------------------
# P10 / P13: the magic radius and the printed radius ladder
# --------------------------------------------------------------------------

@pytest.mark.parametrize("c", [1.5, 2.0])
def test_p10_magic_radius_conditions(c):
    X, idx, _ = make_problem(n=2000, seed=11)
    eps = O.epsilon(idx.L, idx.K)
    k, beta = 10, 0.1
    N_S = O.n_stop(len(X), k, beta)
    for q in X[:5] + 0.2:
        qp = O.project(q[None, :], idx.A)[0]
        r = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, k, beta)
        r_min = math.sqrt(r.thr) / eps
        m2 = O.lower_bounds(qp, idx.codes, idx.B, idx.L, idx.K).min(axis=1)
        assert (m2 <= (eps * r_min) ** 2 * (1 + 1e-12)).sum() >= N_S
        assert (m2 <= (eps * r_min / c) ** 2).sum() < N_S


@pytest.mark.parametrize("kind", ["mixture", "integer"])
def test_magic_equals_printed_loop_from_magic_radius(kind):
    X, idx, _ = make_problem(n=1500, seed=12, kind=kind)
    eps = O.epsilon(idx.L, idx.K)
    for q in X[:5] + 0.3:
        qp = O.project(q[None, :], idx.A)[0]
        m = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 10, 0.1)
        r_min = math.sqrt(m.thr) / eps * (1 + 1e-12)
        f = O.query_fixed(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 10, 0.1, 1.5, r_min, eps)
        assert f.rounds == 1 and f.stop_cond == 1
        assert f.stop_tree == m.stop_tree
        assert np.array_equal(f.S, m.S) and np.array_equal(f.ids, m.ids)


@pytest.mark.parametrize("c", [1.5, 2.0])
def test_p13_ladder_equals_entry_step_order(c):
    X, idx, _ = make_problem(n=1500, seed=13)
    eps = O.epsilon(idx.L, idx.K)
    for q in X[:4] + 0.25:
        qp = O.project(q[None, :], idx.A)[0]
        m = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 10, 0.1)
        r_min = math.sqrt(m.thr) / eps / 40.0
        f = O.query_fixed(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 10, 0.1, c, r_min, eps)
        assert f.rounds >= 2
        lb = O.lower_bounds(qp, idx.codes, idx.B, idx.L, idx.K)
        steps = O.entry_steps(lb, eps, r_min, c, idx.L, f.rounds + 1)
        s_star = (f.rounds - 1) * idx.L + f.stop_tree
        assert np.array_equal(f.S, np.flatnonzero(steps <= s_star))
        if f.stop_cond == 1:                 # it had not stopped one step earlier
            assert (steps <= s_star - 1).sum() < O.n_stop(len(X), 10, 0.1)


def test_fixed_stops_on_condition_two_for_tight_clusters():
    """With beta near 1, condition 1 cannot fire early; the ladder stops when k
    candidates lie within c r (line 10 of the printed algorithm)."""
    X, idx, _ = make_problem(n=800, seed=14)
    eps = O.epsilon(idx.L, idx.K)
    q = X[3] + 0.01
    qp = O.project(q[None, :], idx.A)[0]
    f = O.query_fixed(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 5, 0.99, 1.5, 0.05, eps)
    assert f.stop_cond == 2
    d = np.sqrt(O.sq_dists(X[f.S], q))
    r_last = 0.05 * 1.5 ** (f.rounds - 1)
    assert (d <= 1.5 * r_last).sum() >= 5


# --------------------------------------------------------------------------
# planted mistakes: each must be caught by one of the pins above
# --------------------------------------------------------------------------

# --------------------------------------------------------------------------
# the quality measures of Sec. 6.1 (recall, overall ratio)
# --------------------------------------------------------------------------

def test_measures_hand_worked():
    """recall = |R cap R*| / k and overall ratio = mean of ||q,o_i|| / ||q,o_i*||,
    worked by hand: R* at distances 1, 2, 3; R at 1, 2, 4 shares two points
    (recall 2/3) and has ratios 1, 1, 4/3 (mean 10/9)."""
    assert O.recall([1.0, 2.0, 4.0], [1.0, 2.0, 3.0]) == pytest.approx(2 / 3)
    assert O.overall_ratio([1.0, 2.0, 4.0], [1.0, 2.0, 3.0]) == pytest.approx(10 / 9)
    # an exact answer
    assert O.recall([0.5, 0.7], [0.5, 0.7]) == 1.0
    assert O.overall_ratio([0.5, 0.7], [0.5, 0.7]) == 1.0
    # ties at the k-th distance (R16): another point at the k-th distance counts
    assert O.recall([1.0, 2.0, 2.0], [1.0, 2.0, 2.0]) == 1.0
    assert O.recall([1.0, 2.0, 2.0, 2.0], [1.0, 1.5, 2.0, 2.0]) == 1.0
    # a duplicate of the query: 0/0 counts as 1, x/0 as infinity
    assert O.overall_ratio([0.0, 1.0], [0.0, 1.0]) == 1.0
    assert math.isinf(O.overall_ratio([0.1, 1.0], [0.0, 1.0]))
    # a farther answer never has a ratio below 1 or a recall above 1
    rng = np.random.default_rng(3)
    for _ in range(50):
        ref = np.sort(rng.random(10))
        ret = np.sort(ref + rng.random(10) * rng.integers(0, 2, 10))
        assert O.overall_ratio(ret, ref) >= 1.0 and O.recall(ret, ref) <= 1.0


def test_measures_of_the_oracle_answer_against_brute_force():
    """With beta = 1 the oracle's answer is the exact k-NN: recall 1 and ratio 1
    against brute force; at a small beta both stay within their ranges and the
    answer of a worse method (every other point of the exact 2k-NN) is
    measured worse."""
    X, idx, _ = make_problem(n=1200, d=16, seed=11)
    q = X[5] + 0.1
    qp = O.project(q[None, :], idx.A)[0]
    k = 10
    ref_ids, ref_d2 = O.brute_force_knn(X, q, k)
    full = O.query_magic(X, q, qp, idx.codes, idx.B, 4, 8, k, 1.0)
    assert O.recall(full.dists, np.sqrt(ref_d2)) == 1.0
    assert O.overall_ratio(full.dists, np.sqrt(ref_d2)) == pytest.approx(1.0)
    ids2k, d2k = O.brute_force_knn(X, q, 2 * k)
    worse = np.sqrt(d2k[1::2])
    assert O.recall(worse, np.sqrt(ref_d2)) == pytest.approx(0.5)
    assert O.overall_ratio(worse, np.sqrt(ref_d2)) > 1.0


def test_planted_inverted_ratio_is_caught(monkeypatch):
    monkeypatch.setattr(O, "overall_ratio", lambda a, b: float(np.mean(np.asarray(b) / np.asarray(a))))
    with pytest.raises(AssertionError):
        test_measures_hand_worked()


def test_planted_recall_by_rank_is_caught(monkeypatch):
    """Counting hits rank by rank (ret_i <= ref_i) instead of against the k-th
    reference distance misses returned points that are in R* out of order."""
    monkeypatch.setattr(O, "recall", lambda a, b: float(np.mean(np.asarray(a) <= np.asarray(b))))
    with pytest.raises(AssertionError):
        test_measures_hand_worked()


def test_planted_encode_tie_side_is_caught(monkeypatch):
    rng = np.random.default_rng(1)
    Ps = rng.standard_normal((1000, 2))
    B = O.breakpoints_by_sort(Ps, 16)
    real = np.searchsorted

    def wrong(a, v, side="left", sorter=None):
        return real(a, v, side="left", sorter=sorter)
    monkeypatch.setattr(O.np, "searchsorted", wrong)
    assert not check_equal_frequency(Ps, B)


def test_planted_rank_off_by_one_is_caught(monkeypatch):
    rng = np.random.default_rng(2)
    Ps = rng.standard_normal((1000, 2))
    real = O.breakpoint_ranks
    monkeypatch.setattr(O, "breakpoint_ranks", lambda n_s, N_r: np.minimum(real(n_s, N_r) + 1, n_s))
    assert not check_equal_frequency(Ps, O.breakpoints_by_sort(Ps, 16))


def test_planted_closed_region_ends_are_caught(monkeypatch):
    X, idx, _ = make_problem(n=800, frac=0.05, seed=15)
    far = (X[:4] * 5.0).astype(np.float32)
    Xall = np.vstack([X, far])
    idx2 = O.Index(idx.A, idx.B, O.encode(O.project(Xall, idx.A), idx.B), idx.L, idx.K, idx.N_r)

    def closed(B):
        B = np.asarray(B, np.float64)
        return B[:, :-1].copy(), B[:, 1:].copy()
    monkeypatch.setattr(O, "region_bounds", closed)
    assert not check_lb_invariant(Xall, [far[0] * 1.1, X[0]], idx2)


def test_planted_gap_sign_is_caught(monkeypatch):
    X, idx, _ = make_problem(n=600, seed=16)

    def wrong(qp, B):
        lo, hi = O.region_bounds(B)
        q = np.asarray(qp, np.float64)[:, None]
        gap = np.maximum(0.0, np.maximum(q - lo, hi - q))
        return gap * gap
    monkeypatch.setattr(O, "lb_tables", wrong)
    assert not check_lb_invariant(X, [X[0] + 0.1], idx)


def test_planted_tie_order_is_caught(monkeypatch):
    X, idx, _ = make_problem(n=400, seed=17, kind="integer")
    q = X[0] + 0.0
    monkeypatch.setattr(O, "top_k", lambda ids, d2, k: (
        np.asarray(ids)[np.lexsort((-np.asarray(ids), d2))[:k]],
        np.sort(np.asarray(d2, np.float64))[:k]))
    qp = O.project(q[None, :], idx.A)[0]
    r = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, k=10, beta=1.0)
    ids, _ = brute_ids(X, q, 10)
    assert not np.array_equal(r.ids, ids)


def test_planted_wrong_code_column_is_caught(monkeypatch):
    """Every tree reading the first tree's code columns (a wrong index) changes
    S, which the printed-loop equivalence pin detects."""
    X, idx, _ = make_problem(n=1500, seed=18)
    q = X[2] + 0.3
    qp = O.project(q[None, :], idx.A)[0]

    def wrong(qp_, codes, B, L, K):
        T = O.lb_tables(qp_, B)
        out = np.zeros((codes.shape[0], L))
        for i in range(L):
            for j in range(K):
                out[:, i] += T[i * K + j, codes[:, j]]
        return out
    monkeypatch.setattr(O, "lower_bounds", wrong)
    m = O.query_magic(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 10, 0.1)
    monkeypatch.undo()
    eps = O.epsilon(idx.L, idx.K)
    f = O.query_fixed(X, q, qp, idx.codes, idx.B, idx.L, idx.K, 10, 0.1, 1.5,
                      math.sqrt(m.thr) / eps * (1 + 1e-12), eps)
    assert not np.array_equal(f.S, m.S)
