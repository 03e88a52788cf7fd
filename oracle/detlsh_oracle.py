"""Plain, slow FP64 CPU oracle of DET-LSH (Wei, Peng, Lee, Palpanas; PVLDB 17(9), 2024).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run this module.  It shares
no code, table or constant with the HIP library; the two meet only through the
seeded inputs of ``synth`` (data, queries, the projection matrix and the
breakpoint sample ids, which are passed in as inputs).

Everything is float64 NumPy.  Every function follows one passage of the paper:

  project                 Eq. 1 (Sec. 3.2) and the L*K hashes of Sec. 4.1
  breakpoints_by_sort     Sec. 4.1, dynamic encoding: equal-frequency ranks of the
                          sorted sample (reading R3 for ranks when N_r does not
                          divide n_s)
  breakpoints_by_quickselect
                          Alg. 1, divide-and-conquer QuickSelect rounds
  encode                  Alg. 2 with the upper-bound reading of the region test (R4)
  region_bounds / lb_tables / lower_bounds
                          Sec. 4.3, bounds from the breakpoints around a region
                          (readings R5, R6: point-to-box distance, open ends)
  build_trees             Alg. 3 and the split rule of Sec. 4.2 (bulk-built, R15)
  range_query_tree        Alg. 4 / Alg. 5 over a built tree (R7 point predicate)
  query_magic             Alg. 7 started at the smallest radius satisfying both
                          conditions of the "magic" r_min of Sec. 5.2 (R10)
  query_fixed             Alg. 7 literally, from a caller-given r_min
  query_magic_leaf        Alg. 7 with the query-phase optimisation of the
                          experiments (leaves admitted whole by their bound, in
                          bound order, condition 1 checked after every leaf)
  query_rc                Alg. 6, the (r, c)-ANN query with one search radius
  insert                  points added after the encoding phase (Alg. 3 inserts
                          point by point; the breakpoints stay as built)
  paa_matrix              PAA segment means of DET-ONLY (Sec. 6.1), the L = 1
                          projection that replaces the Gaussian hashes
  epsilon, beta_theory    Lemma 3 / Eq. 2
  brute_force_knn         Def. 2 with o_i* exact; ties broken by id (R13)
  recall, overall_ratio   the two quality measures of Sec. 6.1 (ties: R16)

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# --------------------------------------------------------------------------
# parameters (Lemma 3, Eq. 2)
# --------------------------------------------------------------------------


def chi2_upper_quantile(alpha: float, K: int) -> float:
    """chi^2_alpha(K): the x with Pr[Y > x] = alpha for Y ~ chi^2(K) (Lemma 2)."""
    from scipy.stats import chi2
    return float(chi2.isf(alpha, K))


def epsilon(L: int, K: int) -> float:
    """eps = sqrt(chi^2_{alpha1}(K)) with alpha1 = e^{-1/L}, i.e. L = -1/ln alpha1
    (Lemma 3, Eq. 2)."""
    return math.sqrt(chi2_upper_quantile(math.exp(-1.0 / L), K))


def beta_theory(L: int, K: int, c: float) -> float:
    """beta = 2 - 2 alpha2^L where chi^2_{alpha2}(K) = eps^2 / c^2 (Lemma 3)."""
    from scipy.stats import chi2
    eps2 = epsilon(L, K) ** 2
    alpha2 = float(chi2.sf(eps2 / (c * c), K))
    return 2.0 - 2.0 * alpha2 ** L


def n_stop(n: int, k: int, beta: float) -> int:
    """Termination size |S| >= beta*n + k of Alg. 7, as an integer: k + ceil(beta*n)
    evaluated in IEEE double (reading R9)."""
    return int(k + math.ceil(beta * n))


# --------------------------------------------------------------------------
# encoding phase (Sec. 4.1)
# --------------------------------------------------------------------------


def project(X, A):
    """H(o) = [h_11(o), ..., h_LK(o)] with h(o) = a . o (Eq. 1); column i*K + j."""
    return np.asarray(X, np.float64) @ np.asarray(A, np.float64).T


def breakpoint_ranks(n_s: int, N_r: int) -> np.ndarray:
    """1-indexed sample ranks of B(z), z = 1..N_r+1: max(1, floor((z-1) n_s / N_r)).
    Equals the rank floor(n/N_r)(z-1) of Sec. 4.1 whenever N_r divides n_s, gives
    B(1) = minimum and B(N_r+1) = maximum (reading R3)."""
    z = np.arange(1, N_r + 2, dtype=np.int64)
    return np.maximum(1, ((z - 1) * int(n_s)) // int(N_r))


def breakpoints_by_sort(Ps, N_r: int) -> np.ndarray:
    """Equal-frequency breakpoints of each projected dimension from the sorted
    sample (Sec. 4.1).  Ps: (n_s, L*K) projected sample.  Returns B with shape
    (L*K, N_r+1), B[e, z-1] = B_e(z)."""
    Ps = np.asarray(Ps, np.float64)
    n_s = Ps.shape[0]
    srt = np.sort(Ps, axis=0)
    r = breakpoint_ranks(n_s, N_r)
    return np.ascontiguousarray(srt[r - 1, :].T)


def _quickselect(a: np.ndarray, lo: int, hi: int, t: int) -> None:
    """Rearrange a[lo:hi] so that a[t] holds the value it would hold if a[lo:hi]
    were sorted, everything left of t is <= a[t] and everything right is >= a[t]
    (Hoare's selection with Lomuto partitions, middle pivot)."""
    while hi - lo > 1:
        mid = (lo + hi - 1) // 2
        a[mid], a[hi - 1] = a[hi - 1], a[mid]
        pivot = a[hi - 1]
        store = lo
        for i in range(lo, hi - 1):
            if a[i] < pivot:
                a[i], a[store] = a[store], a[i]
                store += 1
        a[store], a[hi - 1] = a[hi - 1], a[store]
        if t == store:
            return
        if t < store:
            hi = store
        else:
            lo = store + 1


def breakpoints_by_quickselect(Ps, N_r: int) -> np.ndarray:
    """Alg. 1: for every projected dimension, log2(N_r) rounds; round z runs one
    QuickSelect inside each of the 2^(z-1) sub-regions left by round z-1, taking
    the q-th smallest element with q = ceil(size/2) (the lower median), which
    becomes the breakpoint between the sub-region's two halves.  B(1) is the
    minimum of the first floor(n_s/N_r) elements and B(N_r+1) the maximum of
    the last ones.  Pure Python: for small samples only."""
    Ps = np.asarray(Ps, np.float64)
    n_s, m = Ps.shape
    rounds = int(round(math.log2(N_r)))
    if 1 << rounds != N_r:
        raise ValueError("N_r must be a power of two")
    B = np.empty((m, N_r + 1))
    frs = n_s // N_r
    for e in range(m):
        c = [float(v) for v in Ps[:, e]]
        # (start, end, z_lo, z_hi): positions [start, end) hold the elements that
        # lie strictly between breakpoints B(z_lo) and B(z_hi)
        regions = [(0, n_s, 1, N_r + 1)]
        for _ in range(rounds):
            nxt = []
            for (s, t, zl, zh) in regions:
                zm = (zl + zh) // 2
                size = t - s
                if size == 0:
                    raise ValueError("sample too small for N_r regions")
                q = (size + 1) // 2          # 1-indexed within the sub-region
                pos = s + q - 1
                _quickselect(c, s, t, pos)
                B[e, zm - 1] = c[pos]
                nxt.append((s, pos, zl, zm))
                nxt.append((pos + 1, t, zm, zh))
            regions = nxt
        B[e, 0] = min(c[0:max(frs, 1)])
        B[e, N_r] = max(c[n_s - max(frs, 1) - 1:n_s])
    return B


def encode(P, B) -> np.ndarray:
    """Alg. 2: the region of h among the N_r regions cut by the breakpoints.
    Reading R4: code = #{z in 2..N_r : B(z) <= h}, i.e. a value equal to a
    breakpoint belongs to the upper region, values below B(2) get 0 and values
    at or above B(N_r) get N_r - 1.  P: (n, L*K), B: (L*K, N_r+1).  Returns
    uint8 (n, L*K) for N_r <= 256, uint16 otherwise."""
    P = np.asarray(P, np.float64)
    B = np.asarray(B, np.float64)
    N_r = B.shape[1] - 1
    out = np.empty(P.shape, np.uint8 if N_r <= 256 else np.uint16)
    for e in range(P.shape[1]):
        interior = B[e, 1:N_r]              # B(2) .. B(N_r), non-decreasing
        out[:, e] = np.searchsorted(interior, P[:, e], side="right")
    return out


# --------------------------------------------------------------------------
# bounds (Sec. 4.3)
# --------------------------------------------------------------------------


def region_bounds(B) -> tuple[np.ndarray, np.ndarray]:
    """[lo_b, hi_b] of region b = 0..N_r-1 for every dimension: lo_b = B(b+1),
    hi_b = B(b+2), except that region 0 is open below and region N_r-1 open
    above (reading R5), so that out-of-sample values keep a valid bound."""
    B = np.asarray(B, np.float64)
    lo = B[:, :-1].copy()
    hi = B[:, 1:].copy()
    lo[:, 0] = -np.inf
    hi[:, -1] = np.inf
    return lo, hi


def lb_tables(qp, B) -> np.ndarray:
    """T[e, b] = squared gap between the projected query coordinate qp[e] and
    region b of dimension e: max(0, lo - q, q - hi)^2 (reading R6)."""
    lo, hi = region_bounds(B)
    q = np.asarray(qp, np.float64)[:, None]
    gap = np.maximum(0.0, np.maximum(lo - q, q - hi))
    return gap * gap


def lower_bounds(qp, codes, B, L: int, K: int) -> np.ndarray:
    """LB_i^2(q, o) for every point o and tree i: the squared distance from
    H_i(q) to the cell of o in the i-th projected space, summed over j in
    ascending order.  Returns (n, L)."""
    T = lb_tables(qp, B)
    codes = np.asarray(codes)
    n = codes.shape[0]
    out = np.zeros((n, L))
    for i in range(L):
        acc = np.zeros(n)
        for j in range(K):
            e = i * K + j
            acc = acc + T[e, codes[:, e]]
        out[:, i] = acc
    return out


def node_lb2(qp_i, lo_code, hi_code, B_i) -> float:
    """Squared distance from the projected query (one tree, K values) to the box
    spanned by regions lo_code[j]..hi_code[j] of every dimension j (R6)."""
    lo, hi = region_bounds(B_i)
    s = 0.0
    for j in range(len(qp_i)):
        a = lo[j, lo_code[j]]
        b = hi[j, hi_code[j]]
        g = max(0.0, a - qp_i[j], qp_i[j] - b)
        s += g * g
    return s


def node_ub2(qp_i, lo_code, hi_code, B_i) -> float:
    """Squared farthest distance from the projected query to that box; infinite
    when the box reaches an open end."""
    lo, hi = region_bounds(B_i)
    s = 0.0
    for j in range(len(qp_i)):
        a = lo[j, lo_code[j]]
        b = hi[j, hi_code[j]]
        g = max(abs(qp_i[j] - a), abs(qp_i[j] - b))
        s += g * g
    return s


# --------------------------------------------------------------------------
# indexing phase (Alg. 3, Sec. 4.2)
# --------------------------------------------------------------------------


@dataclass
class Leaf:
    ids: np.ndarray       # point ids, ascending
    lo: np.ndarray        # per-dimension lowest region code of the node
    hi: np.ndarray        # per-dimension highest region code of the node
    plen: np.ndarray      # per-dimension prefix length in bits


def most_even_dimension(open_dims, ones, size: int) -> int:
    """The split dimension of an overfull node (Sec. 4.2): among the dimensions
    whose prefix is not yet complete, the one whose next bit divides the
    node's ``size`` points most evenly, i.e. with the smallest |#ones - #zeros|
    = |2 ones - size|; ties go to the lowest dimension (reading R15)."""
    best, best_gap = None, None
    for j, c in zip(open_dims, ones):
        gap = abs(2 * c - size)
        if best is None or gap < best_gap:
            best, best_gap = j, gap
    return best


def build_tree(codes_i, N_r: int, max_leaf: int) -> list[Leaf]:
    """One DE-Tree over the K-dimensional codes of one projected space.

    The root has 2^K children, one per combination of the first bit (0* / 1*)
    of every dimension (Alg. 3).  A node holding more than ``max_leaf`` points
    is split in two on the one dimension whose next prefix bit divides its
    points most evenly (Sec. 4.2), ties to the lowest dimension; a node whose
    prefixes are all complete stays a leaf whatever its size.  Bulk-built over
    all points (reading R15).  Leaves are returned root child by root child in
    ascending order of the first-bit vector (dimension 0 most significant), and
    inside a root child depth first, the 0-branch before the 1-branch."""
    codes_i = np.asarray(codes_i).astype(np.int64)
    n, K = codes_i.shape
    bits = int(round(math.log2(N_r)))
    leaves: list[Leaf] = []

    def visit(ids, plen):
        size = len(ids)
        open_dims = [j for j in range(K) if plen[j] < bits]
        if size <= max_leaf or not open_dims:
            first = codes_i[ids[0]]
            lo = np.array([(first[j] >> (bits - plen[j])) << (bits - plen[j]) for j in range(K)])
            hi = lo + (1 << (bits - plen)) - 1
            leaves.append(Leaf(np.sort(ids), lo, hi, plen.copy()))
            return
        ones = [int(((codes_i[ids, j] >> (bits - 1 - plen[j])) & 1).sum()) for j in open_dims]
        best = most_even_dimension(open_dims, ones, size)
        bit = (codes_i[ids, best] >> (bits - 1 - plen[best])) & 1
        child = plen.copy()
        child[best] += 1
        zeros, ones = ids[bit == 0], ids[bit == 1]
        if len(zeros):
            visit(zeros, child)
        if len(ones):
            visit(ones, child)

    msb = (codes_i >> (bits - 1)) & 1
    weights = 1 << np.arange(K - 1, -1, -1, dtype=np.int64)
    root_key = (msb * weights).sum(axis=1)
    order = np.argsort(root_key, kind="stable")
    keys = root_key[order]
    starts = np.flatnonzero(np.r_[True, keys[1:] != keys[:-1]])
    ends = np.r_[starts[1:], n]
    for s, t in zip(starts, ends):
        visit(order[s:t], np.ones(K, np.int64))
    return leaves


def build_trees(codes, L: int, K: int, N_r: int, max_leaf: int) -> list[list[Leaf]]:
    codes = np.asarray(codes)
    return [build_tree(codes[:, i * K:(i + 1) * K], N_r, max_leaf) for i in range(L)]


def range_query_tree(leaves: list[Leaf], qp_i, codes_i, B_i, radius2: float) -> np.ndarray:
    """Alg. 4 / Alg. 5 over one tree: a node (here a leaf run, whose box is its
    prefix box) is pruned when its lower bound exceeds the radius; a leaf whose
    upper bound is within the radius contributes all its points; otherwise
    each point is admitted when its own cell bound is within the radius (R7).
    All comparisons are on squared distances.  Returns sorted ids."""
    lo_b, hi_b = region_bounds(B_i)
    out = []
    qp_i = np.asarray(qp_i, np.float64)
    for lf in leaves:
        if node_lb2(qp_i, lf.lo, lf.hi, B_i) > radius2:
            continue
        if node_ub2(qp_i, lf.lo, lf.hi, B_i) <= radius2:
            out.extend(lf.ids.tolist())
            continue
        for o in lf.ids:
            s = 0.0
            for j in range(len(qp_i)):
                b = int(codes_i[o, j])
                g = max(0.0, lo_b[j, b] - qp_i[j], qp_i[j] - hi_b[j, b])
                s += g * g
            if s <= radius2:
                out.append(int(o))
    return np.array(sorted(out), np.int64)


# --------------------------------------------------------------------------
# query phase (Alg. 7, Sec. 5.2)
# --------------------------------------------------------------------------


def sq_dists(X, q) -> np.ndarray:
    """Exact squared Euclidean distances by direct differences, float64."""
    diff = np.asarray(X, np.float64) - np.asarray(q, np.float64)[None, :]
    return np.einsum("ij,ij->i", diff, diff)


def top_k(ids, d2, k):
    """The k smallest (d2, id) pairs in ascending order (R13)."""
    ids = np.asarray(ids, np.int64)
    d2 = np.asarray(d2, np.float64)
    order = np.lexsort((ids, d2))[:k]
    return ids[order], d2[order]


def brute_force_knn(X, q, k):
    """Exact k nearest neighbours of q (Def. 2 with c = 1), ties by id."""
    d2 = sq_dists(X, q)
    return top_k(np.arange(len(d2)), d2, k)


def recall(ret_d, ref_d) -> float:
    """Recall of one answer (Sec. 6.1, Evaluation Measures): |R cap R*| / k,
    with R* the reference answer (exact k-NN, or another method's answer)
    given by its k distances.  Reading R16: distances may tie, so a returned
    point counts as in R* when its distance is at most the k-th reference
    distance; the count is capped at k."""
    ret_d = np.asarray(ret_d, np.float64)
    ref_d = np.asarray(ref_d, np.float64)
    k = len(ref_d)
    hit = int(np.sum(ret_d <= ref_d[-1]))
    return min(hit, k) / k


def overall_ratio(ret_d, ref_d) -> float:
    """Overall ratio of one answer (Sec. 6.1): the mean over ranks i of
    ||q, o_i|| / ||q, o_i*||, both lists ascending; a 0/0 term counts as 1
    (reading R16)."""
    ret_d = np.asarray(ret_d, np.float64)
    ref_d = np.asarray(ref_d, np.float64)
    terms = np.where(ref_d > 0, ret_d / np.where(ref_d > 0, ref_d, 1.0),
                     np.where(ret_d > 0, np.inf, 1.0))
    return float(np.mean(terms))


@dataclass
class QueryResult:
    ids: np.ndarray          # k ids, ascending (distance, id)
    dists: np.ndarray        # k Euclidean distances
    S: np.ndarray            # candidate ids, ascending
    thr: float               # squared projected radius (eps r)^2 at the stop
    stop_tree: int           # 1-based tree after which the stop fired (L if cond. 2)
    rounds: int              # radius rounds used (1 under the magic radius)
    first_tree: np.ndarray   # per id in S: the 1-based first tree that admitted it
    stop_cond: int           # 1: |S| >= N_S, 2: k points within c r, 0: S = D


def query_magic(X, q, qp, codes, B, L, K, k, beta):
    """Alg. 7 from the magic initial radius of Sec. 5.2.

    Reading R10: with the point-level predicate LB_i^2(o) <= (eps r)^2 the
    candidate set after all L trees at radius r is {o : m^2(o) <= (eps r)^2}
    with m^2(o) = min_i LB_i^2(o).  The smallest radius with at least N_S =
    beta*n + k candidates is eps r* = sqrt(thr), thr the N_S-th smallest m^2;
    it satisfies both conditions of the magic r_min and Alg. 7 stops in its
    first round, inside the tree loop, at the first tree i* after which the
    union holds N_S points.  If N_S >= n, S = D."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    N_S = n_stop(n, k, beta)
    lb = lower_bounds(qp, codes, B, L, K)          # (n, L)
    if N_S >= n:
        S = np.arange(n)
        ids, d2 = top_k(S, sq_dists(X[S], q), k)
        return QueryResult(ids, np.sqrt(d2), S, math.inf, L, 1,
                           np.ones(n, np.int64), 0)
    m2 = lb.min(axis=1)
    thr = float(np.sort(m2, kind="stable")[N_S - 1])
    admitted = lb <= thr                             # (n, L)
    first = np.where(admitted.any(axis=1), admitted.argmax(axis=1) + 1, L + 1)
    stop = None
    for i in range(1, L + 1):                        # condition 1 after each tree
        if int((first <= i).sum()) >= N_S:
            stop = i
            break
    assert stop is not None
    S = np.flatnonzero(first <= stop)
    ids, d2 = top_k(S, sq_dists(X[S], q), k)
    return QueryResult(ids, np.sqrt(d2), S, thr, stop, 1, first[S], 1)


def leaf_bounds(qp, trees, B, L, K):
    """Per point and tree: the squared bound of the point's leaf box (R6 on the
    leaf's prefix box) and the smallest id of that leaf."""
    n = sum(len(lf.ids) for lf in trees[0])
    lb = np.full((n, L), math.inf)
    leafmin = np.zeros((n, L), np.int64)
    for i in range(L):
        qi, Bi = np.asarray(qp, np.float64)[i * K:(i + 1) * K], B[i * K:(i + 1) * K]
        for lf in trees[i]:
            lb[lf.ids, i] = node_lb2(qi, lf.lo, lf.hi, Bi)
            leafmin[lf.ids, i] = int(lf.ids.min())
    return lb, leafmin


def leaf_queue(qp_i, leaves, B_i, radius2):
    """The admitted leaves of one tree (bound within the radius) in the order a
    priority queue on the bound releases them (ties by smallest point id)."""
    queue = []
    for lf in leaves:
        b = node_lb2(qp_i, lf.lo, lf.hi, B_i)
        if b <= radius2:
            queue.append((b, int(lf.ids.min()), lf.ids))
    queue.sort(key=lambda e: (e[0], e[1]))
    return [ids for _, _, ids in queue]


def query_magic_leaf(X, q, qp, codes, B, trees, L, K, k, beta):
    """Alg. 7 with the optimisation of the query phase: a leaf whose lower
    bound is within the radius contributes all its points (relaxed candidate
    test), the admitted leaves of a tree are taken in ascending order of their
    bound (a priority queue; ties by the leaf's smallest point id), and
    condition 1 is checked after every leaf, so the query can stop inside a
    tree.  Started from the magic radius on leaf bounds (R10 with the leaf box
    in place of the cell): the smallest radius at which the union of admitted
    leaves over the L trees holds N_S points."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    N_S = n_stop(n, k, beta)
    if N_S >= n:
        S = np.arange(n)
        ids, d2 = top_k(S, sq_dists(X[S], q), k)
        return QueryResult(ids, np.sqrt(d2), S, math.inf, L, 1, np.ones(n, np.int64), 0)
    lb, _ = leaf_bounds(qp, trees, B, L, K)
    thr = float(np.sort(lb.min(axis=1), kind="stable")[N_S - 1])
    inS = np.zeros(n, bool)
    first = np.full(n, L + 1, np.int64)
    for i in range(1, L + 1):
        qi, Bi = np.asarray(qp, np.float64)[(i - 1) * K:i * K], B[(i - 1) * K:i * K]
        for ids in leaf_queue(qi, trees[i - 1], Bi, thr):
            new = ids[~inS[ids]]
            inS[new] = True
            first[new] = i
            if int(inS.sum()) >= N_S:
                S = np.flatnonzero(inS)
                top, d2 = top_k(S, sq_dists(X[S], q), k)
                return QueryResult(top, np.sqrt(d2), S, thr, i, 1, first[S], 1)
    raise AssertionError("the magic radius admits N_S points")


def query_fixed(X, q, qp, codes, B, L, K, k, beta, c, r_min, eps=None, max_rounds=10_000):
    """Alg. 7 as printed, from a caller-given initial radius r_min: in round t
    the radius is r = r_min c^t; trees are queried in order with radius eps*r
    and their candidates added to S; the query stops as soon as |S| >= N_S
    (checked after every tree) or, after all L trees, when at least k points of
    S lie within c*r.  Comparisons are on squared values (R7, R12)."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    if eps is None:
        eps = epsilon(L, K)
    N_S = n_stop(n, k, beta)
    lb = lower_bounds(qp, codes, B, L, K)
    d2_all = sq_dists(X, q)
    inS = np.zeros(n, bool)
    first = np.full(n, L + 1, np.int64)
    r = float(r_min)
    for t in range(max_rounds):
        rad2 = (eps * r) ** 2
        for i in range(1, L + 1):
            new = (lb[:, i - 1] <= rad2) & ~inS
            first[new] = i
            inS |= new
            if int(inS.sum()) >= N_S:
                S = np.flatnonzero(inS)
                ids, d2 = top_k(S, d2_all[S], k)
                return QueryResult(ids, np.sqrt(d2), S, rad2, i, t + 1, first[S], 1)
        S = np.flatnonzero(inS)
        if int((d2_all[S] <= (c * r) ** 2).sum()) >= k:
            ids, d2 = top_k(S, d2_all[S], k)
            return QueryResult(ids, np.sqrt(d2), S, rad2, L, t + 1, first[S], 2)
        r *= c
    raise RuntimeError("radius ladder did not terminate")


@dataclass
class RcResult:
    id: int                  # nearest point of S, or -1 when nothing is returned
    dist: float              # its Euclidean distance, or +inf
    S: np.ndarray            # candidate ids at the end, ascending
    stop_tree: int           # tree after which |S| reached beta*n + 1 (0: not reached)
    cond: int                # 1: |S| reached beta*n + 1, 2: a point of S within c r, 0: nothing


def query_rc(X, q, qp, codes, B, L, K, r, c, beta, eps=None):
    """The (r, c)-ANN query of Alg. 6: the L projected spaces are visited in
    order; space i adds every point whose cell lies within eps*r of the
    projected query (the range query of Alg. 4/5 with the R7 predicate); as soon
    as S holds beta*n + 1 points (read as ceil(beta*n) + 1, R9 with k = 1) the
    point of S nearest to q is returned.  After all L spaces, the nearest point
    of S is returned if some point of S lies within c*r of q; otherwise nothing."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    if eps is None:
        eps = epsilon(L, K)
    need = n_stop(n, 1, beta)
    lb = lower_bounds(qp, codes, B, L, K)
    d2 = sq_dists(X, q)
    rad2 = (eps * float(r)) ** 2
    inS = np.zeros(n, bool)
    for i in range(1, L + 1):
        inS |= lb[:, i - 1] <= rad2
        if int(inS.sum()) >= need:
            S = np.flatnonzero(inS)
            ids, dd = top_k(S, d2[S], 1)
            return RcResult(int(ids[0]), float(np.sqrt(dd[0])), S, i, 1)
    S = np.flatnonzero(inS)
    if S.size and bool((d2[S] <= (c * float(r)) ** 2).any()):
        ids, dd = top_k(S, d2[S], 1)
        return RcResult(int(ids[0]), float(np.sqrt(dd[0])), S, 0, 2)
    return RcResult(-1, math.inf, S, 0, 0)


def paa_matrix(d: int, K: int) -> np.ndarray:
    """Piecewise Aggregate Approximation used by DET-ONLY: K segments of
    floor(d/K) consecutive coordinates each; row j averages segment j (the
    d - K*floor(d/K) trailing coordinates belong to no segment).  As a
    projection matrix it turns Eq. 1's h_j(o) = a_j . o into segment means."""
    w = d // K
    if w < 1:
        raise ValueError("PAA needs d >= K")
    A = np.zeros((K, d), np.float64)
    for j in range(K):
        A[j, j * w:(j + 1) * w] = 1.0 / w
    return A


def entry_steps(lb, eps, r_min, c, L, rounds):
    """Entry step e(o) = min_i (t_i(o) L + i), t_i(o) the first round t whose
    radius r_min c^t admits o in tree i (LB_i^2(o) <= (eps r_t)^2), with the
    radii formed as in ``query_fixed`` (r_{t+1} = c r_t).  This is the order in
    which the printed loop of Alg. 7 adds points to S; points admitted in no
    round below ``rounds`` get a step beyond rounds*L."""
    lb = np.asarray(lb, np.float64)
    rad2 = np.empty(rounds)
    r = float(r_min)
    for t in range(rounds):
        rad2[t] = (eps * r) ** 2
        r *= c
    steps = np.full(lb.shape[0], rounds * L + L + 1, np.int64)
    for i in range(1, L + 1):
        t = np.searchsorted(rad2, lb[:, i - 1], side="left")
        ok = t < rounds
        steps[ok] = np.minimum(steps[ok], t[ok] * L + i)
    return steps


# --------------------------------------------------------------------------
# whole index (build) for convenience
# --------------------------------------------------------------------------


@dataclass
class Index:
    A: np.ndarray
    B: np.ndarray
    codes: np.ndarray
    L: int
    K: int
    N_r: int


def insert(idx: Index, X_new) -> Index:
    """Points added after the encoding phase: they are projected with the same
    hashes and encoded against the existing breakpoints (Alg. 2), and their
    codes join the index (the trees, built from codes by Alg. 3, take them in
    like any other point)."""
    new = encode(project(X_new, idx.A), idx.B)
    return Index(idx.A, idx.B, np.concatenate([idx.codes, new]), idx.L, idx.K, idx.N_r)


def build_index(X, A, sample, L, K, N_r):
    """Encoding phase of Sec. 4.1: project, breakpoints from the sampled rows,
    encode every point (trees are built separately by ``build_trees``)."""
    P = project(X, A)
    B = breakpoints_by_sort(P[np.asarray(sample)], N_r)
    codes = encode(P, B)
    return Index(np.asarray(A), B, codes, L, K, N_r)
