"""GPU parity of every step of the hot path against the FP64 oracle, through
the C ABI, on seeded inputs that span several tiles and a ragged tail.

Tolerances: projected coordinates within 1e-5 of the
dot product's magnitude sum_l |a_l o_l|; codes bit-exact except coordinates
that close to a breakpoint (counted); candidate sets bit-exact when fed the
oracle's codes, breakpoints and projected queries, except points whose FP64
bound lies within 1e-5 relative of the stop threshold (counted); ids bit-exact
except distance near-ties; distances within 1e-5 relative.
"""
import numpy as np
import pytest

import gpu_util as U
from oracle import detlsh_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2406_10938_amd as dl
    dl._lib.lib()
    return dl


def say(*a):
    print(*a, flush=True)


def t(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


# --------------------------------------------------------------------------
# step a1: projection (MFMA GEMM)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,d,L,K", [(1000, 128, 4, 16), (777, 100, 4, 16), (513, 37, 2, 8),
                                     (300, 960, 4, 16), (129, 96, 1, 32), (2000, 24, 8, 8),
                                     (700, 64, 4, 12), (300, 40, 2, 5)])
def test_projection_parity(dl, n, d, L, K):
    say(f"projection n={n} d={d} L={L} K={K}")
    c = U.case(n=n, d=d, L=L, K=K, N_r=16, frac=0.2, nq=5, seed=n + d)
    idx = dl.build_index(c["X"], L, K, 16, 0.2, A=c["A"], sample_ids=c["sample"])
    got = idx.project(t(c["X"])).cpu().numpy().astype(np.float64)
    ref = O.project(c["X"], c["A"])
    tol = U.REL * U.proj_scale(c["X"], c["A"])
    assert np.all(np.abs(got - ref) <= tol), np.abs(got - ref).max()


@pytest.mark.parametrize("n,d", [(5000, 128), (3001, 96)])
def test_bf16_projection_close(dl, n, d):
    """The BF16 projection form rounds inputs to BF16 (8-bit mantissa); its
    error is bounded by 2^-8 of the magnitude sum (not a parity claim)."""
    say(f"bf16 projection n={n} d={d}")
    c = U.case(n=n, d=d, N_r=64, frac=0.1, seed=7)
    idx = dl.build_index(c["X"], 4, 16, 64, 0.1, A=c["A"], sample_ids=c["sample"], proj_bf16=True)
    ex = idx.export()
    assert ex["codes"].shape == (n, 64)
    B_ref = O.breakpoints_by_sort(O.project(c["X"], c["A"])[c["sample"]], 64)
    scale = U.proj_scale(c["X"][c["sample"]], c["A"]).max(axis=0)
    assert np.all(np.abs(ex["B"] - B_ref) <= (2.0 ** -7) * scale[:, None])


# --------------------------------------------------------------------------
# steps a2 + a3: breakpoints (sample sort) and codes (binary search in LDS)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,d,N_r,frac,L,K", [(10_000, 128, 256, 0.1, 4, 16), (4097, 64, 64, 0.25, 4, 16),
                                              (3000, 32, 16, 0.1, 2, 8), (2500, 48, 4, 0.05, 8, 4),
                                              (20_000, 16, 256, 0.02, 1, 32), (3000, 48, 64, 0.1, 4, 12),
                                              (2000, 20, 16, 0.1, 8, 3), (3000, 64, 16, 0.1, 1, 4),
                                              (3000, 96, 256, 0.1, 8, 8)])
def test_breakpoints_and_codes(dl, n, d, N_r, frac, L, K):
    say(f"breakpoints/codes n={n} d={d} N_r={N_r} frac={frac} L={L} K={K}")
    c = U.case(n=n, d=d, L=L, K=K, N_r=N_r, frac=frac, seed=n % 97)
    idx = dl.build_index(c["X"], L, K, N_r, frac, A=c["A"], sample_ids=c["sample"])
    ex = idx.export()
    assert np.array_equal(ex["sample_ids"], c["sample"])
    P, B_ref, codes_ref = U.oracle_encoding(c)
    scale = U.proj_scale(c["X"], c["A"])
    colscale = scale[c["sample"]].max(axis=0)
    assert np.all(np.abs(ex["B"] - B_ref) <= U.REL * colscale[:, None])
    assert np.all(np.diff(ex["B"], axis=1) >= 0)
    nbad, hard = U.code_mismatches(P, scale, B_ref, ex["B"].astype(np.float64), codes_ref, ex["codes"])
    say(f"  codes differing: {nbad} of {codes_ref.size}, all within tolerance of a breakpoint: {hard == 0}")
    assert hard == 0


@pytest.mark.parametrize("d", [16, 32, 64, 96])
def test_codes_across_persistent_tiles(dl, d):
    """The encode runs a persistent grid whose workgroups each take several
    512-row tiles once n exceeds 512 x 256 rows; codes past the first tile of
    every workgroup are compared with the oracle's too (n = 200,000).  d = 16
    takes the FP32 products; d = 32, 64 and 96 (multiples of 32) the exact
    three-part BF16 split of both operands, whose 32-wide chunks are loaded
    two ahead across tile boundaries: one, two and three chunks per row."""
    n, L, K, N_r = 200_000, 4, 16, 256
    say(f"codes across persistent tiles n={n} d={d}")
    c = U.case(n=n, d=d, L=L, K=K, N_r=N_r, frac=0.01, seed=5)
    idx = dl.build_index(c["X"], L, K, N_r, 0.01, A=c["A"], sample_ids=c["sample"])
    ex = idx.export()
    P = O.project(c["X"], c["A"])
    ref = O.encode(P, ex["B"].astype(np.float64))
    B64 = ex["B"].astype(np.float64)
    nbad, hard = U.code_mismatches(P, U.proj_scale(c["X"], c["A"]), B64, B64, ref, ex["codes"])
    say(f"  codes differing: {nbad} of {ref.size} (non-borderline {hard})")
    assert hard == 0


# --------------------------------------------------------------------------
# step a4: DE-Trees as leaf runs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,K,N_r,max_leaf,kind", [(6000, 16, 64, 16, "mixture"), (20_000, 8, 16, 64, "mixture"),
                                                   (5000, 4, 4, 8, "smallint"), (3000, 32, 256, 4, "mixture"),
                                                   (6000, 12, 64, 16, "mixture"), (4000, 5, 16, 8, "smallint")])
def test_tree_runs_match_oracle_tree(dl, n, K, N_r, max_leaf, kind):
    say(f"trees n={n} K={K} N_r={N_r} max_leaf={max_leaf} kind={kind}")
    L = 2
    c = U.case(n=n, d=32, L=L, K=K, N_r=N_r, frac=0.2, kind=kind, seed=3)
    idx = dl.build_index(c["X"], L, K, N_r, 0.2, A=c["A"], sample_ids=c["sample"], max_leaf=max_leaf)
    codes = idx.export()["codes"]
    bits = int(np.log2(N_r))
    for i in range(L):
        perm, start, lo, hi = idx.tree(i)
        assert np.array_equal(np.sort(perm), np.arange(n))
        assert start[0] == 0 and start[-1] == n and np.all(np.diff(start) > 0)
        ci = codes[:, i * K:(i + 1) * K].astype(np.int64)
        got = set()
        for t in range(len(start) - 1):
            ids = perm[start[t]:start[t + 1]]
            assert np.all(ci[ids] >= lo[t]) and np.all(ci[ids] <= hi[t])
            width = hi[t].astype(int) - lo[t].astype(int) + 1
            if len(ids) > max_leaf:
                assert np.all(width == 1)
            got.add((tuple(sorted(ids.tolist())), tuple(lo[t]), tuple(hi[t])))
        ref = set()
        for lf in O.build_tree(ci, N_r, max_leaf):
            ref.add((tuple(lf.ids.tolist()), tuple(lf.lo.tolist()), tuple(lf.hi.tolist())))
        assert got == ref
        assert bits >= 1


# --------------------------------------------------------------------------
# steps a5 + a6 fed the oracle's encoding: candidate sets, ids, distances
# --------------------------------------------------------------------------

def _fed_oracle_case(dl, c, k, beta, **qkw):
    P, B, codes = U.oracle_encoding(c)
    B32 = B.astype(np.float32)
    idx = dl.import_index(c["X"], c["A"], B32, codes, c["L"], c["K"], c["N_r"])
    Qp32 = O.project(c["Q"], c["A"]).astype(np.float32)
    r = idx.query_debug(t(c["Q"]), k, 1.5, beta, Qp=t(Qp32), **qkw)
    r = {kk: v.cpu().numpy() for kk, v in r.items()}
    border_total = tie_total = 0
    for qi in range(len(c["Q"])):
        ref = U.oracle_query(c["X"], c["Q"][qi], Qp32[qi], codes, B32, c["L"], c["K"], k, beta)
        cnt = int(r["counts"][qi])
        S_gpu = set(r["cand"][qi, :cnt].tolist())
        S_ref = set(ref.S.tolist())
        if S_gpu != S_ref:
            border = U.borderline_points(Qp32[qi], codes, B32, c["L"], c["K"], ref.thr)
            sym = S_gpu ^ S_ref
            assert sym <= border, f"query {qi}: {len(sym - border)} non-borderline differences"
            border_total += len(sym)
            continue
        assert abs(float(r["thr"][qi]) - ref.thr) <= U.REL * max(ref.thr, 1e-30)
        assert int(r["stop_tree"][qi]) == ref.stop_tree
        ft = dict(zip(r["cand"][qi, :cnt].tolist(), r["first_tree"][qi, :cnt].tolist()))
        assert all(ft[o] == f for o, f in zip(ref.S.tolist(), ref.first_tree.tolist()))
        tie_total += U.compare_result(ref.ids, ref.dists, c["X"], c["Q"][qi], r["ids"][qi], r["dists"][qi],
                                      ref.S, k)
    say(f"  borderline candidate differences: {border_total}; near-tie id differences: {tie_total}")
    return r


@pytest.mark.parametrize("n,d,N_r,k,beta,kind", [(10_000, 128, 256, 10, 0.1, "mixture"),
                                                 (7001, 64, 64, 50, 0.05, "integer"),
                                                 (3000, 40, 16, 10, 0.2, "mixture"),
                                                 (20_000, 32, 256, 100, 0.01, "integer")])
def test_candidates_and_results_fed_oracle_encoding(dl, n, d, N_r, k, beta, kind):
    say(f"fed-oracle query n={n} d={d} N_r={N_r} k={k} beta={beta} kind={kind}")
    c = U.case(n=n, d=d, N_r=N_r, frac=0.1, kind=kind, nq=12, seed=11)
    _fed_oracle_case(dl, c, k, beta)


@pytest.mark.parametrize("L,K", [(1, 16), (2, 32), (8, 8), (4, 4), (1, 4), (2, 8), (4, 12), (2, 5), (1, 1),
                                 (8, 3)])
def test_fed_oracle_other_tree_shapes(dl, L, K):
    say(f"fed-oracle query L={L} K={K}")
    c = U.case(n=5000, d=48, L=L, K=K, N_r=32, frac=0.1, nq=8, seed=L * 10 + K)
    _fed_oracle_case(dl, c, 10, 0.1)


def test_ties_and_fallback_path(dl):
    """Few regions and small-integer data: massive ties in the bounds, so the
    candidate count of the guessed threshold overflows and the query is rerun
    with every point a candidate; results still equal the oracle's."""
    say("ties/fallback n=20000 N_r=2 K=4 L=2")
    c = U.case(n=20_000, d=12, L=2, K=4, N_r=2, frac=0.05, kind="smallint", nq=6, seed=5)
    _fed_oracle_case(dl, c, 10, 0.1)


def test_beta_one_is_brute_force(dl):
    say("beta=1 brute force n=2500")
    c = U.case(n=2500, d=72, N_r=16, frac=0.1, kind="integer", nq=10, seed=9)
    idx = dl.build_index(c["X"], 4, 16, 16, 0.1, A=c["A"], sample_ids=c["sample"])
    ids, dists = idx.query(t(c["Q"]), 25, 1.5, 1.0)
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    for qi in range(len(c["Q"])):
        ref_ids, ref_d2 = O.brute_force_knn(c["X"], c["Q"][qi], 25)
        assert np.array_equal(ids[qi], ref_ids)
        np.testing.assert_allclose(dists[qi], np.sqrt(ref_d2), rtol=U.REL)


def test_k_equals_n_and_tiny_n(dl):
    say("tiny n=64 k=64")
    c = U.case(n=64, d=9, L=1, K=4, N_r=4, frac=1.0, nq=3, seed=2)
    idx = dl.build_index(c["X"], 1, 4, 4, 1.0, A=c["A"], sample_ids=c["sample"])
    ids, dists = idx.query(t(c["Q"]), 64, 1.5, 0.5)
    ids = ids.cpu().numpy()
    for qi in range(3):
        ref_ids, _ = O.brute_force_knn(c["X"], c["Q"][qi], 64)
        assert np.array_equal(ids[qi], ref_ids)


# --------------------------------------------------------------------------
# whole path on the GPU's own encoding (a1..a6)
# --------------------------------------------------------------------------

def test_end_to_end_against_oracle_on_gpu_encoding(dl):
    say("end-to-end C1 shape n=10000 d=128")
    import synth
    cfg = synth.config("C1")
    X = synth.make_data(cfg)
    Q = synth.make_queries(cfg)[:30]
    A = synth.projection_matrix(4, 16, 128, cfg.index_seed)
    sample = synth.sample_ids(cfg.n, cfg.n_s, cfg.index_seed)
    idx = dl.build_index(X, 4, 16, 256, cfg.sample_frac, A=A, sample_ids=sample)
    ex = idx.export()
    Qp = idx.project(t(Q)).cpu().numpy()
    r = idx.query_debug(t(Q), 10, 1.5, 0.1, Qp=t(Qp))
    ids = r["ids"].cpu().numpy()
    d = r["dists"].cpu().numpy()
    for qi in range(len(Q)):
        ref = U.oracle_query(X, Q[qi], Qp[qi], ex["codes"], ex["B"], 4, 16, 10, 0.1)
        S_gpu = set(r["cand"][qi, :int(r["counts"][qi])].cpu().numpy().tolist())
        sym = S_gpu ^ set(ref.S.tolist())
        assert sym <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], 4, 16, ref.thr)
        if not sym:
            U.compare_result(ref.ids, ref.dists, X, Q[qi], ids[qi], d[qi], ref.S, 10)


def test_determinism_and_batch_independence(dl):
    """Bitwise-identical results on reruns and whether a query runs alone or
    inside a larger batch (P12)."""
    say("determinism n=20000")
    c = U.case(n=20_000, d=64, N_r=256, frac=0.05, nq=40, seed=21)
    idx = dl.build_index(c["X"], 4, 16, 256, 0.05, A=c["A"], sample_ids=c["sample"])
    Q = t(c["Q"])
    a_ids, a_d = idx.query(Q, 10, 1.5, 0.1)
    b_ids, b_d = idx.query(Q, 10, 1.5, 0.1)
    assert np.array_equal(a_ids.cpu().numpy(), b_ids.cpu().numpy())
    assert np.array_equal(a_d.cpu().numpy(), b_d.cpu().numpy())
    for qi in (0, 17, 39):
        s_ids, s_d = idx.query(Q[qi:qi + 1], 10, 1.5, 0.1)
        assert np.array_equal(s_ids.cpu().numpy()[0], a_ids.cpu().numpy()[qi])
        assert np.array_equal(s_d.cpu().numpy()[0], a_d.cpu().numpy()[qi])


def test_argument_errors(dl):
    say("argument errors")
    c = U.case(n=500, d=16, N_r=16, frac=0.2, nq=2, seed=1)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        dl.build_index(c["X"], 3, 16, 16, 0.2)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        dl.build_index(c["X"], 4, 16, 24, 0.2)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        dl.build_index(c["X"], 4, 16, 256, 0.2)          # n_s < N_r
    idx = dl.build_index(c["X"], 4, 16, 16, 0.2, A=c["A"], sample_ids=c["sample"])
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        idx.query(t(c["Q"]), 0, 1.5, 0.1)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        idx.query(t(c["Q"]), 10, 1.0, 0.1)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        idx.query(t(c["Q"]), 10, 1.5, 1.5)


# --------------------------------------------------------------------------
# masked dense MFMA verification and the BF16 + rerank form
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,d", [("integer", 128), ("integer", 62), ("mixture", 96)])
def test_bf16_copy_changes_no_answer(dl, kind, d):
    """An index with the BF16 copy (integer data, which BF16 holds exactly, and
    float data, which it rounds) answers bit-identically to one without it,
    for the gathered, dense and BF16-screen paths."""
    say(f"BF16 copy changes no answer kind={kind} d={d}")
    c = U.case(n=70_000, d=d, N_r=256, frac=0.01, kind=kind, nq=100, seed=53)
    plain = dl.build_index(c["X"], 4, 16, 256, 0.01, A=c["A"], sample_ids=c["sample"])
    with_bf = dl.build_index(c["X"], 4, 16, 256, 0.01, A=c["A"], sample_ids=c["sample"], keep_bf16=True)
    Q = t(c["Q"])
    ref_ids, ref_d = (x.cpu().numpy() for x in plain.query(Q, 10, 1.5, 0.1, verify="gather"))
    for idx, verify in ((plain, "dense"), (with_bf, "gather"), (with_bf, "dense"), (with_bf, "dense_bf16")):
        ids, dists = (x.cpu().numpy() for x in idx.query(Q, 10, 1.5, 0.1, verify=verify))
        assert np.array_equal(ids, ref_ids), verify
        assert np.array_equal(dists.view(np.uint32), ref_d.view(np.uint32)), verify


@pytest.mark.parametrize("L,K", [(4, 16), (8, 8), (2, 16), (1, 16)])
@pytest.mark.parametrize("verify", ["dense", "dense_bf16"])
def test_small_stop_tree_on_the_implicit_dense_path(dl, verify, L, K):
    """8,001 identical points (more than N_S = 7,010) and queries on them: the
    first tree alone admits the whole cluster at threshold 0, so the stop tree
    is 1.  For L >= 4 that is below the L-2 that the dense path's selection
    settles from the stored running minima, and its exact pass decides it;
    for L <= 3 the minima (or the key) settle it.  The dense path (S kept
    implicit) returns the gathered path's ids and distances bit for bit, the
    stop trees equal the oracle's, and the results are the oracle's."""
    say(f"small stop tree on the dense path n=70000 d=64 cluster=8001 L={L} K={K} verify={verify}")
    c = U.case(n=70_000, d=64, L=L, K=K, N_r=256, frac=0.01, kind="mixture", nq=40, seed=41)
    X, Q = c["X"].copy(), c["Q"].copy()
    X[1000:9000] = X[500]
    Q[0] = X[500]
    Q[7] = X[500]
    Q[13] = X[500]
    k, beta = 10, 0.1
    idx = dl.build_index(X, L, K, 256, 0.01, A=c["A"], sample_ids=c["sample"], keep_bf16=verify == "dense_bf16")
    Qt = t(Q)
    g_ids, g_d = idx.query(Qt, k, 1.5, beta, verify="gather")
    d_ids, d_d = idx.query(Qt, k, 1.5, beta, verify=verify)
    assert np.array_equal(g_ids.cpu().numpy(), d_ids.cpu().numpy())
    assert np.array_equal(g_d.cpu().numpy(), d_d.cpu().numpy())
    ex = idx.export()
    Qp = idx.project(Qt).cpu().numpy()
    r = idx.query_debug(Qt, k, 1.5, beta, Qp=t(Qp), verify="dense")
    for qi in (0, 7, 13, 1, 2):
        ref = U.oracle_query(X, Q[qi], Qp[qi], ex["codes"], ex["B"], L, K, k, beta)
        if qi in (0, 7, 13):
            assert ref.stop_tree == 1
        assert int(r["stop_tree"][qi]) == ref.stop_tree
        U.compare_result(ref.ids, ref.dists, X, Q[qi], d_ids[qi].cpu().numpy(), d_d[qi].cpu().numpy(), ref.S, k)


@pytest.mark.parametrize("n,beta,near", [(200_000, 0.4, 15_000), (600_000, 0.11, 5_000)])
def test_selection_with_a_tied_bin_above_65536_keys(dl, n, beta, near):
    """The selection's second window pass counts the keys of one first-pass bin
    in 16-bit bins, which holds below 65,536 keys; a bin with more takes the
    three-pass selection.  Here 66,000 identical points hold the N_S-th
    smallest m^2 (a few thousand points lie next to the query, the rest at
    about twice the cluster's m^2, so that the guess threshold stays within
    the window's four binades of it), so one bin holds at least 66,000 keys
    while the candidate count stays inside the planned capacity (N_S = 0.4 n:
    the plain filter; N_S = 0.11 n: the range screen).  The threshold, the
    stop tree and the answers are the oracle's."""
    say(f"selection with a tied bin n={n} beta={beta} near={near}")
    c = U.case(n=n, d=32, L=4, K=16, N_r=256, frac=0.01, kind="mixture", nq=4, seed=43)
    X, Q = c["X"].copy(), c["Q"].copy()
    q = Q[0]
    rng = np.random.default_rng(44)
    ncl = 66_000
    X[:near] = q + 1e-3 * rng.standard_normal((near, X.shape[1])).astype(np.float32)
    X[near:near + ncl] = q + 0.5
    X[near + ncl:] = q + 0.7 + 0.05 * rng.standard_normal((n - near - ncl, X.shape[1])).astype(np.float32)
    k = 10
    idx = dl.build_index(X, 4, 16, 256, 0.01, A=c["A"], sample_ids=c["sample"], keep_bf16=True)
    Qt = t(Q[:1])
    ids, dists = idx.query(Qt, k, 1.5, beta)
    ex = idx.export()
    Qp = idx.project(Qt).cpu().numpy()
    r = idx.query_debug(Qt, k, 1.5, beta, Qp=t(Qp))
    ref = U.oracle_query(X, q, Qp[0], ex["codes"], ex["B"], 4, 16, k, beta)
    m2 = O.lower_bounds(np.asarray(Qp[0], np.float64), ex["codes"], np.asarray(ex["B"], np.float64), 4, 16).min(axis=1)
    ties = int(np.count_nonzero(m2 == ref.thr))
    say(f"  keys tied at the threshold: {ties}")
    assert ties >= 65_536
    assert abs(float(r["thr"][0]) - ref.thr) <= U.REL * ref.thr
    assert int(r["stop_tree"][0]) == ref.stop_tree
    U.compare_result(ref.ids, ref.dists, X, q, ids[0].cpu().numpy(), dists[0].cpu().numpy(), ref.S, k)


@pytest.mark.parametrize("n,d,kind,k,nq", [(70_001, 128, "integer", 10, 150), (66_000, 37, "mixture", 20, 130),
                                           (80_000, 96, "mixture", 100, 64), (65_600, 200, "mixture", 1, 257),
                                           (65_857, 300, "mixture", 10, 140), (65_536, 962, "integer", 5, 70)])
def test_dense_verification_equals_gathered(dl, n, d, kind, k, nq):
    """Survivors of the dense pass are re-ranked with the same FP32 direct
    distances as the gathered pass, so both return identical ids and bits."""
    say(f"dense vs gathered n={n} d={d} kind={kind} k={k} nq={nq}")
    c = U.case(n=n, d=d, N_r=256, frac=0.01, kind=kind, nq=nq, seed=31)
    idx = dl.build_index(c["X"], 4, 16, 256, 0.01, A=c["A"], sample_ids=c["sample"])
    Q = t(c["Q"])
    g_ids, g_d = idx.query(Q, k, 1.5, 0.1, verify="gather")
    d_ids, d_d = idx.query(Q, k, 1.5, 0.1, verify="dense")
    assert np.array_equal(g_ids.cpu().numpy(), d_ids.cpu().numpy())
    assert np.array_equal(g_d.cpu().numpy(), d_d.cpu().numpy())
    ex = idx.export()
    Qp = idx.project(Q).cpu().numpy()
    r = idx.query_debug(Q[:4], k, 1.5, 0.1, Qp=t(Qp[:4]), verify="dense")
    for qi in range(4):
        ref = U.oracle_query(c["X"], c["Q"][qi], Qp[qi], ex["codes"], ex["B"], 4, 16, k, 0.1)
        S_gpu = set(r["cand"][qi, :int(r["counts"][qi])].cpu().numpy().tolist())
        sym = S_gpu ^ set(ref.S.tolist())
        assert sym <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], 4, 16, ref.thr)
        if not sym:
            U.compare_result(ref.ids, ref.dists, c["X"], c["Q"][qi], r["ids"][qi].cpu().numpy(),
                             r["dists"][qi].cpu().numpy(), ref.S, k)


@pytest.mark.parametrize("n,d,kind,k,nq", [(70_001, 128, "integer", 10, 150), (66_000, 37, "mixture", 20, 130),
                                           (80_000, 96, "mixture", 100, 64), (65_600, 200, "mixture", 1, 257),
                                           (65_536, 962, "integer", 5, 70), (70_000, 128, "mixture", 50, 200)])
def test_bf16_screen_gives_the_fp32_results(dl, n, d, kind, k, nq):
    """The FP32 form may screen with BF16 products against a bound widened by
    the BF16 rounding of both vectors; survivors are re-ranked with the same
    FP32 direct distances, so ids and distance bits equal those of the
    gathered pass and of the FP32-product screen."""
    say(f"bf16 screen n={n} d={d} kind={kind} k={k} nq={nq}")
    c = U.case(n=n, d=d, N_r=256, frac=0.01, kind=kind, nq=nq, seed=37)
    idx = dl.build_index(c["X"], 4, 16, 256, 0.01, A=c["A"], sample_ids=c["sample"], keep_bf16=True)
    Q = t(c["Q"])
    out = {v: idx.query(Q, k, 1.5, 0.1, verify=v) for v in ("gather", "dense", "dense_bf16", "auto")}
    g_ids, g_d = (x.cpu().numpy() for x in out["gather"])
    for v in ("dense", "dense_bf16", "auto"):
        ids, dd = (x.cpu().numpy() for x in out[v])
        assert np.array_equal(g_ids, ids), v
        assert np.array_equal(g_d, dd), v
    idx.free()
    plain = dl.build_index(c["X"][:5000], 4, 16, 256, 0.1)
    with pytest.raises(dl.DetlshError, match="keep_bf16"):
        plain.query(Q[:2], k, 1.5, 0.1, verify="dense_bf16")


@pytest.mark.parametrize("n,d,k", [(70_000, 128, 10), (66_000, 96, 25), (66_000, 300, 10), (65_600, 960, 10)])
def test_bf16_rerank_form(dl, n, d, k):
    """BF16 products with FP32 accumulation keep candidates by the rerank
    bound; the returned distances are exact FP32 distances of the returned
    ids and the ids agree with the FP32 form at recall >= 0.98."""
    say(f"bf16 rerank n={n} d={d} k={k}")
    c = U.case(n=n, d=d, N_r=256, frac=0.01, kind="mixture", nq=100, seed=41)
    idx = dl.build_index(c["X"], 4, 16, 256, 0.01, A=c["A"], sample_ids=c["sample"], keep_bf16=True)
    Q = t(c["Q"])
    f_ids, f_d = idx.query(Q, k, 1.5, 0.1)
    b_ids, b_d = idx.query(Q, k, 1.5, 0.1, precision=dl.BF16_RERANK, rerank_mult=4)
    f_ids, b_ids, b_d = f_ids.cpu().numpy(), b_ids.cpu().numpy(), b_d.cpu().numpy()
    agree = np.mean([len(set(a) & set(b)) / k for a, b in zip(f_ids, b_ids)])
    say(f"  BF16+rerank agreement with FP32: {agree:.4f}")
    assert agree >= 0.98
    for qi in range(0, 100, 7):
        exact = np.sqrt(O.sq_dists(c["X"][b_ids[qi]], c["Q"][qi]))
        np.testing.assert_allclose(b_d[qi], exact, rtol=U.REL)
        assert np.all(np.diff(b_d[qi]) >= 0)
    with pytest.raises(dl.DetlshError, match="keep_bf16"):
        dl.build_index(c["X"][:5000], 4, 16, 256, 0.1).query(Q[:2], k, 1.5, 0.1, precision=dl.BF16_RERANK)


@pytest.mark.parametrize("n,d,L,K,N_r,beta,k,kind,nq", [
    (70_001, 96, 4, 16, 256, 0.01, 10, "mixture", 37),
    (65_600, 128, 4, 16, 256, 0.1, 10, "integer", 40),
    (9_000, 64, 4, 16, 64, 0.05, 5, "mixture", 21),
    (20_000, 48, 2, 8, 256, 0.2, 25, "mixture", 33),
    (12_345, 32, 1, 32, 128, 0.02, 7, "mixture", 17),
    (8_200, 40, 4, 4, 16, 0.1, 10, "smallint", 19),
    (30_000, 64, 2, 32, 256, 0.3, 3, "integer", 16),
    (25_000, 48, 4, 12, 128, 0.02, 10, "mixture", 20),
])
def test_screen_filter_equals_plain_filter(dl, n, d, L, K, N_r, beta, k, kind, nq):
    """The MFMA screen (ball around each clamped cell) plus exact bounds of its
    survivors keeps exactly the plain filter's candidates with bit-identical
    keys: the same S, threshold, stop tree and first trees, and bit-identical
    answers on the dumps path and on the implicit-S dense path; and both
    equal the oracle on its own encoding up to points on the threshold."""
    say(f"screen vs plain filter n={n} d={d} L={L} K={K} N_r={N_r} beta={beta} k={k} kind={kind} nq={nq}")
    c = U.case(n=n, d=d, L=L, K=K, N_r=N_r, frac=0.05, kind=kind, nq=nq, seed=n % 101)
    idx = dl.build_index(c["X"], L, K, N_r, 0.05, A=c["A"], sample_ids=c["sample"], keep_bf16=True)
    Qh = c["Q"].copy()
    Qh[: min(3, nq)] = c["X"][[0, n // 2, n - 1][: min(3, nq)]]   # queries on data points (bounds of 0)
    Q = t(Qh)
    dbg = {}
    for f in ("plain", "screen"):
        dbg[f] = idx.query_debug(Q, k, 1.5, beta, filter=f)
    a, b = dbg["plain"], dbg["screen"]
    for key in ("counts", "thr", "stop_tree", "ids", "dists"):
        assert torch_equal(a[key], b[key]), key
    ca, cb = a["cand"].cpu().numpy(), b["cand"].cpu().numpy()
    fa, fb = a["first_tree"].cpu().numpy(), b["first_tree"].cpu().numpy()
    counts = a["counts"].cpu().numpy()
    for qi in range(nq):
        m = int(counts[qi])
        oa, ob = np.argsort(ca[qi, :m]), np.argsort(cb[qi, :m])
        assert np.array_equal(ca[qi, :m][oa], cb[qi, :m][ob])
        assert np.array_equal(fa[qi, :m][oa], fb[qi, :m][ob])
    pa = idx.query(Q, k, 1.5, beta, filter="plain")
    pb = idx.query(Q, k, 1.5, beta, filter="screen")
    assert torch_equal(pa[0], pb[0]) and torch_equal(pa[1], pb[1])
    ex = idx.export()
    Qp = idx.project(Q).cpu().numpy()
    r = idx.query_debug(Q, k, 1.5, beta, Qp=t(Qp), filter="screen")
    for qi in range(0, nq, 4):
        ref = U.oracle_query(c["X"], Qh[qi], Qp[qi], ex["codes"], ex["B"], L, K, k, beta)
        S_gpu = set(r["cand"][qi, :int(r["counts"][qi])].cpu().numpy().tolist())
        assert S_gpu ^ set(ref.S.tolist()) <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], L, K, ref.thr)


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))


@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_compensated_distances_d960(dl, form):
    """At d = 960 the exact distances of the final ranking are compensated
    sums: every returned distance is within 4e-7 relative of the FP64 distance
    of the returned id (an uncompensated FP32 sum of 960 squares may be off by
    up to about 1e-4), and the FP32 form's answers equal the oracle's on the
    GPU's own encoding (ids up to near-ties, distances within 1e-5)."""
    import synth
    n, d, k = 65_600, 960, 10
    say(f"compensated distances n={n} d={d} form={form}")
    X = synth.beta_copula(n, d, 91)
    Qh = synth.beta_copula(12, d, 92)
    A = synth.projection_matrix(4, 16, d, 93)
    sample = synth.sample_ids(n, 656, 94)
    idx = dl.build_index(X, 4, 16, 256, 0.01, A=A, sample_ids=sample, keep_bf16=(form == "bf16"))
    Q = t(Qh)
    kw = {"precision": dl.BF16_RERANK} if form == "bf16" else {}
    ids, dists = (v.cpu().numpy() for v in idx.query(Q, k, 1.5, 0.1, **kw))
    worst = 0.0
    for qi in range(len(Qh)):
        exact = np.sqrt(O.sq_dists(X[ids[qi]], Qh[qi]))
        worst = max(worst, float(np.max(np.abs(dists[qi] - exact) / exact)))
    say(f"  largest relative distance error {worst:.3g}")
    assert worst <= 4e-7
    if form == "fp32":
        ex = idx.export()
        Qp = idx.project(Q).cpu().numpy()
        r = idx.query_debug(Q, k, 1.5, 0.1, Qp=t(Qp))
        g_ids, g_d = r["ids"].cpu().numpy(), r["dists"].cpu().numpy()
        for qi in range(len(Qh)):
            ref = U.oracle_query(X, Qh[qi], Qp[qi], ex["codes"], ex["B"], 4, 16, k, 0.1)
            S_gpu = set(r["cand"][qi, :int(r["counts"][qi])].cpu().numpy().tolist())
            sym = S_gpu ^ set(ref.S.tolist())
            assert sym <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], 4, 16, ref.thr)
            if not sym:
                U.compare_result(ref.ids, ref.dists, X, Qh[qi], g_ids[qi], g_d[qi], ref.S, k)


# --------------------------------------------------------------------------
# the printed radius ladder from a given r_min (Alg. 7), both stop conditions
# --------------------------------------------------------------------------

def _ladder_borderline(lb, eps, r_min, c, rounds, rel=1e-5):
    """Points whose bound lies within rel of one of the ladder's radii."""
    r = r_min
    out = set()
    for _ in range(rounds):
        rad2 = (eps * r) ** 2
        near = np.abs(lb - rad2) <= rel * rad2
        out |= set(np.flatnonzero(near.any(axis=1)).tolist())
        r *= c
    return out


@pytest.mark.parametrize("c,div,beta,k,kind,L,K", [(1.5, 40.0, 0.1, 10, "mixture", 4, 16),
                                                    (2.0, 40.0, 0.1, 10, "integer", 4, 16),
                                                    (1.5, 5.0, 0.05, 25, "mixture", 4, 16),
                                                    (1.5, 40.0, 0.99, 5, "mixture", 4, 16),
                                                    (1.5, 40.0, 0.1, 10, "mixture", 2, 5),
                                                    (2.0, 40.0, 0.1, 10, "mixture", 4, 7)])
def test_fixed_ladder_fed_oracle_encoding(dl, c, div, beta, k, kind, L, K):
    """The radius ladder fed the oracle's encoding; odd K checks the chi-square
    quantile of eps (Lemma 3) for odd degrees of freedom."""
    say(f"fixed ladder c={c} r_min=r*/{div} beta={beta} k={k} kind={kind} L={L} K={K}")
    cc = U.case(n=6000, d=48, L=L, K=K, N_r=64, frac=0.1, kind=kind, nq=10, seed=61)
    P, B, codes = U.oracle_encoding(cc)
    B32 = B.astype(np.float32)
    idx = dl.import_index(cc["X"], cc["A"], B32, codes, L, K, 64)
    Qp32 = O.project(cc["Q"], cc["A"]).astype(np.float32)
    eps = O.epsilon(L, K)
    stops = {1: 0, 2: 0}
    for qi in range(len(cc["Q"])):
        qp = Qp32[qi].astype(np.float64)
        mg = O.query_magic(cc["X"], cc["Q"][qi], qp, codes, B32.astype(np.float64), L, K, k, min(beta, 0.5))
        r_min = float(np.sqrt(max(mg.thr, 1e-12)) / eps / div)
        ref = O.query_fixed(cc["X"], cc["Q"][qi], qp, codes, B32.astype(np.float64), L, K, k, beta, c, r_min, eps)
        r = idx.query_debug(t(cc["Q"][qi:qi + 1]), k, c, beta, Qp=t(Qp32[qi:qi + 1]), rmin_policy=dl.RMIN_FIXED,
                            r_min=r_min, max_rounds=64)
        S = set(r["cand"][0, :int(r["counts"][0])].cpu().numpy().tolist())
        if S != set(ref.S.tolist()):
            lb = O.lower_bounds(qp, codes, B32.astype(np.float64), L, K)
            assert S ^ set(ref.S.tolist()) <= _ladder_borderline(lb, eps, r_min, c, ref.rounds + 1)
            continue
        assert int(r["rounds"][0]) == ref.rounds and int(r["stop_tree"][0]) == ref.stop_tree
        assert float(r["thr"][0]) == pytest.approx(ref.thr, rel=1e-6)
        ft = dict(zip(r["cand"][0, :len(S)].cpu().numpy().tolist(), r["first_tree"][0, :len(S)].cpu().numpy().tolist()))
        assert all(ft[o] == f for o, f in zip(ref.S.tolist(), ref.first_tree.tolist()))
        U.compare_result(ref.ids, ref.dists, cc["X"], cc["Q"][qi], r["ids"][0].cpu().numpy(),
                         r["dists"][0].cpu().numpy(), ref.S, k)
        stops[ref.stop_cond] += 1
        if div >= 40:
            assert ref.rounds >= 2
    say(f"  stops by condition 1 / 2: {stops}")
    if beta > 0.9:
        assert stops[2] > 0


def test_fixed_ladder_without_stop_is_answered_over_D(dl):
    """One round from a tiny radius admits nothing: the query is answered over
    all points (exact k-NN)."""
    say("fixed ladder, no stop within max_rounds")
    cc = U.case(n=3000, d=32, N_r=16, frac=0.1, kind="integer", nq=4, seed=62)
    idx = dl.build_index(cc["X"], 4, 16, 16, 0.1, A=cc["A"], sample_ids=cc["sample"])
    ids, dists = idx.query(t(cc["Q"]), 7, 1.5, 0.1, rmin_policy=dl.RMIN_FIXED, r_min=1e-6, max_rounds=1)
    for qi in range(4):
        ref_ids, _ = O.brute_force_knn(cc["X"], cc["Q"][qi], 7)
        assert np.array_equal(ids[qi].cpu().numpy(), ref_ids)
    with pytest.raises(dl.DetlshError, match="r_min"):
        idx.query(t(cc["Q"]), 7, 1.5, 0.1, rmin_policy=dl.RMIN_FIXED, r_min=0.0)


def test_borrowed_x_answers_like_a_copy(dl):
    """An index that reads X in place (borrow_x) answers bit for bit like one
    built over a copy, in both precision forms, and leaves X unchanged; an
    insert moves its points into an array of the index's own, after which it
    answers like the copy-built index after the same insert, also once the
    caller's X is gone."""
    import torch
    say("borrowed X n=20000 d=64")
    c = U.case(n=24_000, d=64, L=4, K=16, N_r=64, frac=0.05, kind="mixture", nq=50, seed=91)
    X1, X2 = c["X"][:20_000], c["X"][20_000:]
    sample = c["sample"][c["sample"] < 20_000][:1000]
    Xd = t(X1)
    before = Xd.clone()
    Q = t(c["Q"])
    a = dl.build_index(Xd, 4, 16, 64, len(sample) / 20_000, A=c["A"], sample_ids=sample, keep_bf16=True)
    b = dl.build_index(Xd, 4, 16, 64, len(sample) / 20_000, A=c["A"], sample_ids=sample, keep_bf16=True,
                       borrow_x=True)
    for prec in (dl.FP32, dl.BF16_RERANK):
        ia, da = a.query(Q, 10, 1.5, 0.1, precision=prec)
        ib, db = b.query(Q, 10, 1.5, 0.1, precision=prec)
        assert torch.equal(ia, ib) and torch.equal(da, db)
    torch.cuda.synchronize()
    assert torch.equal(Xd, before)
    a.insert(t(X2))
    b.insert(t(X2))
    # the caller's block goes back to torch's cache and is refilled with NaN:
    # an index still reading it would return NaN distances
    del Xd
    b._borrowed_x = None   # the index owns its points now
    torch.cuda.synchronize()
    junk = torch.full_like(before, float("nan"))
    ia, da = a.query(Q, 10, 1.5, 0.1)
    ib, db = b.query(Q, 10, 1.5, 0.1)
    assert torch.equal(ia, ib) and torch.equal(da, db)
    assert not torch.isnan(db).any()
    a.free()
    b.free()
    del junk
    assert torch.equal(before, t(X1))
