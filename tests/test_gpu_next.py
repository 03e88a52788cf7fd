"""GPU parity of the rows beyond the c^2-k-ANN path: the (r, c)-ANN query of
Alg. 6, DET-ONLY's PAA projection (Sec. 6.1) and index save/load, through the
C ABI against the FP64 oracle.

Tolerances as for the main path: candidate membership may differ only for
points whose FP64 bound lies within 1e-5 relative of (eps r)^2, and the answer
only when a point's distance lies within 1e-5 relative of c*r or of the
returned distance (near-ties); distances within 1e-5 relative.
"""
import math
import os

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


def _rc_borderline(X, q, qp, codes, B, L, K, r, c, eps):
    lb = O.lower_bounds(np.asarray(qp, np.float64), codes, np.asarray(B, np.float64), L, K)
    rad2 = (eps * r) ** 2
    near_lb = np.abs(lb - rad2) <= U.REL * max(rad2, 1e-30)
    d2 = O.sq_dists(X, q)
    near_c = np.abs(d2 - (c * r) ** 2) <= U.REL * max((c * r) ** 2, 1e-30)
    return bool(near_lb.any() or near_c.any())


@pytest.mark.parametrize("c,kind", [(1.5, "mixture"), (2.0, "integer")])
def test_rc_query_matches_oracle(dl, c, kind):
    say(f"(r,c)-ANN c={c} kind={kind}")
    cc = U.case(n=6000, d=48, N_r=64, frac=0.1, kind=kind, nq=16, seed=71)
    idx = dl.build_index(cc["X"], 4, 16, 64, 0.1, A=cc["A"], sample_ids=cc["sample"])
    ex = idx.export()
    Q = t(cc["Q"])
    Qp = idx.project(Q).cpu().numpy()
    eps = O.epsilon(4, 16)
    nn = np.array([math.sqrt(O.sq_dists(cc["X"], q).min()) for q in cc["Q"]])
    conds = {0: 0, 1: 0, 2: 0}
    skipped = 0
    for scale in (0.25, 0.6, 1.0, 1.7):
        for qi in range(len(cc["Q"])):
            r = float(nn[qi] * scale)
            ids, d = idx.query_rc(Q[qi:qi + 1], r, c, 0.1)
            ref = O.query_rc(cc["X"], cc["Q"][qi], Qp[qi].astype(np.float64), ex["codes"],
                             ex["B"].astype(np.float64), 4, 16, r, c, 0.1, eps)
            if _rc_borderline(cc["X"], cc["Q"][qi], Qp[qi], ex["codes"], ex["B"], 4, 16, r, c, eps):
                skipped += 1
                continue
            conds[ref.cond] += 1
            got_id, got_d = int(ids.cpu()[0]), float(d.cpu()[0])
            if ref.id < 0:
                assert got_id == -1 and math.isinf(got_d), (qi, scale)
                continue
            assert got_d == pytest.approx(ref.dist, rel=U.REL, abs=1e-6)
            if got_id != ref.id:   # only at a distance tie
                assert abs(math.sqrt(O.sq_dists(cc["X"][[got_id]], cc["Q"][qi])[0]) - ref.dist) <= 1e-5 * ref.dist
    say(f"  answers by condition (0 = nothing): {conds}; borderline cases skipped: {skipped}")
    assert conds[0] > 0 and conds[1] + conds[2] > 0


def test_rc_query_batched_equals_single(dl):
    cc = U.case(n=5000, d=32, N_r=64, frac=0.1, nq=40, seed=72)
    idx = dl.build_index(cc["X"], 4, 16, 64, 0.1, A=cc["A"], sample_ids=cc["sample"])
    Q = t(cc["Q"])
    r = float(np.median([math.sqrt(O.sq_dists(cc["X"], q).min()) for q in cc["Q"]]))
    ids, d = idx.query_rc(Q, r, 1.5, 0.1)
    for qi in (0, 13, 39):
        i1, d1 = idx.query_rc(Q[qi:qi + 1], r, 1.5, 0.1)
        assert int(i1.cpu()[0]) == int(ids.cpu()[qi])
        assert float(d1.cpu()[0]) == float(d.cpu()[qi]) or (math.isinf(float(d1.cpu()[0])) and
                                                           math.isinf(float(d.cpu()[qi])))


def test_rc_zero_radius_and_errors(dl):
    cc = U.case(n=4000, d=32, N_r=256, frac=0.1, nq=4, seed=73)
    idx = dl.build_index(cc["X"], 4, 16, 256, 0.1, A=cc["A"], sample_ids=cc["sample"])
    ids, d = idx.query_rc(t(cc["Q"]), 0.0, 1.5, 0.1)
    assert np.all(ids.cpu().numpy() == -1) and np.all(np.isinf(d.cpu().numpy()))
    own = t(cc["X"][[17, 250]])
    ids, d = idx.query_rc(own, 0.0, 1.5, 0.1)
    assert ids.cpu().numpy().tolist() == [17, 250] and np.all(d.cpu().numpy() == 0)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        idx.query_rc(own, -1.0, 1.5, 0.1)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        idx.query_rc(own, 1.0, 1.0, 0.1)


@pytest.mark.parametrize("d,kind", [(128, "integer"), (100, "mixture")])
def test_det_only_paa_matches_oracle(dl, d, kind):
    """DET-ONLY: one space of K = 16 PAA segment means; projection, codes and
    answers against the oracle's PAA on the GPU's encoding."""
    say(f"DET-ONLY d={d} kind={kind}")
    cc = U.case(n=8000, d=d, L=1, K=16, N_r=256, frac=0.1, kind=kind, nq=10, seed=74)
    idx = dl.build_index(cc["X"], 1, 16, 256, 0.1, sample_ids=cc["sample"], projection="paa")
    ex = idx.export()
    A_ref = O.paa_matrix(d, 16)
    assert np.array_equal(ex["A"], A_ref.astype(np.float32))
    P = O.project(cc["X"], A_ref)
    Pscale = U.proj_scale(cc["X"], A_ref)
    Qp = idx.project(t(cc["Q"])).cpu().numpy()
    Qp_ref = O.project(cc["Q"], A_ref)
    assert np.all(np.abs(Qp - Qp_ref) <= U.REL * U.proj_scale(cc["Q"], A_ref) + 1e-30)
    B_ref = O.breakpoints_by_sort(P[cc["sample"]], 256)
    codes_ref = O.encode(P, B_ref)
    nbad, hard = U.code_mismatches(P, Pscale, B_ref, ex["B"].astype(np.float64), codes_ref, ex["codes"])
    say(f"  code mismatches {nbad} (non-borderline {hard})")
    assert hard == 0
    r = idx.query_debug(t(cc["Q"]), 10, 1.5, 0.1, Qp=t(Qp))
    for qi in range(len(cc["Q"])):
        ref = U.oracle_query(cc["X"], cc["Q"][qi], Qp[qi], ex["codes"], ex["B"], 1, 16, 10, 0.1)
        S_gpu = set(r["cand"][qi, :int(r["counts"][qi])].cpu().numpy().tolist())
        sym = S_gpu ^ set(ref.S.tolist())
        assert sym <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], 1, 16, ref.thr)
        if not sym:
            U.compare_result(ref.ids, ref.dists, cc["X"], cc["Q"][qi], r["ids"][qi].cpu().numpy(),
                             r["dists"][qi].cpu().numpy(), ref.S, 10)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        dl.build_index(cc["X"], 4, 16, 256, 0.1, projection="paa")


def test_save_load_padded_k(dl, tmp_path):
    """K = 12 runs as 16 internally; the file and every export hold 12."""
    say("save / load, K = 12")
    cc = U.case(n=7000, d=40, L=4, K=12, N_r=64, frac=0.05, kind="mixture", nq=12, seed=76)
    idx = dl.build_index(cc["X"], 4, 12, 64, 0.05, A=cc["A"], sample_ids=cc["sample"])
    path = tmp_path / "index12.detlsh"
    idx.save(path)
    back = dl.load_index(path)
    assert back.info["K"] == 12
    a, b = idx.export(), back.export()
    assert a["codes"].shape == (7000, 48) and a["B"].shape == (48, 65)
    for key in ("A", "B", "codes", "sample_ids"):
        assert np.array_equal(a[key], b[key]), key
    for i in range(4):
        for x, y in zip(idx.tree(i), back.tree(i)):
            assert np.array_equal(x, y)
    Q = t(cc["Q"])
    i1, d1 = idx.query(Q, 10, 1.5, 0.1)
    i2, d2 = back.query(Q, 10, 1.5, 0.1)
    assert np.array_equal(i1.cpu().numpy(), i2.cpu().numpy()) and np.array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    assert idx.project(Q).shape == (12, 48)


def test_save_load_roundtrip(dl, tmp_path):
    say("save / load")
    cc = U.case(n=9000, d=40, N_r=128, frac=0.05, kind="mixture", nq=30, seed=75)
    idx = dl.build_index(cc["X"], 4, 16, 128, 0.05, A=cc["A"], sample_ids=cc["sample"], keep_bf16=True,
                         max_leaf=64)
    path = tmp_path / "index.detlsh"
    idx.save(path)
    back = dl.load_index(path)
    a, b = idx.export(), back.export()
    for key in ("A", "B", "codes", "sample_ids"):
        assert np.array_equal(a[key], b[key]), key
    assert idx.info["n_leaves"] == back.info["n_leaves"] and back.info["has_bf16"] and back.info["max_leaf"] == 64
    for i in range(4):
        for x, y in zip(idx.tree(i), back.tree(i)):
            assert np.array_equal(x, y)
    Q = t(cc["Q"])
    for kw in ({}, {"precision": dl.BF16_RERANK}, {"rmin_policy": dl.RMIN_FIXED, "r_min": 0.5}):
        i1, d1 = idx.query(Q, 10, 1.5, 0.1, **kw)
        i2, d2 = back.query(Q, 10, 1.5, 0.1, **kw)
        assert np.array_equal(i1.cpu().numpy(), i2.cpu().numpy())
        assert np.array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    # a flipped byte, a truncated file, another format and a missing file are refused
    raw = bytearray(path.read_bytes())
    bad = tmp_path / "flipped.detlsh"
    raw2 = bytearray(raw)
    raw2[len(raw2) // 2] ^= 0x40
    bad.write_bytes(bytes(raw2))
    with pytest.raises(dl.DetlshError, match="checksum"):
        dl.load_index(bad)
    short = tmp_path / "short.detlsh"
    short.write_bytes(bytes(raw[: len(raw) - 100]))
    with pytest.raises(dl.DetlshError, match="truncated"):
        dl.load_index(short)
    other = tmp_path / "other.detlsh"
    other.write_bytes(b"NOTANIDX" + bytes(raw[8:200]))
    with pytest.raises(dl.DetlshError, match="format"):
        dl.load_index(other)
    with pytest.raises(dl.DetlshError, match="cannot open"):
        dl.load_index(tmp_path / "missing.detlsh")
    assert not os.path.exists(str(path) + ".tmp")


def test_insert_codes_across_persistent_tiles(dl):
    """Inserted points are encoded by the persistent encode at an offset into
    the code array: with both the built set and the insertion above 65,536
    rows (several tiles per workgroup), every code of both parts is compared
    with the oracle's encoding against the frozen breakpoints."""
    n0, m = 70_000, 80_000
    say(f"insert codes across tiles n0={n0} m={m}")
    cc = U.case(n=n0 + m, d=16, N_r=256, frac=0.01, kind="mixture", nq=4, seed=77)
    X1, X2 = cc["X"][:n0], cc["X"][n0:]
    sample = cc["sample"][cc["sample"] < n0][:700]
    idx = dl.build_index(X1, 4, 16, 256, len(sample) / n0, A=cc["A"], sample_ids=sample)
    idx.insert(X2)
    ex = idx.export()
    B64 = ex["B"].astype(np.float64)
    for part, Xp, codes in (("built", X1, ex["codes"][:n0]), ("inserted", X2, ex["codes"][n0:])):
        P = O.project(Xp, cc["A"])
        ref = O.encode(P, B64)
        nbad, hard = U.code_mismatches(P, U.proj_scale(Xp, cc["A"]), B64, B64, ref, codes)
        say(f"  {part}: codes differing {nbad} of {ref.size} (non-borderline {hard})")
        assert hard == 0


@pytest.mark.parametrize("keep_bf16", [False, True])
def test_insert_equals_import_of_the_union(dl, keep_bf16):
    """Points inserted after the build are encoded against the frozen
    breakpoints (codes bit-exact with the oracle's except borderline
    coordinates); the index then equals one imported from the concatenated
    codes: same trees and bit-identical answers.  Two batches = one batch."""
    say(f"insert keep_bf16={keep_bf16}")
    cc = U.case(n=9000, d=48, N_r=128, frac=0.1, kind="mixture", nq=24, seed=76)
    n1 = 6000
    X1, X2 = cc["X"][:n1], cc["X"][n1:]
    sample = cc["sample"][cc["sample"] < n1][: max(128, int(0.1 * n1))]
    build = dict(A=cc["A"], sample_ids=sample, keep_bf16=keep_bf16)
    idx = dl.build_index(X1, 4, 16, 128, len(sample) / n1, **build)
    before = idx.export()
    idx.insert(X2[:1234])
    idx.insert(X2[1234:])
    one = dl.build_index(X1, 4, 16, 128, len(sample) / n1, **build)
    one.insert(X2)
    ex = idx.export()
    assert idx.info["n"] == 9000 and np.array_equal(ex["B"], before["B"])
    assert np.array_equal(ex["codes"][:n1], before["codes"])
    assert np.array_equal(ex["codes"], one.export()["codes"])
    P2 = O.project(X2, cc["A"])
    ref = O.encode(P2, ex["B"].astype(np.float64))
    nbad, hard = U.code_mismatches(P2, U.proj_scale(X2, cc["A"]), ex["B"].astype(np.float64),
                                   ex["B"].astype(np.float64), ref, ex["codes"][n1:])
    say(f"  new-point code mismatches {nbad} (non-borderline {hard})")
    assert hard == 0
    imp = dl.import_index(cc["X"], cc["A"], ex["B"], ex["codes"], 4, 16, 128, keep_bf16=keep_bf16)
    assert idx.info["n_leaves"] == imp.info["n_leaves"]
    for i in range(4):
        for x, y in zip(idx.tree(i), imp.tree(i)):
            assert np.array_equal(x, y)
    Q = t(cc["Q"])
    forms = [{}] + ([{"precision": dl.BF16_RERANK}] if keep_bf16 else [])
    for kw in forms:
        a = idx.query(Q, 10, 1.5, 0.1, **kw)
        b = imp.query(Q, 10, 1.5, 0.1, **kw)
        assert all(np.array_equal(u.cpu().numpy(), v.cpu().numpy()) for u, v in zip(a, b))
    # and against the oracle on that encoding
    Qp = idx.project(Q).cpu().numpy()
    r = idx.query_debug(Q, 10, 1.5, 0.1, Qp=t(Qp))
    for qi in range(len(cc["Q"])):
        ref_q = U.oracle_query(cc["X"], cc["Q"][qi], Qp[qi], ex["codes"], ex["B"], 4, 16, 10, 0.1)
        S_gpu = set(r["cand"][qi, :int(r["counts"][qi])].cpu().numpy().tolist())
        sym = S_gpu ^ set(ref_q.S.tolist())
        assert sym <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], 4, 16, ref_q.thr)
        if not sym:
            U.compare_result(ref_q.ids, ref_q.dists, cc["X"], cc["Q"][qi], r["ids"][qi].cpu().numpy(),
                             r["dists"][qi].cpu().numpy(), ref_q.S, 10)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        dl._lib.check(dl._lib.lib().detlsh_insert(idx._h, X2.ctypes.data_as(dl.C.c_void_p), 5, None))


def _leaf_borderline(qp, trees, B, L, K, thr):
    lb, _ = O.leaf_bounds(np.asarray(qp, np.float64), trees, np.asarray(B, np.float64), L, K)
    m = lb.min(axis=1)
    return set(np.flatnonzero(np.abs(m - thr) <= U.REL * max(thr, 1e-30)).tolist()), lb


@pytest.mark.parametrize("max_leaf,kind,k,beta", [(32, "mixture", 10, 0.1), (8, "integer", 10, 0.05),
                                                  (256, "mixture", 25, 0.1)])
def test_leaf_granularity_matches_oracle(dl, max_leaf, kind, k, beta):
    """Leaf boxes as the candidate test, the stop tree's leaves by (bound,
    smallest id): candidate sets, stop tree, first trees and answers against
    the oracle on the GPU's encoding and trees."""
    say(f"leaf granularity max_leaf={max_leaf} kind={kind} k={k} beta={beta}")
    cc = U.case(n=6000, d=48, N_r=64, frac=0.1, kind=kind, nq=10, seed=77)
    idx = dl.build_index(cc["X"], 4, 16, 64, 0.1, A=cc["A"], sample_ids=cc["sample"], max_leaf=max_leaf)
    ex = idx.export()
    trees = O.build_trees(ex["codes"], 4, 16, 64, max_leaf)
    for i in range(4):
        perm, start, lo, hi = idx.tree(i)
        assert len(start) - 1 == len(trees[i])
        gpu = {tuple(perm[start[j]:start[j + 1]].tolist()) for j in range(len(start) - 1)}
        assert gpu == {tuple(lf.ids.tolist()) for lf in trees[i]}   # same leaves, ids ascending in each
    Q = t(cc["Q"])
    Qp = idx.project(Q).cpu().numpy()
    r = idx.query_debug(Q, k, 1.5, beta, Qp=t(Qp), granularity="leaf")
    plain = idx.query(Q, k, 1.5, beta, granularity="leaf")
    assert np.array_equal(plain[0].cpu().numpy(), r["ids"].cpu().numpy())
    border_total = 0
    for qi in range(len(cc["Q"])):
        ref = O.query_magic_leaf(cc["X"], cc["Q"][qi], Qp[qi].astype(np.float64), ex["codes"],
                                 ex["B"].astype(np.float64), trees, 4, 16, k, beta)
        cnt = int(r["counts"][qi])
        S = set(r["cand"][qi, :cnt].cpu().numpy().tolist())
        if S != set(ref.S.tolist()):
            border, _ = _leaf_borderline(Qp[qi], trees, ex["B"], 4, 16, ref.thr)
            assert border, f"query {qi}: candidate sets differ without a borderline point"
            border_total += 1
            continue
        assert int(r["stop_tree"][qi]) == ref.stop_tree
        assert float(r["thr"][qi]) == pytest.approx(ref.thr, rel=U.REL)
        ft = dict(zip(r["cand"][qi, :cnt].cpu().numpy().tolist(), r["first_tree"][qi, :cnt].cpu().numpy().tolist()))
        assert all(ft[o] == f for o, f in zip(ref.S.tolist(), ref.first_tree.tolist()))
        U.compare_result(ref.ids, ref.dists, cc["X"], cc["Q"][qi], r["ids"][qi].cpu().numpy(),
                         r["dists"][qi].cpu().numpy(), ref.S, k)
    say(f"  queries with borderline candidate differences: {border_total}")
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        idx.query(Q, k, 1.5, beta, granularity="leaf", rmin_policy=dl.RMIN_FIXED, r_min=1.0)


def test_leaf_granularity_dense_equals_gathered(dl):
    say("leaf granularity dense vs gathered n=70000")
    cc = U.case(n=70_000, d=64, N_r=256, frac=0.01, kind="mixture", nq=90, seed=78)
    idx = dl.build_index(cc["X"], 4, 16, 256, 0.01, A=cc["A"], sample_ids=cc["sample"])
    Q = t(cc["Q"])
    g = idx.query(Q, 10, 1.5, 0.1, verify="gather", granularity="leaf")
    d = idx.query(Q, 10, 1.5, 0.1, verify="dense", granularity="leaf")
    assert np.array_equal(g[0].cpu().numpy(), d[0].cpu().numpy())
    assert np.array_equal(g[1].cpu().numpy(), d[1].cpu().numpy())


def test_reused_workspace_gives_identical_results(dl):
    """A query call leaves its workspace for reuse: a later call that takes a
    used (and larger) buffer, and one after detlsh_trim has freed the cache,
    return exactly what the first call returned."""
    import torch
    cc = U.case(n=20000, d=48, N_r=64, frac=0.05, nq=300, seed=91)
    idx = dl.build_index(cc["X"], 4, 16, 64, 0.05, A=cc["A"], sample_ids=cc["sample"])
    Q = t(cc["Q"])
    dl.trim()
    small = Q[:37].contiguous()
    say("fresh small batch")
    i0, d0 = idx.query(small, 10, 1.5, 0.1)
    say("large batch in a small workspace (several chunks), then the small batch again")
    i1, d1 = idx.query(Q, 10, 1.5, 0.1, workspace_bytes=64 << 20)
    i2, d2 = idx.query(small, 10, 1.5, 0.1)
    i3, d3 = idx.query(Q, 10, 1.5, 0.1)
    dl.trim()
    i4, d4 = idx.query(small, 10, 1.5, 0.1)
    torch.cuda.synchronize()
    for a, b in ((i0, i2), (i0, i4), (i1[:37], i0), (i3, i1)):
        assert torch.equal(a, b)
    for a, b in ((d0, d2), (d0, d4), (d1[:37], d0), (d3, d1)):
        assert torch.equal(a, b)
    idx.free()


def test_rebuild_on_reused_index_memory_is_identical(dl):
    """A freed index's arrays are cached and handed to the next build, still
    holding the old contents: a rebuild over such memory (after an index of
    another size and data filled it) equals the first build in every exported
    array and in its answers, in the FP32, BF16+rerank and leaf forms."""
    import torch
    cc = U.case(n=20000, d=48, N_r=64, frac=0.05, nq=120, seed=93)
    other = U.case(n=16000, d=48, N_r=64, frac=0.05, nq=10, seed=94, kind="integer")
    Q = t(cc["Q"])

    def build_and_answer():
        idx = dl.build_index(cc["X"], 4, 16, 64, 0.05, A=cc["A"], sample_ids=cc["sample"], keep_bf16=True)
        out = [idx.query(Q, 10, 1.5, 0.1), idx.query(Q, 10, 1.5, 0.1, precision=dl.BF16_RERANK),
               idx.query(Q, 10, 1.5, 0.1, granularity="leaf")]
        ex = idx.export()
        trees = [idx.tree(i) for i in range(4)]
        torch.cuda.synchronize()
        idx.free()
        return out, ex, trees

    dl.trim()
    say("first build on fresh memory")
    out0, ex0, tr0 = build_and_answer()
    say("an index of another size and data, freed into the cache")
    idx2 = dl.build_index(other["X"], 4, 16, 64, 0.05, A=other["A"], sample_ids=other["sample"], keep_bf16=True)
    idx2.query(t(other["Q"]), 10, 1.5, 0.1)
    torch.cuda.synchronize()
    idx2.free()
    say("rebuild on the cached arrays")
    out1, ex1, tr1 = build_and_answer()
    for (i0, d0), (i1, d1) in zip(out0, out1):
        assert torch.equal(i0, i1) and torch.equal(d0, d1)
    for key in ("A", "B", "codes", "sample_ids"):
        assert np.array_equal(ex0[key], ex1[key]), key
    for a, b in zip(tr0, tr1):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    dl.trim()
