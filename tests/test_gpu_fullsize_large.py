"""Parity at the two largest workloads, at full size and in the benchmark's
launch configuration (default workspace, the same query chunking):

  d = 960 Beta-copula set  n = 10^6,  1,000 queries, k = 10, beta = 0.5
  normalised mixture       n = 10^7, 10,000 queries, k = 10, beta = 0.01
                                                      (k = 100, beta = 0.05)

Sampled queries are recomputed one by one by the FP64 oracle on the GPU's own
encoding (candidate sets up to points on the threshold, ids up to distance
near-ties, distances within 1e-5 relative).  Every query is checked for the
properties that hold at any size, the two exact FP32 forms (BF16-product and
FP32-product screens) are compared bit for bit on all queries, and the
BF16+rerank form (BF16 projection and products) is measured against the
oracle's answers: recall and overall ratio (Sec. 6.1), asserted at >= 0.95 and
<= 1.01."""
import math

import numpy as np
import pytest

import gpu_util as U
from oracle import detlsh_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _load(name, k, beta, n_oracle):
    import torch

    import paper_2406_10938_amd as dl
    import synth
    assert torch.cuda.is_available()
    cfg = synth.config(name)
    dev = torch.device("cuda:0")
    say(f"full-size {name}: generating n={cfg.n} d={cfg.d} nq={cfg.nq}")
    Xd = synth.make_data(cfg, device=dev)
    Qd = synth.make_queries(cfg, device=dev)
    A = synth.projection_matrix(cfg.L, cfg.K, cfg.d, cfg.index_seed)
    sample = synth.sample_ids(cfg.n, cfg.n_s, cfg.index_seed)
    say(f"full-size {name}: build (FP32 projection, BF16 copy kept)")
    idx = dl.build_index(Xd, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
    X = Xd.cpu().numpy().astype(np.float64)
    Q = Qd.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(17)
    picks = sorted(rng.choice(cfg.nq, n_oracle, replace=False).tolist())
    return dict(dl=dl, cfg=cfg, Xd=Xd, Qd=Qd, A=A, sample=sample, idx=idx, X=X, Q=Q, picks=picks, k=k,
                beta=beta)


def _oracle_answers(w):
    """The oracle's answers to the picked queries on the GPU's encoding."""
    cfg, idx = w["cfg"], w["idx"]
    ex = idx.export()
    Qp = idx.project(w["Qd"]).cpu().numpy()
    out = {}
    for qi in w["picks"]:
        say(f"  oracle on query {qi}")
        out[qi] = U.oracle_query(w["X"], w["Q"][qi], Qp[qi], ex["codes"], ex["B"], cfg.L, cfg.K, w["k"], w["beta"])
    return ex, Qp, out


def _check_sampled(w, ex, Qp, refs):
    import torch
    cfg, idx, k, beta = w["cfg"], w["idx"], w["k"], w["beta"]
    ids, dists = (v.cpu().numpy() for v in idx.query(w["Qd"], k, cfg.c, beta))
    near_ties = 0
    for qi, ref in refs.items():
        r = idx.query_debug(w["Qd"][qi:qi + 1], k, cfg.c, beta, Qp=torch.from_numpy(Qp[qi:qi + 1]).cuda())
        S = set(r["cand"][0, :int(r["counts"][0])].cpu().numpy().tolist())
        sym = S ^ set(ref.S.tolist())
        assert sym <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], cfg.L, cfg.K, ref.thr)
        if not sym:
            near_ties += U.compare_result(ref.ids, ref.dists, w["X"], w["Q"][qi], ids[qi], dists[qi], ref.S, k)
    say(f"  {len(refs)} sampled queries match the oracle ({near_ties} positions differ at near-ties)")


def _check_every_query(w):
    import torch
    cfg, idx, k, beta = w["cfg"], w["idx"], w["k"], w["beta"]
    N_S = k + math.ceil(beta * cfg.n)
    a_ids, a_d = idx.query(w["Qd"], k, cfg.c, beta)                    # BF16-product screen
    b_ids, b_d = idx.query(w["Qd"], k, cfg.c, beta, verify="dense")    # FP32 products
    assert torch.equal(a_ids, b_ids) and torch.equal(a_d, b_d)
    d = a_d.cpu().numpy()
    assert np.all(np.diff(d, axis=1) >= 0)
    for s in range(0, cfg.nq, 1000):
        ids = a_ids[s:s + 1000]
        exact = ((w["Xd"][ids].double() - w["Qd"][s:s + 1000, None, :].double()) ** 2).sum(-1).sqrt()
        np.testing.assert_allclose(d[s:s + 1000], exact.cpu().numpy(), rtol=1e-5)
    r = idx.query_debug(w["Qd"], k, cfg.c, beta, cand_cap=1)
    assert np.all(r["counts"].cpu().numpy() >= N_S)
    assert np.array_equal(r["ids"].cpu().numpy(), a_ids.cpu().numpy())


def _check_bf16_form(w, refs):
    """BF16 projection and products, top-4k reranked in FP32: recall and
    overall ratio against the oracle's answers."""
    cfg, dl = w["cfg"], w["dl"]
    ib = dl.build_index(w["Xd"], cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=w["A"], sample_ids=w["sample"],
                        keep_bf16=True, proj_bf16=True)
    ids, dists = (v.cpu().numpy() for v in ib.query(w["Qd"], w["k"], cfg.c, w["beta"], precision=dl.BF16_RERANK))
    ib.free()
    rec, rat = [], []
    for qi, ref in refs.items():
        exact = np.sqrt(O.sq_dists(w["X"][ids[qi]], w["Q"][qi]))
        np.testing.assert_allclose(dists[qi], exact, rtol=1e-5)
        rec.append(O.recall(dists[qi], ref.dists))
        rat.append(O.overall_ratio(dists[qi], ref.dists))
    say(f"  BF16+rerank against the oracle: recall {np.mean(rec):.4f}, overall ratio {np.mean(rat):.6f}")
    assert np.mean(rec) >= 0.95 and np.mean(rat) <= 1.01


@pytest.fixture(scope="module")
def c3():
    w = _load("C3", 10, 0.5, 6)
    yield w
    w["idx"].free()


@pytest.fixture(scope="module")
def c4():
    w = _load("C4", 10, 0.01, 8)
    yield w
    w["idx"].free()


def test_c3_sampled_queries_match_oracle(c3):
    ex, Qp, refs = _oracle_answers(c3)
    c3["refs"] = refs
    _check_sampled(c3, ex, Qp, refs)


def test_c3_every_query_and_forms_agree(c3):
    _check_every_query(c3)


def test_c3_bf16_rerank_against_oracle(c3):
    _check_bf16_form(c3, c3["refs"])


def test_c4_sampled_queries_match_oracle(c4):
    ex, Qp, refs = _oracle_answers(c4)
    c4["refs"] = refs
    _check_sampled(c4, ex, Qp, refs)


def test_c4_every_query_and_forms_agree(c4):
    _check_every_query(c4)


def test_c4_bf16_rerank_against_oracle(c4):
    _check_bf16_form(c4, c4["refs"])


def test_c4_k100_sampled_queries_match_oracle(c4):
    """The configuration's own k = 100, beta = 0.05 on three sampled queries."""
    w = dict(c4, k=100, beta=0.05, picks=c4["picks"][:3])
    ex, Qp, refs = _oracle_answers(w)
    _check_sampled(w, ex, Qp, refs)
