"""Parity at the benchmark's full size and launch configuration: the SIFT-shaped
set (n = 10^6, d = 128), 10,000 queries, k = 10, beta = 0.1, default
workspace (the same chunking as bench.py), index with its BF16 copy.  Sampled queries are recomputed by
the FP64 oracle on the GPU's own encoding; every query is checked for the
properties that hold at any size (|S| >= N_S, sorted results, distances equal
to exact distances of the returned ids, determinism)."""
import math

import numpy as np
import pytest

import gpu_util as U
from oracle import detlsh_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    import torch

    import paper_2406_10938_amd as dl
    import synth
    assert torch.cuda.is_available()
    cfg = synth.config("C2")
    print("full-size C2: generating", flush=True)
    X = synth.make_data(cfg)
    Q = synth.make_queries(cfg)
    A = synth.projection_matrix(cfg.L, cfg.K, cfg.d, cfg.index_seed)
    sample = synth.sample_ids(cfg.n, cfg.n_s, cfg.index_seed)
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    print("full-size C2: build", flush=True)
    # with the BF16 copy, as bench.py builds it: the FP32 form screens with BF16 products
    idx = dl.build_index(Xd, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
    return dict(dl=dl, cfg=cfg, X=X, Q=Q, Xd=Xd, Qd=Qd, idx=idx)


def test_fullsize_sampled_queries_match_oracle(c2):
    import torch
    cfg, idx, X, Q = c2["cfg"], c2["idx"], c2["X"], c2["Q"]
    k, beta = 10, cfg.beta
    print("full-size C2: query 10,000", flush=True)
    ids, dists = idx.query(c2["Qd"], k, cfg.c, beta)
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    ex = idx.export()
    Qp = idx.project(c2["Qd"]).cpu().numpy()
    rng = np.random.default_rng(7)
    picks = sorted(rng.choice(len(Q), 8, replace=False).tolist()) + [0, len(Q) - 1]
    for qi in picks:
        print(f"  oracle on query {qi}", flush=True)
        ref = U.oracle_query(X, Q[qi], Qp[qi], ex["codes"], ex["B"], cfg.L, cfg.K, k, beta)
        r = idx.query_debug(c2["Qd"][qi:qi + 1], k, cfg.c, beta, Qp=torch.from_numpy(Qp[qi:qi + 1]).cuda())
        S = set(r["cand"][0, :int(r["counts"][0])].cpu().numpy().tolist())
        sym = S ^ set(ref.S.tolist())
        assert sym <= U.borderline_points(Qp[qi], ex["codes"], ex["B"], cfg.L, cfg.K, ref.thr)
        if not sym:
            # integer data: FP32 distances are exact, ids must match bit for bit
            assert np.array_equal(ids[qi], ref.ids), (qi, ids[qi], ref.ids)
            np.testing.assert_allclose(dists[qi], ref.dists, rtol=1e-6)


def test_fullsize_properties_every_query(c2):
    import torch
    cfg, idx = c2["cfg"], c2["idx"]
    k, beta = 10, cfg.beta
    N_S = k + math.ceil(beta * cfg.n)
    ids, dists = idx.query(c2["Qd"], k, cfg.c, beta)
    ids2, dists2 = idx.query(c2["Qd"], k, cfg.c, beta)
    assert torch.equal(ids, ids2) and torch.equal(dists, dists2)
    d = dists.cpu().numpy()
    assert np.all(np.diff(d, axis=1) >= 0)
    exact = ((c2["Xd"][ids].double() - c2["Qd"][:, None, :].double()) ** 2).sum(-1).sqrt().cpu().numpy()
    np.testing.assert_allclose(d, exact, rtol=1e-6)
    r = idx.query_debug(c2["Qd"], k, cfg.c, beta, cand_cap=1)
    counts = r["counts"].cpu().numpy()
    assert np.all(counts >= N_S)
    assert np.all(r["stop_tree"].cpu().numpy() >= 1)
    assert np.array_equal(r["ids"].cpu().numpy(), ids.cpu().numpy())


def test_fullsize_bf16_screen_equals_fp32_products(c2):
    """Every one of the 10,000 answers of the FP32 form is bit-identical whether
    the dense pass screens with BF16 products (the benchmark's path) or with
    FP32 products."""
    import torch
    cfg, idx = c2["cfg"], c2["idx"]
    print("full-size C2: BF16 screen vs FP32 products", flush=True)
    a_ids, a_d = idx.query(c2["Qd"], 10, cfg.c, cfg.beta, verify="dense_bf16")
    b_ids, b_d = idx.query(c2["Qd"], 10, cfg.c, cfg.beta, verify="dense")
    assert torch.equal(a_ids, b_ids)
    assert torch.equal(a_d, b_d)
