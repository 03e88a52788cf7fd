"""Serving form: continuous batching over a fixed workspace (detlsh_server_*).

Every request served in a mix (merged with other requests, split across
batches and slots, run in a tight workspace in several passes) returns ids and
distances bit-identical to the same request run alone through detlsh_query,
whose parity with the oracle the other GPU tests establish (determinism
independent of batch composition, P12).  Invalid, oversized and cancelled
requests fail on their own tickets while the others are served.
"""
import ctypes as C

import numpy as np
import pytest

import gpu_util as U

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2406_10938_amd as dl
    say("serve: build n=80000 d=96 keep_bf16")
    c = U.case(n=80_000, d=96, N_r=256, frac=0.01, nq=1500, seed=41)
    idx = dl.build_index(c["X"], 4, 16, 256, 0.01, A=c["A"], sample_ids=c["sample"], keep_bf16=True)
    Q = torch.as_tensor(c["Q"]).cuda()
    return dict(dl=dl, idx=idx, Q=Q, d=c["d"], torch=torch)


def _requests(seed, nreq, Q):
    """Seeded request mix: log-uniform nq in 1..96, k in {1, 10, 100},
    c in {1.5, 2.0}; mostly FP32 MAGIC, some BF16 + rerank and FIXED ladders."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(nreq):
        nq = int(min(96, max(1, np.floor(np.exp(rng.uniform(0, np.log(97)))))))
        q0 = int(rng.integers(0, Q.shape[0] - nq))
        kw = dict(k=int(rng.choice([1, 10, 100])), c=float(rng.choice([1.5, 2.0])), beta=0.1)
        form = rng.random()
        if form < 0.15:
            kw["precision"] = 1
        elif form < 0.25:
            kw.update(rmin_policy=1, r_min=2.0, max_rounds=16)
            kw["k"] = min(kw["k"], 10)
        reqs.append((Q[q0:q0 + nq], kw))
    return reqs


def _alone(idx, reqs):
    return [tuple(t.cpu().numpy() for t in idx.query(q, **kw)) for q, kw in reqs]


def _serve(dl, idx, reqs, **skw):
    srv = dl.Server(idx, **skw)
    try:
        tickets = [srv.submit(q, **kw) for q, kw in reqs]
        out = []
        for t in tickets:
            ids, d, info = srv.wait(t)
            out.append((ids.cpu().numpy(), d.cpu().numpy(), info))
        return out
    finally:
        srv.close()


@pytest.mark.parametrize("ws_mb,slots,max_batch", [(512, 3, 64), (24, 2, 1024), (256, 1, 16)])
def test_alone_vs_mix_bit_identical(env, ws_mb, slots, max_batch):
    dl, idx = env["dl"], env["idx"]
    # a large request first: while its pieces occupy the slots, the later
    # requests queue up and are merged by parameters
    reqs = [(env["Q"][:1000], dict(k=10, c=1.5, beta=0.1))] + _requests(7 + slots, 40, env["Q"])
    say(f"serve: {len(reqs)} requests alone, then in a mix ws={ws_mb}MB slots={slots} max_batch={max_batch}")
    ref = _alone(idx, reqs)
    got = _serve(dl, idx, reqs, workspace_bytes=ws_mb << 20, slots=slots, max_batch=max_batch)
    merged = split = 0
    for i, ((ri, rd), (gi, gd, info)) in enumerate(zip(ref, got)):
        assert np.array_equal(ri, gi), (i, reqs[i][1])
        assert np.array_equal(rd, gd), (i, reqs[i][1])
        assert info["t_submit"] <= info["t_start"] <= info["t_end"]
        merged += info["max_batch_requests"] > 1
        split += info["batches"] > 1
    say(f"  requests merged with others: {merged}, split over batches: {split}")
    assert merged > 0
    if max_batch < 96 or ws_mb < 64:
        assert split > 0


def test_failure_isolation_and_cancel(env):
    dl, idx, Q, torch = env["dl"], env["idx"], env["Q"], env["torch"]
    reqs = _requests(3, 24, Q)
    ref = _alone(idx, reqs)
    srv = dl.Server(idx, workspace_bytes=256 << 20, slots=1, max_batch=32)
    try:
        tickets = []
        for i, (q, kw) in enumerate(reqs):
            tickets.append(srv.submit(q, **kw))
            # invalid requests between valid ones: rejected at submit, no ticket
            if i == 3:
                with pytest.raises(dl.DetlshError, match="EINVAL"):
                    srv.submit(q, 0, 1.5, 0.1)
            if i == 5:
                with pytest.raises(dl.DetlshError, match="EINVAL"):
                    srv.submit(q, 10, 1.0, 0.1)
            if i == 7:
                with pytest.raises(dl.DetlshError, match="EINVAL"):
                    srv.submit(q, 300, 1.5, 0.1, precision=dl.BF16_RERANK)   # rerank_mult*k > 1024
            if i == 9:
                host = np.zeros((2, env["d"]), np.float32)
                ids = torch.empty((2, 10), dtype=torch.int64, device="cuda")
                ds = torch.empty((2, 10), dtype=torch.float32, device="cuda")
                t = C.c_uint64()
                st = dl._lib.lib().detlsh_server_submit(srv._h, host.ctypes.data_as(C.c_void_p), 2, 10, 1.5, 0.1,
                                                        None, C.c_void_p(ids.data_ptr()),
                                                        C.c_void_p(ds.data_ptr()), C.byref(t))
                assert st == dl._lib.EINVAL and t.value == 0
        empty = srv.submit(Q[:0], 10, 1.5, 0.1)
        cancelled = {}
        for i in (20, 22, 23):
            cancelled[i] = srv.cancel(tickets[i])
        for i, t in enumerate(tickets):
            if cancelled.get(i):
                with pytest.raises(dl.DetlshError, match="ECANCELED"):
                    srv.wait(t)
                continue
            ids, d, _ = srv.wait(t)
            assert np.array_equal(ids.cpu().numpy(), ref[i][0]) and np.array_equal(d.cpu().numpy(), ref[i][1])
        ids, d, info = srv.wait(empty)
        assert ids.shape == (0, 10) and info["batches"] == 0
        with pytest.raises(dl.DetlshError, match="EINVAL"):
            srv.wait(tickets[0])                       # released by its wait
        say(f"  cancellations that took effect: {sum(cancelled.values())} of {len(cancelled)}")
    finally:
        srv.close()


def test_workspace_admission(env):
    """A request of which not one query fits a slot's workspace is refused
    with ENOMEM at submit; a server with room serves it."""
    dl, idx, Q = env["dl"], env["idx"], env["Q"]
    tiny = dl.Server(idx, workspace_bytes=1 << 20, slots=1)
    try:
        with pytest.raises(dl.DetlshError, match="ENOMEM"):
            tiny.submit(Q[:4], 10, 1.5, 0.1)
    finally:
        tiny.close()
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        dl.Server(idx, workspace_bytes=1000, slots=1)
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        dl.Server(idx, workspace_bytes=1 << 30, slots=17)


def test_poll_and_destroy_with_pending(env):
    """wait with a zero timeout returns at once; destroying a server with
    requests still queued cancels them and returns."""
    dl, idx, Q = env["dl"], env["idx"], env["Q"]
    srv = dl.Server(idx, workspace_bytes=128 << 20, slots=1, max_batch=8)
    ts = [srv.submit(Q[i * 40:(i + 1) * 40], 10, 1.5, 0.1) for i in range(12)]
    r = srv.wait(ts[-1], timeout=0)
    assert r is None or r[0].shape == (40, 10)
    ids, d, _ = srv.wait(ts[0])
    ref_ids, ref_d = idx.query(Q[:40], 10, 1.5, 0.1)
    assert np.array_equal(ids.cpu().numpy(), ref_ids.cpu().numpy())
    srv.close()
