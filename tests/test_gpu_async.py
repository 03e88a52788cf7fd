"""The stream-ordered query (detlsh_query_async): the same answers as
detlsh_query, every step enqueued without a host wait, and calls on two
streams running at the same time on the device, each with its solo answer."""
import time

import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def mix():
    import torch

    import paper_2406_10938_amd as dl
    assert torch.cuda.is_available()
    cfg = synth.config("C4")
    dev = torch.device("cuda:0")
    n = 1_000_000
    X = synth.make_data(cfg, n=n, device=dev)
    Q = synth.make_queries(cfg, nq=4000, device=dev)
    A = synth.projection_matrix(4, 16, cfg.d, cfg.index_seed)
    sample = synth.sample_ids(n, n // 100, cfg.index_seed)
    say(f"async: normalised mixture n={n} d={cfg.d}, building")
    idx = dl.build_index(X, 4, 16, 256, 0.01, A=A, sample_ids=sample, keep_bf16=True)
    yield dict(dl=dl, idx=idx, X=X, Q=Q)
    idx.free()


def _check_same(mix, kw, nq=700, k=10, beta=0.01):
    import torch
    idx, Q = mix["idx"], mix["Q"][:nq]
    ids0, d0 = idx.query(Q, k, 1.5, beta, **kw)
    ids1, d1, st = idx.query_async(Q, k, 1.5, beta, **kw)
    torch.cuda.synchronize()
    ok = st == 0
    say(f"  {kw}: {int(ok.sum())} of {nq} answered in stream order")
    assert torch.equal(ids0[ok], ids1[ok]) and torch.equal(d0[ok], d1[ok])
    return ok


@pytest.mark.parametrize("kw", [dict(), dict(verify="gather"), dict(precision=1), dict(filter="plain"),
                                dict(rmin_policy=1, r_min=0.05, max_rounds=12)],
                         ids=["magic", "gather", "bf16", "plain_filter", "fixed"])
def test_async_matches_sync(mix, kw):
    ok = _check_same(mix, kw)
    if kw.get("rmin_policy", 0) == 0:
        assert bool(ok.all())


def test_two_streams_overlap_and_keep_their_answers(mix):
    import torch
    idx, Q = mix["idx"], mix["Q"]
    Q1, Q2 = Q[:2000].contiguous(), Q[2000:4000].contiguous()
    solo1 = idx.query(Q1, 10, 1.5, 0.01)
    solo2 = idx.query(Q2, 10, 1.5, 0.01)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(2):   # the first pass fills the workspace cache
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s1):
            ev[0].record()
            r1 = idx.query_async(Q1, 10, 1.5, 0.01)
            ev[1].record()
        with torch.cuda.stream(s2):
            ev[2].record()
            r2 = idx.query_async(Q2, 10, 1.5, 0.01)
            ev[3].record()
        host_ms = (time.perf_counter() - t0) * 1e3
        torch.cuda.synchronize()
        end1 = ev[0].elapsed_time(ev[1])    # stream 1's work, from its start
        start2 = ev[0].elapsed_time(ev[2])  # stream 2's start, from stream 1's start
        end2 = ev[0].elapsed_time(ev[3])
        say(f"  pass {rep}: host {host_ms:.2f} ms to enqueue both; device: stream 1 [0, {end1:.2f}] ms, "
            f"stream 2 [{start2:.2f}, {end2:.2f}] ms")
    for r, solo in ((r1, solo1), (r2, solo2)):
        assert bool((r[2] == 0).all())
        assert torch.equal(r[0], solo[0]) and torch.equal(r[1], solo[1])
    # the second stream's work began before the first stream's had ended
    assert start2 < end1
    # enqueueing returned well before the device finished the work
    assert host_ms < max(end1, end2)


def test_back_to_back_calls_on_one_stream(mix):
    """A second call enqueued behind a first one on the same stream takes a
    workspace of its own (the first's is still in use) and both answers hold."""
    import torch
    idx, Q = mix["idx"], mix["Q"]
    a = idx.query(Q[:500], 10, 1.5, 0.01)
    b = idx.query(Q[500:1000], 10, 1.5, 0.01)
    ra = idx.query_async(Q[:500], 10, 1.5, 0.01)
    rb = idx.query_async(Q[500:1000], 10, 1.5, 0.01)
    torch.cuda.synchronize()
    for r, s in ((ra, a), (rb, b)):
        assert bool((r[2] == 0).all())
        assert torch.equal(r[0], s[0]) and torch.equal(r[1], s[1])
