"""detlsh_query_noalloc (the query inside the library's fixed device array)
against detlsh_query through the C ABI: bit-identical ids and distances on two
calls in a row, the second with a smaller input; sizes beyond the array and
the FIXED policy are refused before any work."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2406_10938_amd as dl
    n, d = 200_000, 48
    X = synth.gaussian_mixture(n, d, 64, 4.0, 1.0, 901)
    Q = synth.gaussian_mixture(700, d, 64, 4.0, 1.0, 901, rows_seed=902)
    A = synth.projection_matrix(4, 16, d, 903)
    sample = synth.sample_ids(n, n // 100, 904)
    Xd = torch.from_numpy(X).cuda()
    idx = dl.build_index(Xd, 4, 16, 256, 0.01, A=A, sample_ids=sample, keep_bf16=True)
    yield dl, torch, idx, torch.from_numpy(Q).cuda()
    idx.free()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_equals_query_twice_second_smaller(setup, precision):
    dl, torch, idx, Q = setup
    prec = dl.BF16_RERANK if precision == "bf16" else dl.FP32
    for nq, k, beta in ((700, 10, 0.1), (37, 5, 0.05)):
        print(f"[noalloc] {precision} nq={nq} k={k} beta={beta}", flush=True)
        ref_ids, ref_d = idx.query(Q[:nq], k, 1.5, beta, precision=prec)
        ids, dists = idx.query_noalloc(Q[:nq], k, 1.5, beta, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(ids, ref_ids)
        assert torch.equal(dists.view(torch.int32), ref_d.view(torch.int32))


def test_noalloc_refuses_what_does_not_fit(setup):
    dl, torch, idx, Q = setup
    L = dl.lib()
    cap = int(L.detlsh_noalloc_scratch_bytes())
    assert cap == 256 << 20
    nq = cap // (64 * 4) + 1                 # the projections alone exceed the array
    Qbig = torch.zeros((nq, Q.shape[1]), dtype=torch.float32, device=Q.device)
    ids = torch.empty((1, 1), dtype=torch.int64, device=Q.device)
    dd = torch.empty((1, 1), dtype=torch.float32, device=Q.device)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = L.detlsh_query_noalloc(idx._h, C.c_void_p(Qbig.data_ptr()), nq, 10, 1.5, 0.1, None,
                               C.c_void_p(ids.data_ptr()), C.c_void_p(dd.data_ptr()), st)
    assert r == dl._lib.ENOMEM
    assert b"bytes of scratch" in L.detlsh_last_error()
    with pytest.raises(dl.DetlshError, match="EINVAL"):
        o = dl._lib.QueryOpts()
        o.rmin_policy = dl.RMIN_FIXED
        o.r_min = 1.0
        dl._lib.check(L.detlsh_query_noalloc(idx._h, C.c_void_p(Q.data_ptr()), 4, 10, 1.5, 0.1, C.byref(o),
                                             C.c_void_p(ids.data_ptr()), C.c_void_p(dd.data_ptr()), st))
