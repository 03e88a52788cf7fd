"""DET-LSH indexing-and-query hot path on one MI355X (gfx950).

Python binding of the C ABI in include/detlsh.h.  It only marshals arguments:
torch supplies device memory and the current stream; every step of the method
runs in the HIP kernels of libdetlsh.so.  Nothing here computes on the CPU.

    import paper_2406_10938_amd as dl
    idx = dl.build_index(X, L=4, K=16, N_r=256, sample_frac=0.01)
    ids, dists = idx.query(Q, k=10, c=1.5, beta=0.1)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import BF16_RERANK, FP32, PROJ_GAUSSIAN, PROJ_PAA, RMIN_FIXED, RMIN_MAGIC, DetlshError, check, lib

__all__ = ["build_index", "import_index", "load_index", "Index", "Server", "DetlshError", "FP32", "BF16_RERANK",
           "RMIN_MAGIC", "RMIN_FIXED", "PROJ_GAUSSIAN", "PROJ_PAA", "profile_enable", "profile_read", "profile_counters",
           "trim"]


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f32(x, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(np.asarray(x, np.float32))
    if x.device.type != "cuda":
        x = x.to("cuda")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return x.contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _build_opts(seed, max_leaf, keep_bf16, proj_bf16, A, sample_ids, keep, projection=PROJ_GAUSSIAN, borrow_x=False):
    o = _lib.BuildOpts()
    o.borrow_x = int(bool(borrow_x))
    o.projection = {"gaussian": PROJ_GAUSSIAN, "paa": PROJ_PAA}.get(projection, projection)
    o.seed = int(seed)
    o.max_leaf = int(max_leaf)
    o.keep_bf16 = int(bool(keep_bf16))
    o.proj_bf16 = int(bool(proj_bf16))
    if A is not None:
        a = np.ascontiguousarray(A, np.float32)
        keep.append(a)
        o.A = a.ctypes.data_as(C.POINTER(C.c_float))
    if sample_ids is not None:
        s = np.ascontiguousarray(sample_ids, np.int64)
        keep.append(s)
        o.sample_ids = s.ctypes.data_as(C.POINTER(C.c_int64))
    return o


def _query_opts(precision, rerank_mult, rmin_policy, r_min, max_rounds, workspace_bytes, verify=0,
                granularity="point", filter="auto"):
    o = _lib.QueryOpts()
    o.filter = {"auto": 0, "plain": 1, "screen": 2}.get(filter, filter)
    o.granularity = {"point": 0, "leaf": 1}.get(granularity, granularity)
    o.verify = {"auto": 0, "gather": 1, "dense": 2, "dense_bf16": 3}.get(verify, verify)
    o.precision = int(precision)
    o.rerank_mult = int(rerank_mult)
    o.rmin_policy = int(rmin_policy)
    o.r_min = float(r_min)
    o.max_rounds = int(max_rounds)
    o.workspace_bytes = int(workspace_bytes)
    return o


class Index:
    """A built DET-LSH index resident in HBM (owned by the library)."""

    def __init__(self, handle):
        self._h = handle

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None):
            try:
                lib().detlsh_free(self._h)
            except TypeError:   # interpreter shutdown: the module is already torn down
                pass
            self._h = None
            self._borrowed_x = None

    @property
    def info(self) -> dict:
        inf = _lib.Info()
        check(lib().detlsh_index_info(self._h, C.byref(inf)))
        return {"n": inf.n, "d": inf.d, "L": inf.L, "K": inf.K, "N_r": inf.N_r, "n_s": inf.n_s,
                "max_leaf": inf.max_leaf, "has_bf16": bool(inf.has_bf16),
                "n_leaves": list(inf.n_leaves[:inf.L]), "device_bytes": inf.device_bytes}

    def project(self, Q):
        torch = _torch()
        Q = _dev_f32(Q, "Q")
        inf = self.info
        out = torch.empty((Q.shape[0], inf["L"] * inf["K"]), dtype=torch.float32, device=Q.device)
        check(lib().detlsh_project(self._h, _ptr(Q), Q.shape[0], _ptr(out), _stream_ptr()))
        return out

    def query(self, Q, k, c=1.5, beta=0.1, precision=FP32, rerank_mult=4, rmin_policy=RMIN_MAGIC,
              r_min=0.0, max_rounds=0, workspace_bytes=0, verify="auto", granularity="point", filter="auto"):
        torch = _torch()
        Q = _dev_f32(Q, "Q")
        nq = Q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
        dists = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        o = _query_opts(precision, rerank_mult, rmin_policy, r_min, max_rounds, workspace_bytes, verify, granularity,
                        filter)
        check(lib().detlsh_query(self._h, _ptr(Q), nq, int(k), float(c), float(beta), C.byref(o), _ptr(ids),
                                 _ptr(dists), _stream_ptr()))
        return ids, dists

    def query_async(self, Q, k, c=1.5, beta=0.1, precision=FP32, rerank_mult=4, rmin_policy=RMIN_MAGIC,
                    r_min=0.0, max_rounds=0, workspace_bytes=0, verify="auto", granularity="point",
                    filter="auto"):
        """detlsh_query_async on torch's current stream: returns (ids, dists,
        status) as soon as the work is enqueued.  The outputs are allocated on
        that stream and are complete once the stream has run past the call;
        Q must not be freed or overwritten before then.  status[q] != 0 marks
        a query that needs one of detlsh_query's fallbacks."""
        torch = _torch()
        Q = _dev_f32(Q, "Q")
        nq = Q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
        dists = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        status = torch.empty(nq, dtype=torch.int32, device=Q.device)
        o = _query_opts(precision, rerank_mult, rmin_policy, r_min, max_rounds, workspace_bytes, verify, granularity,
                        filter)
        check(lib().detlsh_query_async(self._h, _ptr(Q), nq, int(k), float(c), float(beta), C.byref(o), _ptr(ids),
                                       _ptr(dists), _ptr(status), _stream_ptr()))
        return ids, dists, status

    def query_noalloc(self, Q, k, c=1.5, beta=0.1, precision=FP32, rerank_mult=4, verify="auto",
                      granularity="point"):
        """detlsh_query inside the library's fixed device array: the call
        allocates no device memory (the outputs here are the caller's)."""
        torch = _torch()
        Q = _dev_f32(Q, "Q")
        nq = Q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
        dists = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        o = _query_opts(precision, rerank_mult, RMIN_MAGIC, 0.0, 0, 0, verify, granularity)
        check(lib().detlsh_query_noalloc(self._h, _ptr(Q), nq, int(k), float(c), float(beta), C.byref(o),
                                         _ptr(ids), _ptr(dists), _stream_ptr()))
        return ids, dists

    def query_rc(self, Q, r, c=1.5, beta=0.1):
        """(r, c)-ANN query (Alg. 6): per query the nearest point of S, or id -1
        and distance +inf when the algorithm returns nothing."""
        torch = _torch()
        Q = _dev_f32(Q, "Q")
        nq = Q.shape[0]
        ids = torch.empty(nq, dtype=torch.int64, device=Q.device)
        dists = torch.empty(nq, dtype=torch.float32, device=Q.device)
        check(lib().detlsh_query_rc(self._h, _ptr(Q), nq, float(r), float(c), float(beta), None, _ptr(ids),
                                    _ptr(dists), _stream_ptr()))
        return ids, dists

    def insert(self, X_new):
        """Append rows (ids n..n+m-1), encoded with the frozen breakpoints."""
        X_new = _dev_f32(X_new, "X_new")
        check(lib().detlsh_insert(self._h, _ptr(X_new), X_new.shape[0], _stream_ptr()))

    def save(self, path):
        """Write the index to `path` (rebuilt bit-identically by load_index)."""
        check(lib().detlsh_index_save(self._h, str(path).encode()))

    def query_debug(self, Q, k, c=1.5, beta=0.1, Qp=None, cand_cap=None, precision=FP32, rerank_mult=4,
                    rmin_policy=RMIN_MAGIC, r_min=0.0, max_rounds=0, workspace_bytes=0, verify="auto",
                    granularity="point", filter="auto"):
        """Query that also returns S, first trees, thr, stop tree and rounds."""
        torch = _torch()
        Q = _dev_f32(Q, "Q")
        nq = Q.shape[0]
        inf = self.info
        cap = int(cand_cap or inf["n"])
        dev = Q.device
        ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
        dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
        cand = torch.full((nq, cap), -1, dtype=torch.int32, device=dev)
        counts = torch.zeros(nq, dtype=torch.int64, device=dev)
        first = torch.zeros((nq, cap), dtype=torch.int32, device=dev)
        thr = torch.zeros(nq, dtype=torch.float32, device=dev)
        stop = torch.zeros(nq, dtype=torch.int32, device=dev)
        rounds = torch.zeros(nq, dtype=torch.int32, device=dev)
        qp_ptr = C.c_void_p(0)
        if Qp is not None:
            Qp = _dev_f32(Qp, "Qp")
            qp_ptr = _ptr(Qp)
        o = _query_opts(precision, rerank_mult, rmin_policy, r_min, max_rounds, workspace_bytes, verify, granularity,
                        filter)
        check(lib().detlsh_query_debug(self._h, qp_ptr, _ptr(Q), nq, int(k), float(c), float(beta), C.byref(o),
                                       _ptr(cand), cap, _ptr(counts), _ptr(first), _ptr(thr), _ptr(stop),
                                       _ptr(rounds), _ptr(ids), _ptr(dists), _stream_ptr()))
        return {"ids": ids, "dists": dists, "cand": cand, "counts": counts, "first_tree": first, "thr": thr,
                "stop_tree": stop, "rounds": rounds}

    def export(self):
        """Host copies of A, B, codes (n x L*K) and the sample ids."""
        inf = self.info
        LK = inf["L"] * inf["K"]
        A = np.empty((LK, inf["d"]), np.float32)
        B = np.empty((LK, inf["N_r"] + 1), np.float32)
        codes = np.empty((inf["n"], LK), np.uint8)
        sample = np.empty(max(inf["n_s"], 1), np.int64)
        check(lib().detlsh_export(self._h, A.ctypes.data_as(C.c_void_p), B.ctypes.data_as(C.c_void_p),
                                  codes.ctypes.data_as(C.c_void_p), sample.ctypes.data_as(C.c_void_p)))
        return {"A": A, "B": B, "codes": codes, "sample_ids": sample[:inf["n_s"]]}

    def tree(self, i):
        """DE-Tree i as (perm, leaf_start, leaf_lo, leaf_hi) host arrays."""
        inf = self.info
        nl = inf["n_leaves"][i]
        perm = np.empty(inf["n"], np.int32)
        start = np.empty(nl + 1, np.int32)
        lo = np.empty((max(nl, 1), inf["K"]), np.uint8)
        hi = np.empty((max(nl, 1), inf["K"]), np.uint8)
        check(lib().detlsh_export_tree(self._h, int(i), perm.ctypes.data_as(C.c_void_p),
                                       start.ctypes.data_as(C.c_void_p), lo.ctypes.data_as(C.c_void_p),
                                       hi.ctypes.data_as(C.c_void_p), max(nl, 1)))
        return perm, start, lo[:nl], hi[:nl]


class Server:
    """Continuous-batching query server over one index (detlsh_server_* in the C ABI).

    submit() returns a ticket at once; wait(ticket) returns (ids, dists, info)
    when the request's results are complete.  The server allocates its device
    workspace once, at construction.
    """

    def __init__(self, index: Index, workspace_bytes: int, slots: int = 2, max_batch: int = 1024):
        self._index = index   # the index must outlive the server
        h = C.c_void_p()
        check(lib().detlsh_server_create(index._h, int(workspace_bytes), int(slots), int(max_batch), C.byref(h)))
        self._h = h
        self._live = {}

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            lib().detlsh_server_destroy(self._h)
            self._h = None
            self._live = {}

    def submit(self, Q, k, c=1.5, beta=0.1, precision=FP32, rerank_mult=4, rmin_policy=RMIN_MAGIC, r_min=0.0,
               max_rounds=0, verify="auto", granularity="point", sync=True, filter="auto") -> int:
        """Queue Q (nq x d) for k-ANN; the server reads Q on its own streams, so
        with sync=True the current stream is synchronised first."""
        torch = _torch()
        Q = _dev_f32(Q, "Q")
        nq = Q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
        dists = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        if sync:
            torch.cuda.current_stream().synchronize()
        o = _query_opts(precision, rerank_mult, rmin_policy, r_min, max_rounds, 0, verify, granularity, filter)
        t = C.c_uint64()
        check(lib().detlsh_server_submit(self._h, _ptr(Q), nq, int(k), float(c), float(beta), C.byref(o), _ptr(ids),
                                         _ptr(dists), C.byref(t)))
        self._live[t.value] = (Q, ids, dists)
        return t.value

    def wait(self, ticket, timeout=None):
        """(ids, dists, info) of a finished request; None if `timeout` seconds
        passed first.  Raises DetlshError with the request's status on failure."""
        us = -1 if timeout is None else int(timeout * 1e6)
        inf = _lib.RequestInfo()
        st = lib().detlsh_server_wait(self._h, int(ticket), us, C.byref(inf))
        if st == _lib.EBUSY:
            return None
        bufs = self._live.pop(int(ticket), None)
        check(st)
        info = {"t_submit": inf.t_submit, "t_start": inf.t_start, "t_end": inf.t_end, "batches": inf.batches,
                "max_batch_requests": inf.max_batch_requests, "max_batch_queries": inf.max_batch_queries}
        return bufs[1], bufs[2], info

    def cancel(self, ticket) -> bool:
        """True if the cancellation took effect, False if the request had finished."""
        st = lib().detlsh_server_cancel(self._h, int(ticket))
        if st == _lib.EBUSY:
            return False
        check(st)
        return True


def build_index(X, L=4, K=16, N_r=256, sample_frac=0.01, A=None, sample_ids=None, seed=0, max_leaf=256,
                keep_bf16=False, proj_bf16=False, projection="gaussian", borrow_x=False) -> Index:
    """Encoding and indexing phases over X (n x d float32, device or host).
    projection="paa" with L=1 is DET-ONLY (PAA segment means).  borrow_x: the
    index reads X's device memory in place (no copy); the index holds a
    reference to the tensor, which must not be modified while the index lives."""
    X = _dev_f32(X, "X")
    keep = []
    o = _build_opts(seed, max_leaf, keep_bf16, proj_bf16, A, sample_ids, keep, projection, borrow_x)
    h = C.c_void_p()
    check(lib().detlsh_build_index(_ptr(X), X.shape[0], X.shape[1], int(L), int(K), int(N_r), float(sample_frac),
                                   C.byref(o), _stream_ptr(), C.byref(h)))
    idx = Index(h)
    if borrow_x:
        idx._borrowed_x = X
    return idx


def import_index(X, A, B, codes, L, K, N_r, max_leaf=256, keep_bf16=False) -> Index:
    """Index from given projection matrix, breakpoints and codes (host arrays)."""
    X = _dev_f32(X, "X")
    A = np.ascontiguousarray(A, np.float32)
    B = np.ascontiguousarray(B, np.float32)
    codes = np.ascontiguousarray(codes, np.uint8)
    keep = []
    o = _build_opts(0, max_leaf, keep_bf16, False, None, None, keep)
    h = C.c_void_p()
    check(lib().detlsh_index_import(_ptr(X), X.shape[0], X.shape[1], int(L), int(K), int(N_r),
                                    A.ctypes.data_as(C.c_void_p), B.ctypes.data_as(C.c_void_p),
                                    codes.ctypes.data_as(C.c_void_p), C.byref(o), _stream_ptr(), C.byref(h)))
    return Index(h)


def load_index(path) -> Index:
    """Index written by Index.save, on the current device."""
    h = C.c_void_p()
    check(lib().detlsh_index_load(str(path).encode(), _stream_ptr(), C.byref(h)))
    return Index(h)


def trim():
    """Free the idle query workspaces that earlier query calls left for reuse."""
    lib().detlsh_trim()


def profile_enable(on=True, reset=True):
    check(lib().detlsh_profile_enable(int(on), int(reset)))


def probe_valu(nq=2048, lanes=256 * 1024 * 3):
    """Measured lane operations per second of the range filter's bound
    arithmetic (3 per tree and dimension plus 1 per tree, L = 4, K = 16) on the
    current device, and the probe launch's duration in ms."""
    rate = C.c_double()
    ms = C.c_double()
    check(lib().detlsh_probe_valu(int(nq), int(lanes), C.byref(rate), C.byref(ms)))
    return rate.value, ms.value


def profile_counters() -> dict:
    """Work counters of the profiled queries (see detlsh_profile_counters):
    {"exact_survivors": n, "exact_candidates": n}."""
    names = (C.c_char_p * 8)()
    vals = (C.c_int64 * 8)()
    cnt = C.c_int32()
    check(lib().detlsh_profile_counters(names, vals, 8, C.byref(cnt)))
    return {names[i].decode(): vals[i] for i in range(cnt.value)}


def profile_read() -> dict:
    names = (C.c_char_p * 32)()
    launches = (C.c_int64 * 32)()
    ms = (C.c_double * 32)()
    cnt = C.c_int32()
    check(lib().detlsh_profile_read(names, launches, ms, 32, C.byref(cnt)))
    return {names[i].decode(): {"launches": launches[i], "ms": ms[i]} for i in range(cnt.value)}
