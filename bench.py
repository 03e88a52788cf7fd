#!/usr/bin/env python3
"""Benchmark of the DET-LSH hot path on one MI355X.

One step = the whole hot path over one batch: build the index over the
SIFT-shaped set (n = 1,000,000, d = 128, integers in [0, 255]; L = 4, K = 16,
N_r = 256, 1% breakpoint sample) and answer 10,000 queries from the same
generator (k = 10, c = 1.5, beta = 0.1) with plain FP32 verification.  Inputs
are resident in HBM before the timed region.  `value` is the whole-step
throughput in queries/s (build included); the query-only rate and the build
rate are reported beside it.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build uses one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # lane-ops/s without packed FP32: 39.32 T
FP32_MFMA_PEAK = 157.3           # TFLOP/s dense


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ground_truth_kth(X, Q, k, chunk=1000):
    """Exact k-th nearest distance per query (recall reading: a returned point
    counts when its distance is <= this).  FP32 products of integers < 2^24 are
    exact; candidates are re-measured in float64."""
    import torch
    xn = (X.double() ** 2).sum(1).float()
    out = torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device)
    for s in range(0, Q.shape[0], chunk):
        q = Q[s:s + chunk]
        d2 = xn[None, :] - 2.0 * (q @ X.T) + (q.double() ** 2).sum(1).float()[:, None]
        cand = torch.topk(d2, k + 32, dim=1, largest=False).indices
        exact = ((X[cand].double() - q[:, None, :].double()) ** 2).sum(-1)
        out[s:s + chunk] = torch.sort(exact, dim=1).values[:, k - 1].sqrt()
    return out


def recall_at_k(X, Q, ids, k, kth):
    import torch
    d = ((X[ids].double() - Q[:, None, :].double()) ** 2).sum(-1).sqrt()
    hit = (d <= kth[:, None] * (1 + 1e-12)).sum(1).clamp(max=k)
    return float(hit.double().mean() / k)


def counted_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, scaled by the
    copy calibration) from the committed counter summaries under profiles/, or
    None when none matches the current kernel source."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic-per-launch "):
                continue
            f = dict(kv.split("=", 1) for kv in line.split()[2:])
            if line.split()[1] != kernel:
                continue
            src = os.path.join(ROOT, f["source"])
            if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != f["sha256"]:
                return None
            return int(f["read_bytes"]) + int(f["write_bytes"])
    return None


def cpu_baseline(X_host, Q_host, A, sample, cfg, k, beta, nq_total, n_queries):
    """The FP64 oracle on the host cores (one BLAS thread): full-n build, then
    `n_queries` queries; scaled to whole-job queries/s."""
    from threadpoolctl import threadpool_limits

    from oracle import detlsh_oracle as O
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        idx = O.build_index(X_host, A, sample, cfg.L, cfg.K, cfg.N_r)
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        for qi in range(n_queries):
            qp = O.project(Q_host[qi:qi + 1], A)[0]
            O.query_magic(X_host, Q_host[qi], qp, idx.codes, idx.B, cfg.L, cfg.K, k, beta)
        t_q = (time.perf_counter() - t0) / n_queries
    total = t_build + nq_total * t_q
    return {"value": nq_total / total, "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle, 1 thread: full build over n={X_host.shape[0]} "
                       f"({t_build:.2f} s) + {n_queries} of the {nq_total} queries "
                       f"({t_q * 1e3:.1f} ms each), scaled to the whole step"),
            "build_s": t_build, "query_ms": t_q * 1e3}


def serve_load(dl, torch, idx, Qpool, reqs, rate, form, workspace, slots, max_batch):
    """Serve the request stream through a detlsh server.  rate = None submits
    every request at once (closed-loop backlog: saturation); otherwise Poisson
    arrivals at `rate` requests/s.  Latency of a request = completion of its
    last result minus its scheduled arrival (submitter lag included)."""
    import queue
    import threading
    srv = dl.Server(idx, workspace_bytes=workspace, slots=slots, max_batch=max_batch)
    nreq = len(reqs["nq"])
    prec = dl.BF16_RERANK if form == "bf16" else dl.FP32
    tickets = queue.Queue()
    results = [None] * nreq

    def waiter():
        for _ in range(nreq):
            i, t, t_arr = tickets.get()
            ids, d, info = srv.wait(t)
            results[i] = (t_arr, info, ids)

    th = threading.Thread(target=waiter)
    th.start()
    torch.cuda.synchronize()
    t0 = time.monotonic() + 0.01
    arrivals = t0 + (np.cumsum(reqs["gaps"]) / rate if rate else np.zeros(nreq))
    for i in range(nreq):
        if rate:
            dt = arrivals[i] - time.monotonic()
            if dt > 0:
                time.sleep(dt)
        q0, nq = int(reqs["q0"][i]), int(reqs["nq"][i])
        t = srv.submit(Qpool[q0:q0 + nq], int(reqs["k"][i]), float(reqs["c"][i]), 0.1, precision=prec, sync=False)
        tickets.put((i, t, float(arrivals[i]) if rate else time.monotonic()))
    th.join()
    srv.close()
    lat = np.array([r[1]["t_end"] - r[0] for r in results])
    t_first = min(r[0] for r in results)
    t_last = max(r[1]["t_end"] for r in results)
    nq_tot = int(reqs["nq"].sum())
    return {"offered_req_s": rate, "requests": nreq, "queries": nq_tot,
            "qps": nq_tot / (t_last - t_first), "req_s": nreq / (t_last - t_first),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_batch_queries": float(np.mean([r[1]["max_batch_queries"] for r in results])),
            "mean_batch_requests": float(np.mean([r[1]["max_batch_requests"] for r in results]))}, results


def serve_bench(dl, torch, nreq, loads=(0.5, 0.8, 1.1), slots=3, max_batch=512, pool=8192, log_prefix="[serve]"):
    """Serving form on the resident 256-d mixture index (n = 1,000,000):
    saturation by a closed-loop backlog, then Poisson arrivals at the given
    fractions of it, for plain FP32 and BF16 + rerank."""
    import synth
    cfg = synth.config("C5")
    dev = torch.device("cuda:0")
    log(f"{log_prefix} generating the 256-d mixture: n={cfg.n}, query pool {pool}")
    X = torch.from_numpy(synth.make_data(cfg)).to(dev)
    Qpool = torch.from_numpy(synth.make_queries(cfg, nq=pool)).to(dev)
    A = synth.projection_matrix(cfg.L, cfg.K, cfg.d, cfg.index_seed)
    sample = synth.sample_ids(cfg.n, cfg.n_s, cfg.index_seed)
    tb = time.perf_counter()
    idx = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
    build_s = time.perf_counter() - tb
    reqs = synth.request_stream(nreq, pool, cfg.arrival_seed)
    log(f"{log_prefix} ground truth of the query pool")
    kth = ground_truth_kth(X, Qpool, 10)
    workspace = slots * (max_batch * 5_200_000 + (64 << 20))
    out = {"workload": f"256-d Gaussian mixture n={cfg.n}, L=4 K=16 N_r=256, 1% sample, beta=0.1; "
                       f"{nreq} requests, nq log-uniform 1..256, k in {{1,10,100}}, c in {{1.5,2.0}}",
           "slots": slots, "max_batch": max_batch, "workspace_bytes": workspace, "build_s": build_s, "forms": {}}
    for form in ("fp32", "bf16"):
        warm = {key: v[:min(64, nreq)] for key, v in reqs.items()}
        serve_load(dl, torch, idx, Qpool, warm, None, form, workspace, slots, max_batch)
        sat, res = serve_load(dl, torch, idx, Qpool, reqs, None, form, workspace, slots, max_batch)
        # recall@10 of the served results of every request with k >= 10 (first 10 ids)
        hits = tot = 0
        for i, (_, _, ids) in enumerate(res):
            if int(reqs["k"][i]) < 10:
                continue
            q0, nq = int(reqs["q0"][i]), int(reqs["nq"][i])
            q = Qpool[q0:q0 + nq]
            d = ((X[ids[:, :10]].double() - q[:, None, :].double()) ** 2).sum(-1).sqrt()
            hits += int((d <= kth[q0:q0 + nq, None] * (1 + 1e-12)).sum())
            tot += 10 * nq
        rec = hits / tot if tot else None
        log(f"{log_prefix} {form}: saturation {sat['qps']:.0f} q/s ({sat['req_s']:.0f} req/s), recall@10 {rec}")
        f = {"saturation": sat, "recall_at_10": rec, "loads": []}
        for frac in loads:
            r, _ = serve_load(dl, torch, idx, Qpool, reqs, frac * sat["req_s"], form, workspace, slots, max_batch)
            r["load_frac"] = frac
            log(f"{log_prefix} {form} at {frac}x: {r['qps']:.0f} q/s, p50 {r['p50_ms']:.2f} ms, "
                f"p99 {r['p99_ms']:.2f} ms, mean batch {r['mean_batch_queries']:.0f} queries")
            f["loads"].append(r)
        out["forms"][form] = f
    idx.free()
    del X, Qpool
    torch.cuda.empty_cache()
    return out


def beta_grid_run(run, beta0):
    """QPS at recall >= 0.9 by the beta grid: if beta0 misses 0.9, raise beta
    over {0.15, 0.2, 0.3, 0.5}; if it clears 0.9, also try the lower values
    {0.05, 0.02, 0.01}.  run(beta) -> (qps, recall).  Returns every point tried
    and the smallest beta that meets 0.9."""
    tried = []
    qps, rec = run(beta0)
    tried.append({"beta": beta0, "qps": qps, "recall": rec})
    best = tried[-1] if rec >= 0.9 else None
    if rec >= 0.9:
        for b in (0.05, 0.02, 0.01):
            if b >= beta0:
                continue
            qps, rec = run(b)
            tried.append({"beta": b, "qps": qps, "recall": rec})
            if rec < 0.9:
                break
            best = tried[-1]
    else:
        for b in (0.15, 0.2, 0.3, 0.5):
            if b <= beta0:
                continue
            qps, rec = run(b)
            tried.append({"beta": b, "qps": qps, "recall": rec})
            if rec >= 0.9:
                best = tried[-1]
                break
    return {"tried": tried, "at_recall_0.9": best}


def precision_bench(dl, torch, name, steps, warmup, ks):
    """A precision-form workload (d = 960 Beta-copula set, or the n = 10^7
    normalised mixture): the index is built once (timed), then for each k and
    form the query set is answered `steps` times per beta of the grid, with
    recall@k against exact ground truth."""
    import synth
    cfg = synth.config(name)
    dev = torch.device("cuda:0")
    log(f"[{name}] generating on the GPU: n={cfg.n} d={cfg.d} nq={cfg.nq}")
    X = synth.make_data(cfg, device=dev)
    Q = synth.make_queries(cfg, device=dev)
    A = synth.projection_matrix(cfg.L, cfg.K, cfg.d, cfg.index_seed)
    sample = synth.sample_ids(cfg.n, cfg.n_s, cfg.index_seed)
    torch.cuda.synchronize()
    idx = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
    idx.free()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    idx = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
    build_s = time.perf_counter() - tb
    out = {"workload": name, "n": cfg.n, "d": cfg.d, "nq": cfg.nq, "beta0": cfg.beta, "L": cfg.L, "K": cfg.K,
           "N_r": cfg.N_r, "build_s": build_s, "build_mpts_s": cfg.n / build_s / 1e6,
           "build_note": "build includes a BF16 copy of X", "results": []}
    chunk = max(1, int(2e9 // (cfg.n * 4)))
    for k in ks:
        log(f"[{name}] ground truth k={k}")
        kth = ground_truth_kth(X, Q, k, chunk=chunk)
        for form in ("fp32", "bf16"):
            prec = dl.BF16_RERANK if form == "bf16" else dl.FP32

            def run(beta):
                for _ in range(warmup):
                    idx.query(Q, k, cfg.c, beta, precision=prec)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    ids, _ = idx.query(Q, k, cfg.c, beta, precision=prec)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / steps
                rec = recall_at_k(X, Q, ids, k, kth)
                log(f"[{name}] k={k} {form} beta={beta}: {cfg.nq / dt:.0f} q/s, recall@{k} {rec:.4f}")
                return cfg.nq / dt, rec

            r = beta_grid_run(run, cfg.beta)
            r.update({"k": k, "form": form})
            best = r["at_recall_0.9"]
            if best is not None:
                dl.profile_enable(True, reset=True)
                idx.query(Q, k, cfg.c, best["beta"], precision=prec)
                torch.cuda.synchronize()
                dl.profile_enable(False, reset=False)
                r["kernels_at_best"] = {name: {"launches": v["launches"], "total_ms": v["ms"]}
                                        for name, v in dl.profile_read().items() if v["launches"]}
                log(f"[{name}] k={k} {form} kernels at beta={best['beta']}: " +
                    ", ".join(f"{kn} {kv['total_ms']:.1f} ms" for kn, kv in r["kernels_at_best"].items()))
            out["results"].append(r)
    idx.free()
    del X, Q
    torch.cuda.empty_cache()
    return out


def next_rows_bench(dl, torch, steps, warmup):
    """The rows beyond the c^2-k-ANN path on the SIFT-shaped set: DET-ONLY
    (one PAA space) against DET-LSH, the (r, c)-ANN query (Alg. 6) at the median
    nearest-neighbour distance, and save / load of the index."""
    import tempfile

    import synth
    cfg = synth.config("C2")
    dev = torch.device("cuda:0")
    log("[next] generating C2")
    X_host = synth.make_data(cfg)
    Q_host = synth.make_queries(cfg)
    X = torch.from_numpy(X_host).to(dev)
    Q = torch.from_numpy(Q_host).to(dev)
    A = synth.projection_matrix(cfg.L, cfg.K, cfg.d, cfg.index_seed)
    sample = synth.sample_ids(cfg.n, cfg.n_s, cfg.index_seed)
    kth = ground_truth_kth(X, Q, 10)
    nn = ground_truth_kth(X, Q, 1)
    out = {"workload": "SIFT-shaped n=1,000,000 d=128, 10,000 queries"}

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    for name, kw in (("det_lsh", dict(L=cfg.L, A=A)), ("det_only", dict(L=1, projection="paa"))):
        tb, ix = timed(lambda: dl.build_index(X, kw["L"], cfg.K, cfg.N_r, cfg.sample_frac, sample_ids=sample,
                                              **{k: v for k, v in kw.items() if k != "L"}))
        tq, (ids, _) = timed(lambda: ix.query(Q, 10, cfg.c, cfg.beta))
        rec = recall_at_k(X, Q, ids, 10, kth)
        out[name] = {"L": kw["L"], "build_ms": tb * 1e3, "build_mpts_s": cfg.n / tb / 1e6, "qps": cfg.nq / tq,
                     "recall_at_10": rec}
        log(f"[next] {name}: build {tb * 1e3:.1f} ms, {cfg.nq / tq:.0f} q/s, recall@10 {rec:.4f}")
        if name == "det_lsh":
            idx = ix
        else:
            ix.free()
    fine = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, max_leaf=16)
    tq, (ids, _) = timed(lambda: fine.query(Q, 10, cfg.c, cfg.beta, granularity="leaf"))
    out["leaf_max_leaf16_beta0.1"] = {"qps": cfg.nq / tq, "recall_at_10": recall_at_k(X, Q, ids, 10, kth)}
    log(f"[next] leaf granularity, max_leaf 16: {cfg.nq / tq:.0f} q/s recall "
        f"{out['leaf_max_leaf16_beta0.1']['recall_at_10']:.4f}")
    fine.free()
    for gran in ("leaf",):
        for beta in (cfg.beta, 0.05):
            tq, (ids, _) = timed(lambda: idx.query(Q, 10, cfg.c, beta, granularity=gran))
            rec = recall_at_k(X, Q, ids, 10, kth)
            tq0, (ids0, _) = timed(lambda: idx.query(Q, 10, cfg.c, beta))
            rec0 = recall_at_k(X, Q, ids0, 10, kth)
            out[f"{gran}_beta{beta}"] = {"qps": cfg.nq / tq, "recall_at_10": rec, "point_qps": cfg.nq / tq0,
                                         "point_recall_at_10": rec0}
            log(f"[next] {gran} granularity beta={beta}: {cfg.nq / tq:.0f} q/s recall {rec:.4f} "
                f"(point: {cfg.nq / tq0:.0f} q/s recall {rec0:.4f})")
    r = float(nn.median())
    for c in (1.5, 2.0):
        tq, (ids, dists) = timed(lambda: idx.query_rc(Q, r, c, cfg.beta))
        got = ids >= 0
        ok = got & (dists.double() <= c * r * (1 + 1e-12))
        has = nn <= r
        out[f"rc_c{c}"] = {"r": r, "qps": cfg.nq / tq, "answered": float(got.double().mean()),
                           "within_cr": float(ok.double().mean()),
                           "within_cr_given_point_within_r": float((ok & has).double().sum() / has.double().sum())}
        log(f"[next] (r,c)-ANN c={c} r={r:.2f}: {cfg.nq / tq:.0f} q/s, answered {float(got.double().mean()):.3f}")
    # insertion into the built index: batches of SIFT-shaped rows from their own seed
    ins = {}
    for m in (10_000, 100_000):
        Xn = torch.from_numpy(synth.sift_like(m, cfg.d, 7000 + m)).to(dev)
        ixi = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ixi.insert(Xn)
        torch.cuda.synchronize()
        ti = time.perf_counter() - t0
        ins[str(m)] = {"seconds": ti, "points_per_s": m / ti, "n_after": ixi.info["n"]}
        log(f"[next] insert {m} into {cfg.n}: {ti * 1e3:.1f} ms, {m / ti / 1e6:.2f} M points/s")
        ixi.free()
    out["insert"] = ins
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "c2.detlsh")
        t0 = time.perf_counter()
        idx.save(path)
        ts = time.perf_counter() - t0
        size = os.path.getsize(path)
        t0 = time.perf_counter()
        back = dl.load_index(path)
        tl = time.perf_counter() - t0
        same = bool(torch.equal(back.query(Q[:256], 10, cfg.c, cfg.beta)[0], idx.query(Q[:256], 10, cfg.c,
                                                                                      cfg.beta)[0]))
        back.free()
    out["save_load"] = {"bytes": size, "save_s": ts, "load_s": tl, "save_gb_s": size / ts / 1e9,
                        "load_gb_s": size / tl / 1e9, "identical_answers": same}
    log(f"[next] save {size / 1e6:.0f} MB in {ts:.2f} s, load in {tl:.2f} s, identical {same}")
    idx.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--cpu-queries", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-bf16", action="store_true", help="skip timing the BF16+rerank form")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-form block")
    ap.add_argument("--serve-requests", type=int, default=1500)
    ap.add_argument("--serve-only", action="store_true", help="print only the serving-form block")
    ap.add_argument("--beta-sweep", action="store_true",
                    help="also run the beta grid for QPS at recall@10 >= 0.9 (query only, both forms)")
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "next"], default=None,
                    help="print only the named workload's beta grid for both forms (c2: SIFT-shaped, k = 10 "
                         "and 50; c3: d=960 copula; c4: n=10^7 mixture, k = 10 and 100; next: the extra rows)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the index and query batch fit one MI355X; see DESIGN.md for sharding).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2406_10938_amd as dl
    import synth
    torch.backends.cuda.matmul.allow_tf32 = False
    if args.serve_only:
        print(json.dumps(serve_bench(dl, torch, args.serve_requests)), flush=True)
        return
    if args.workload == "next":
        print(json.dumps(next_rows_bench(dl, torch, args.steps, args.warmup)), flush=True)
        return
    if args.workload:
        name = args.workload.upper()
        ks = {"C2": (10, 50), "C3": (10,)}.get(name, (10, 100))
        print(json.dumps(precision_bench(dl, torch, name, args.steps, args.warmup, ks)), flush=True)
        return

    cfg = synth.config("C2")
    nq = args.nq or cfg.nq
    k = args.k
    beta = cfg.beta if args.beta is None else args.beta
    log(f"[bench] generating C2: n={cfg.n} d={cfg.d} nq={nq}")
    X_host = synth.make_data(cfg)
    Q_host = synth.make_queries(cfg, nq=nq)
    A = synth.projection_matrix(cfg.L, cfg.K, cfg.d, cfg.index_seed)
    sample = synth.sample_ids(cfg.n, cfg.n_s, cfg.index_seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    X = torch.from_numpy(X_host).to(dev)
    Q = torch.from_numpy(Q_host).to(dev)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
        del src, dst

    # both forms build the BF16 copy of X: the FP32 form screens with BF16
    # products against a bound widened by their rounding (exact FP32 results)
    def step(bf16=False):
        idx = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
        ids, dists = idx.query(Q, k, cfg.c, beta, precision=dl.BF16_RERANK if bf16 else dl.FP32)
        return idx, ids, dists

    def timed(bf16, steps):
        """`steps` whole steps between two events on the launch stream."""
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        bsum = 0.0
        last = None
        for _ in range(steps):
            tb = time.perf_counter()
            ix = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
            bsum += time.perf_counter() - tb
            last = ix.query(Q, k, cfg.c, beta, precision=dl.BF16_RERANK if bf16 else dl.FP32)
            ix.free()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), bsum, last

    log(f"[bench] warmup x{args.warmup}")
    idx = ids = dists = None
    for _ in range(args.warmup):
        if idx is not None:
            idx.free()
        idx, ids, dists = step()
    torch.cuda.synchronize()
    recall = None
    if not args.no_recall:
        log("[bench] ground truth for recall@k")
        if ids is None:
            idx, ids, dists = step()
        kth = ground_truth_kth(X, Q, k)
        recall = recall_at_k(X, Q, ids, k, kth)
        log(f"[bench] recall@{k} = {recall:.4f}")
    if idx is not None:
        idx.free()

    dl.profile_enable(True, reset=True)
    log(f"[bench] timed x{args.steps}")
    t0 = time.perf_counter()
    ms_total, build_s, _ = timed(False, args.steps)
    wall = time.perf_counter() - t0
    dl.profile_enable(False, reset=False)
    prof = dl.profile_read()
    ms_per_step = ms_total / args.steps
    value = nq * args.steps / (ms_total / 1e3)
    build_ms = build_s * 1e3 / args.steps
    query_ms = ms_per_step - build_ms

    # roofline of the dominant kernel (largest total time in the timed region)
    n, LK, L, K, d = cfg.n, cfg.L * cfg.K, cfg.L, cfg.K, cfg.d
    N_S = k + math.ceil(beta * n)
    kernels = {}
    for name, v in prof.items():
        if v["launches"]:
            kernels[name] = {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"], "total_ms": v["ms"]}
    dom = max(kernels, key=lambda s: kernels[s]["total_ms"])
    avg_s = kernels[dom]["avg_ms"] / 1e3
    launches_per_step = kernels[dom]["launches"] / args.steps
    if dom == "range_filter":
        # VALU lane-ops per (query, point): 3 per (tree, dim) + 1 per tree
        ops = (3 * LK + L) * n * (nq / launches_per_step)
        roof = {"bound": "alu", "achieved": ops / avg_s / 1e12, "peak": VALU_PEAK_TOPS, "unit": "Tops/s"}
    elif dom == "verify_topk":
        byts = N_S * d * 4 * (nq / launches_per_step)
        roof = {"bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif dom == "dense_verify":
        fl = 2.0 * n * d * (nq / launches_per_step)
        roof = {"bound": "mfma", "achieved": fl / avg_s / 1e12, "peak": FP32_MFMA_PEAK, "unit": "TFLOP/s"}
    elif dom == "project_encode":
        fl = 2.0 * n * LK * d
        roof = {"bound": "mfma", "achieved": fl / avg_s / 1e12, "peak": FP32_MFMA_PEAK, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = (roof["achieved"] / roof["peak"]) if roof["achieved"] else None
    roof["traffic"] = counted_traffic(dom)
    roof["kernel"] = dom

    bf = None
    if not args.no_bf16:
        log(f"[bench] BF16+rerank form: warmup x{args.warmup}, timed x{args.steps}")
        for _ in range(args.warmup):
            ixb, ids_b, _ = step(True)
            ixb.free()
        ms_b, bs_b, (ids_b, _) = timed(True, args.steps)
        rec_b = recall_at_k(X, Q, ids_b, k, kth) if recall is not None else None
        bf = {"value": nq * args.steps / (ms_b / 1e3), "unit": "queries/s", "ms_per_step": ms_b / args.steps,
              "build_ms": bs_b * 1e3 / args.steps, "recall_at_k": rec_b, "rerank_mult": 4,
              "dtype": "bf16 products, fp32 accumulate and rerank"}
        log(f"[bench] BF16+rerank: {bf['value']:.0f} q/s, recall {rec_b}")

    sweep = None
    if args.beta_sweep and recall is not None:
        ixs = dl.build_index(X, cfg.L, cfg.K, cfg.N_r, cfg.sample_frac, A=A, sample_ids=sample, keep_bf16=True)
        sweep = {}
        for form in ("fp32", "bf16"):
            prec = dl.BF16_RERANK if form == "bf16" else dl.FP32

            def run(b):
                ixs.query(Q, k, cfg.c, b, precision=prec)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ids_s, _ = ixs.query(Q, k, cfg.c, b, precision=prec)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                rec = recall_at_k(X, Q, ids_s, k, kth)
                log(f"[bench] sweep {form} beta={b}: {nq / dt:.0f} q/s, recall {rec:.4f}")
                return nq / dt, rec

            sweep[form] = beta_grid_run(run, beta)
        ixs.free()

    serving = None
    if not args.no_serve:
        del X, Q
        torch.cuda.empty_cache()
        serving = serve_bench(dl, torch, args.serve_requests)

    cpu = None
    if not args.no_cpu:
        log(f"[bench] oracle on host cores ({args.cpu_queries} queries)")
        cpu = cpu_baseline(X_host, Q_host, A, sample, cfg, k, beta, nq, args.cpu_queries)

    out = {
        "metric": "QPS @ recall@10>=0.9 (plain FP32 vs BF16+rerank); build Mpts/s; p50/p99 latency",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "SIFT-shaped n=1,000,000 d=128, 10,000 queries, k=10 c=1.5 beta=0.1, "
                               "L=4 K=16 N_r=256, 1% sample; step = build + query batch",
                   "n": n, "d": d, "nq": nq, "k": k, "beta": beta, "L": L, "K": K, "N_r": cfg.N_r,
                   "precision": "fp32",
                   "verification": "FP32 direct distances rank the members of S that survive a BF16-product "
                                   "screen whose bound is widened by the BF16 rounding (results identical to "
                                   "an all-FP32 pass)"},
        "recall_at_k": recall,
        "query_qps": nq / (query_ms / 1e3) if query_ms > 0 else None,
        "build_mpts_s": n / (build_ms / 1e3) / 1e6,
        "build_ms": build_ms,
        "query_ms": query_ms,
        "wall_s": wall,
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
        "bf16_rerank": bf,
        "serving": serving,
        "beta_sweep": sweep,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
