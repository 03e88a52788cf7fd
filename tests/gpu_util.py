"""Helpers shared by the GPU parity tests: seeded cases, the oracle side of
each comparison and the tolerance rules (projections: 1e-5 of sum_l |a_l o_l|;
candidate sets: exact except points whose FP64 bound is within 1e-5 relative
of the stop threshold; ids: exact except (k, k+1) distance near-ties;
distances: 1e-5 relative)."""
from __future__ import annotations

import math

import numpy as np

import synth
from oracle import detlsh_oracle as O

REL = 1e-5


def case(n=3000, d=64, L=4, K=16, N_r=64, frac=0.1, seed=0, kind="mixture", nq=20):
    rng = np.random.default_rng(seed)
    if kind == "integer":
        X = synth.sift_like(n, d, 100 + seed)
        Q = synth.sift_like(nq, d, 200 + seed)
    elif kind == "smallint":
        X = rng.integers(0, 4, (n, d)).astype(np.float32)
        Q = rng.integers(0, 4, (nq, d)).astype(np.float32)
    else:
        X = synth.gaussian_mixture(n, d, 16, 4.0, 1.0, 100 + seed)
        Q = synth.gaussian_mixture(nq, d, 16, 4.0, 1.0, 100 + seed, rows_seed=200 + seed)
    A = synth.projection_matrix(L, K, d, 300 + seed)
    sample = synth.sample_ids(n, max(N_r, int(math.floor(frac * n))), 400 + seed)
    return dict(X=X, Q=Q, A=A, sample=sample, L=L, K=K, N_r=N_r, frac=frac, n=n, d=d)


def proj_scale(X, A):
    """sum_l |a_el x_ol| for every (o, e): the scale of a dot product's rounding error."""
    return np.abs(np.asarray(X, np.float64)) @ np.abs(np.asarray(A, np.float64)).T


def oracle_encoding(c):
    P = O.project(c["X"], c["A"])
    B = O.breakpoints_by_sort(P[c["sample"]], c["N_r"])
    codes = O.encode(P, B)
    return P, B, codes


def code_mismatches(P, Pscale, B_ref, B_gpu, codes_ref, codes_gpu):
    """(number of mismatching codes, number of them that are NOT borderline).
    Borderline: the FP64 coordinate lies within tolerance of an interior
    breakpoint (by the projection rule, widened by the breakpoint difference)."""
    bad = np.argwhere(codes_ref != codes_gpu)
    hard = 0
    for o, e in bad:
        tol = REL * Pscale[o, e] + np.abs(B_ref[e] - B_gpu[e]).max()
        inner = B_ref[e, 1:-1]
        if np.min(np.abs(inner - P[o, e])) > tol:
            hard += 1
    return len(bad), hard


def oracle_query(X, q, qp, codes, B, L, K, k, beta):
    return O.query_magic(X, q, np.asarray(qp, np.float64), codes, np.asarray(B, np.float64), L, K, k, beta)


def borderline_points(qp, codes, B, L, K, thr):
    lb = O.lower_bounds(np.asarray(qp, np.float64), codes, np.asarray(B, np.float64), L, K)
    m2 = lb.min(axis=1)
    return set(np.flatnonzero(np.abs(m2 - thr) <= REL * max(thr, 1e-30)).tolist())


def compare_result(ref_ids, ref_d, X, q, got_ids, got_d, S_ref, k):
    """Ids must match except at distance near-ties; distances within 1e-5.
    Returns the number of positions whose id differs (all near-ties)."""
    got_ids = np.asarray(got_ids)
    got_d = np.asarray(got_d, np.float64)
    np.testing.assert_allclose(got_d, ref_d, rtol=REL, atol=1e-6)
    diff = np.flatnonzero(got_ids != ref_ids)
    if len(diff) == 0:
        return 0
    d_all = np.sqrt(O.sq_dists(X[S_ref], q))
    for j in diff:
        close = np.abs(d_all - ref_d[j]) <= REL * max(ref_d[j], 1e-30) + 1e-7
        assert close.sum() >= 2, f"id differs at rank {j} without a near-tie"
    return len(diff)
