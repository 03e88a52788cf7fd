"""The range screen's FP16 test is conservative (CPU).

The screen keeps a (query, point) pair of tree i when the dot product
V_i = u.p of two FP16 vectors is negative.  The vectors are rebuilt here in
NumPy step by step as the kernels build them (per-tree power-of-two scale,
FP16 rounding with subnormals flushed, radii rounded up to FP16, the hi + lo
splits of the two norm terms, the 2^-12 relative and absolute slacks, the
negative last term), and V is summed in FP32 in two orders.  Every pair that
the plain filter keeps (its FP32 bound LB_i^2 <= thr, here with thr equal to
the pair's own bound) must get V < 0, and by the margin the construction
promises.  Queries beyond a cell's corner, on the line through its centre,
make the ball test tight; the other cases cover normal and duplicate-heavy
breakpoints (cells of width zero), very large and very small coordinate
scales, queries outside the breakpoint range, and thr = 0.  A naive
construction (no slacks, roundings to nearest) fails the margin.
"""
import numpy as np
import pytest

DELTA = 2.0 ** -12
ABS = 2.0 ** -12
SIGN = -(2.0 ** -14)
F16_MIN = 2.0 ** -14


def f16r(x):
    """FP16 rounding (to nearest even) as FP32, subnormal results flushed."""
    r = np.asarray(x, np.float32).astype(np.float16).astype(np.float32)
    return np.where(np.abs(r) < F16_MIN, np.float32(0), r)


def f16_up(x):
    """The smallest normal FP16 >= x (x >= 0), elementwise; 0 for x = 0."""
    x = np.asarray(x, np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        h = x.astype(np.float32).astype(np.float16)
    for _ in range(2):
        low = h.astype(np.float64) < x
        h = np.where(low, np.nextafter(h, np.float16(np.inf)), h)
    r = h.astype(np.float32)
    return np.where(x > 0, np.maximum(r, np.float32(F16_MIN)), np.float32(0))


def scale_of(E):
    """s = 2^k with s * max|interior breakpoint| in [4, 8)."""
    M = float(np.max(np.abs(E[:, [1, -2]])))
    if not (M > 0 and np.isfinite(M)):
        return np.float32(1)
    _, ex = np.frexp(M)
    return np.float32(np.ldexp(1.0, 3 - int(ex)))


def table(E, codes, planted=False):
    """Point vectors p = [c^, 1, 1, P_hi, P_lo, W^, 1] for codes (n, K)
    (planted: without the relative slack, W rounded to nearest)."""
    n, K = codes.shape
    s = scale_of(E)
    a, b = E[:, 1], E[:, -2]
    j = np.arange(K)
    lo = np.clip(E[j, codes], a, b).astype(np.float32) * s
    hi = np.clip(E[j, codes + 1], a, b).astype(np.float32) * s
    c = f16r(np.float32(0.5) * (lo + hi))   # the FP32 midpoint, as the kernel forms it
    w = np.maximum(hi.astype(np.float64) - c, c.astype(np.float64) - lo)
    cc = np.sum(c.astype(np.float64) ** 2, axis=1)
    if planted:
        W = f16r(np.sqrt(np.sum(w * w, axis=1)).astype(np.float32))
    else:
        W = f16_up(np.sqrt(np.sum(w * w, axis=1)) * (1.0 + 2.0 ** -40))
    dl = 0.0 if planted else DELTA
    P = ((1 - dl) * cc - (1 + dl) * W.astype(np.float64) ** 2).astype(np.float32)
    Ph = f16r(P)
    Pl = f16r(P - Ph)
    one = np.ones(n, np.float32)
    return np.concatenate([c, np.stack([one, one, Ph, Pl, W, one], axis=1)], axis=1)


def query_vecs(E, q, thr, planted=False):
    """Query vectors u = [-2 q^, U_hi, U_lo, 1, 1, -2 R^, -2^-14] (or pass-all).
    planted: a deliberate mistake (no slacks, R rounded to nearest and
    without the query's rounding distance) that the tests must catch."""
    nq, K = q.shape
    s = scale_of(E)
    a, b = E[:, 1], E[:, -2]
    qt = np.clip(q, a, b).astype(np.float32) * s
    qh = f16r(qt)
    qq = np.sum(qh.astype(np.float64) ** 2, axis=1)
    ee = np.sum((qt.astype(np.float64) - qh) ** 2, axis=1)
    tp = thr.astype(np.float64) * (1 + DELTA)
    if planted:
        R = f16r((float(s) * np.sqrt(tp)).astype(np.float32))
    else:
        R = f16_up((float(s) * np.sqrt(tp) + np.sqrt(ee)) * (1.0 + 2.0 ** -40))
    dl, ab, sg = (0.0, 0.0, 0.0) if planted else (DELTA, ABS, SIGN)
    U = ((1 - dl) * qq - (1 + dl) * R.astype(np.float64) ** 2 - ab).astype(np.float32)
    Uh = f16r(U)
    with np.errstate(invalid="ignore"):
        Ul = f16r(U - Uh)
    one = np.ones(nq, np.float32)
    u = np.concatenate([-2 * qh, np.stack([Uh, Ul, one, one, -2 * R, np.full(nq, sg, np.float32)], axis=1)],
                       axis=1)
    all_pass = ~(thr < np.inf) | (R >= 128)
    u[all_pass] = 0
    u[all_pass, K] = -1
    return u


def v_fp32(u, p, reverse=False):
    """u.p with exact FP16 products summed in FP32, entry by entry."""
    prod = u[:, None, :].astype(np.float32) * p[None, :, :].astype(np.float32)   # exact
    acc = np.zeros(prod.shape[:2], np.float32)
    idx = range(prod.shape[2] - 1, -1, -1) if reverse else range(prod.shape[2])
    for k in idx:
        acc = (acc + prod[:, :, k]).astype(np.float32)
    return acc


# Every pair the filter keeps has V <= -(d/2.01 - 2^-17) sum_k |u_k p_k|: the
# relative slack, less the FP32 sums' error (the absolute terms only add).
MARGIN = DELTA / 2.01 - 2.0 ** -17


def abs_sum(u, p):
    return np.sum(np.abs(u[:, None, :].astype(np.float64) * p[None, :, :]), axis=2)


def lb2_fp32(E, q, codes):
    """The plain filter's bound: d = q - med3(q, lo, hi), fma-accumulated in FP32."""
    K = codes.shape[1]
    j = np.arange(K)
    lo = E[j, codes].astype(np.float32)
    hi = E[j, codes + 1].astype(np.float32)
    acc = np.zeros((q.shape[0], codes.shape[0]), np.float32)
    for jj in range(K):
        med = np.clip(q[:, None, jj], lo[None, :, jj], hi[None, :, jj]).astype(np.float32)
        dd = (q[:, None, jj] - med).astype(np.float32)
        acc = (acc.astype(np.float64) + dd.astype(np.float64) ** 2).astype(np.float32)   # one rounding, as fma
    return acc


def breakpoints(kind, K, N_r, rng):
    vals = rng.standard_normal((K, 4000))
    if kind == "dups":
        vals = np.round(vals * 2) / 2        # few distinct values: many equal breakpoints
    elif kind == "huge":
        vals = vals * 3.0e4
    elif kind == "tiny":
        vals = vals * 2.0e-6
    elif kind == "offset":
        vals = vals * 0.01 + 50.0
    qs = np.quantile(vals, np.arange(1, N_r) / N_r, axis=1, method="lower").T
    E = np.empty((K, N_r + 1), np.float32)
    E[:, 0] = -np.inf
    E[:, 1:N_r] = qs
    E[:, N_r] = np.inf
    return E, vals


def corner_queries(E, codes, rng, m):
    """Queries beyond a corner of the cell of a point with interior codes,
    along the line from the cell's centre through that corner: the box's
    nearest point is the corner, which lies on the ball around the centre, so
    the screen's test is tight there (up to the FP16 roundings).  Returns the
    queries and the points they were built for."""
    K = codes.shape[1]
    N_r = E.shape[1] - 1
    j = np.arange(K)
    inner = np.where(np.all((codes > 0) & (codes < N_r - 1), axis=1))[0]
    tgt = rng.choice(inner, m)
    lo = E[j, codes[tgt]].astype(np.float64)
    hi = E[j, codes[tgt] + 1].astype(np.float64)
    c = 0.5 * (lo + hi)
    corner = np.where(rng.random((m, K)) < 0.5, lo, hi)
    lam = rng.uniform(0.05, 0.6, size=(m, 1))
    q = c + (1 + lam) * (corner - c)
    return np.clip(q, E[:, 1], E[:, -2]).astype(np.float32), tgt


@pytest.mark.parametrize("kind", ["normal", "dups", "huge", "tiny", "offset"])
def test_screen_keeps_every_filter_candidate(kind):
    rng = np.random.default_rng({"normal": 1, "dups": 2, "huge": 3, "tiny": 4, "offset": 5}[kind])
    K, N_r, n, nq = 16, 64, 600, 40
    E, vals = breakpoints(kind, K, N_r, rng)
    codes = rng.integers(0, N_r, size=(n, K))
    codes[:50] = 0            # the outer regions (one side open)
    codes[50:100] = N_r - 1
    spread = np.std(vals, axis=1)
    q = (vals[:, rng.integers(0, vals.shape[1], nq)].T + rng.standard_normal((nq, K)) * spread * 0.05)
    q[:5] *= 3.0              # outside the breakpoint range: clamped
    q = q.astype(np.float32)
    qc, tgt = corner_queries(E, codes, rng, nq)
    q = np.concatenate([q, qc])
    lb = lb2_fp32(E, q, codes)
    p = table(E, codes)
    checked = 0
    for qi in range(2 * nq):
        # thr at the bounds of several pairs (for a corner query, first its own
        # point): each of them passes with equality
        pairs = rng.choice(n, 12, replace=False)
        if qi >= nq:
            pairs[0] = tgt[qi - nq]
        for o in pairs:
            thr = np.array([lb[qi, o]], np.float32)
            keep = lb[qi] <= thr[0]
            u = query_vecs(E, q[qi:qi + 1], thr)
            S = abs_sum(u, p)[0]
            for rev in (False, True):
                V = v_fp32(u, p, reverse=rev)[0]
                assert np.all(np.signbit(V[keep]) & (V[keep] != 0)), (kind, qi, o, rev)
                assert np.all(V[keep] <= -MARGIN * S[keep]), (kind, qi, o, rev)
            checked += int(keep.sum())
    assert checked > 1000


def test_screen_zero_threshold_and_zero_width_cells():
    """thr = 0 keeps exactly the points whose cells hold the query; with cells of
    width zero (equal breakpoints) and the query on them the bound is 0 too."""
    K, N_r = 16, 16
    E = np.empty((K, N_r + 1), np.float32)
    E[:, 0], E[:, N_r] = -np.inf, np.inf
    E[:, 1:N_r] = np.sort(np.r_[np.zeros(7), np.arange(1, 9)].astype(np.float32))[None, :]   # B = 0 seven times
    rng = np.random.default_rng(7)
    codes = rng.integers(0, N_r, size=(500, K))
    codes[:100] = rng.integers(0, 8, size=(100, K))   # cells [-inf, 0], [0, 0] x 6, [0, 1]: all hold 0
    codes[100:150] = 7                                # [0, 1] holds 0.5
    codes[150:200] = N_r - 1                          # [8, inf] holds 100
    q = np.zeros((3, K), np.float32)
    q[1] = 0.5
    q[2] = 100.0
    lb = lb2_fp32(E, q, codes)
    p = table(E, codes)
    u = query_vecs(E, q, np.zeros(3, np.float32))
    V = v_fp32(u, p)
    keep = lb <= 0
    assert keep[0].sum() >= 100 and keep[1].sum() >= 50 and keep[2].sum() >= 50
    assert np.all(np.signbit(V[keep]) & (V[keep] != 0))


def test_screen_pass_all_for_infinite_or_huge_threshold():
    rng = np.random.default_rng(3)
    E, _ = breakpoints("normal", 16, 64, rng)
    codes = rng.integers(0, 64, size=(100, 16))
    p = table(E, codes)
    u = query_vecs(E, np.zeros((2, 16), np.float32), np.array([np.inf, 1e30], np.float32))
    assert np.all(v_fp32(u, p) == -1)


def test_fp16_helpers():
    assert f16r(np.float32(1.0 + 2 ** -12)) == 1.0                 # nearest even
    assert f16r(np.float32(3e-5)) == 0.0                           # below the smallest normal: flushed
    x = np.float64(1.0 + 2 ** -12)
    assert f16_up(x) == np.float32(1.0 + 2 ** -10) and f16_up(x) >= x
    assert f16_up(np.float64(1e-9)) == np.float32(2 ** -14)
    assert f16_up(np.float64(0.0)) == 0.0
    assert np.all(f16_up(np.linspace(0.01, 100, 1001)) >= np.linspace(0.01, 100, 1001))


def test_planted_radius_mistake_is_caught():
    """The naive construction (no slacks, no query rounding distance, R and W
    rounded to nearest) leaves pairs on their threshold without the margin
    the main test asserts: the corner cases detect it."""
    rng = np.random.default_rng(11)
    K, N_r, n, nq = 16, 64, 600, 40
    E, vals = breakpoints("normal", K, N_r, rng)
    codes = rng.integers(0, N_r, size=(n, K))
    q, tgt = corner_queries(E, codes, rng, nq)
    lb = lb2_fp32(E, q, codes)
    p = table(E, codes, planted=True)
    short = 0
    for qi in range(nq):
        o = tgt[qi]
        thr = np.array([lb[qi, o]], np.float32)
        u = query_vecs(E, q[qi:qi + 1], thr, planted=True)
        V = v_fp32(u, p)[0, o]
        short += int(V > -MARGIN * abs_sum(u, p)[0, o])
    assert short > nq // 2
