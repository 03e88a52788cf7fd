"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the indexing method itself: it only draws
data sets, query sets and the random quantities the method consumes (the
Gaussian projection matrix of Eq. 1 and the breakpoint sample of Sec. 4.1),
so that both the CPU oracle and the GPU library can be fed the same draws.

Workload shapes (the paper's public data sets are not available; these stand
in for their shapes):

  C1  10,000 x 128   mixture of 32 isotropic Gaussians, centres ~ N(0, 10^2 I), sigma 1
  C2  1,000,000 x 128 SIFT-shaped: round(min(Gamma(0.5, 40), 255)), then 20% zero mask
  C3  1,000,000 x 960 Beta(2,5) marginals, Gaussian copula over blocks of 32 dims, rho 0.5
  C4  10,000,000 x 96 1,024-component mixture, centres ~ N(0, I), noise 0.3, unit-normalised
  C5  1,000,000 x 256 256-component mixture, centres ~ N(0, 5^2 I), sigma 1

Seeds: data = 1000 + cfg, queries = 2000 + cfg, index draws = 3000 + cfg,
arrivals = 4000 + cfg.  All host generation uses NumPy's PCG64 in float64 and
stores float32.  ``device="cuda"`` generates the same distributions with
torch's GPU generator (a different random stream) for the two largest shapes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Config", "CONFIGS", "config", "projection_matrix", "sample_ids",
    "gaussian_mixture", "sift_like", "beta_copula", "normalized_mixture",
    "make_data", "make_queries", "beta25_ppf",
]

_CHUNK = 1 << 18  # rows generated per chunk on the host


@dataclass(frozen=True)
class Config:
    name: str
    cfg: int
    n: int
    d: int
    nq: int
    ks: tuple
    beta: float
    sample_frac: float
    L: int = 4
    K: int = 16
    N_r: int = 256
    c: float = 1.5
    extra: dict = field(default_factory=dict)

    @property
    def data_seed(self):
        return 1000 + self.cfg

    @property
    def query_seed(self):
        return 2000 + self.cfg

    @property
    def index_seed(self):
        return 3000 + self.cfg

    @property
    def arrival_seed(self):
        return 4000 + self.cfg

    @property
    def n_s(self):
        return int(math.floor(self.sample_frac * self.n))


CONFIGS = {
    "C1": Config("C1", 1, 10_000, 128, 100, (10,), 0.1, 0.10),
    "C2": Config("C2", 2, 1_000_000, 128, 10_000, (10, 50), 0.1, 0.01),
    "C3": Config("C3", 3, 1_000_000, 960, 1_000, (10,), 0.1, 0.01),
    "C4": Config("C4", 4, 10_000_000, 96, 10_000, (10, 100), 0.05, 0.01),
    "C5": Config("C5", 5, 1_000_000, 256, 0, (1, 10, 100), 0.1, 0.01),
}


def config(name: str, **overrides) -> Config:
    base = CONFIGS[name]
    if not overrides:
        return base
    kw = dict(base.__dict__)
    kw.update(overrides)
    return Config(**kw)


# --------------------------------------------------------------------------
# random quantities the method draws
# --------------------------------------------------------------------------

def projection_matrix(L: int, K: int, d: int, seed: int) -> np.ndarray:
    """(L*K) x d matrix, entries i.i.d. N(0,1) drawn in float64 and rounded to
    float32 (Eq. 1).  Row i*K + j is the hash h_ij."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((L * K, d)).astype(np.float32)


def sample_ids(n: int, n_s: int, seed: int) -> np.ndarray:
    """n_s distinct point ids drawn uniformly without replacement, ascending."""
    if not (0 < n_s <= n):
        raise ValueError("need 0 < n_s <= n")
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    ids = rng.choice(n, size=n_s, replace=False)
    ids.sort()
    return ids.astype(np.int64)


# --------------------------------------------------------------------------
# data generators (host, numpy)
# --------------------------------------------------------------------------

def _mixture_centres(rng, n_comp, d, scale):
    return rng.standard_normal((n_comp, d)) * scale


def gaussian_mixture(n, d, n_comp, centre_scale, sigma, data_seed, rows_seed=None):
    """Points centre_c + sigma * N(0, I) with c uniform over n_comp centres.
    Centres come from ``data_seed``; rows from ``rows_seed`` (default data_seed)."""
    crng = np.random.Generator(np.random.PCG64(data_seed))
    centres = _mixture_centres(crng, n_comp, d, centre_scale)
    rrng = crng if rows_seed is None else np.random.Generator(np.random.PCG64(rows_seed))
    out = np.empty((n, d), np.float32)
    for s in range(0, n, _CHUNK):
        m = min(_CHUNK, n - s)
        lab = rrng.integers(0, n_comp, size=m)
        out[s:s + m] = centres[lab] + sigma * rrng.standard_normal((m, d))
    return out


def sift_like(n, d, seed, zero_prob=0.2):
    """Non-negative integers in [0, 255]: round(min(Gamma(0.5, 40), 255)) per
    coordinate, then an independent zero mask with probability ``zero_prob``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, d), np.float32)
    for s in range(0, n, _CHUNK):
        m = min(_CHUNK, n - s)
        v = np.rint(np.minimum(rng.gamma(0.5, 40.0, size=(m, d)), 255.0))
        v[rng.random((m, d)) < zero_prob] = 0.0
        out[s:s + m] = v
    return out


def beta25_ppf(u, xp=np):
    """Inverse CDF of Beta(2, 5).  The CDF has the closed form
    F(x) = 1 - (1 - x)^5 (1 + 5x); it is inverted by bisection (monotone on
    [0, 1]), 52 halvings, i.e. to float64 resolution."""
    lo = xp.zeros_like(u)
    hi = xp.ones_like(u)
    for _ in range(52):
        mid = 0.5 * (lo + hi)
        f = 1.0 - (1.0 - mid) ** 5 * (1.0 + 5.0 * mid)
        below = f < u
        lo = xp.where(below, mid, lo)
        hi = xp.where(below, hi, mid)
    return 0.5 * (lo + hi)


def beta_copula(n, d, seed, block=32, rho=0.5):
    """Beta(2,5) marginals joined by a Gaussian copula: within each block of
    ``block`` dimensions z = sqrt(rho) g_b + sqrt(1-rho) e, x = F^-1(Phi(z))."""
    from scipy.special import ndtr
    if d % block:
        raise ValueError("d must be a multiple of block")
    nb = d // block
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, d), np.float32)
    a, b = math.sqrt(rho), math.sqrt(1.0 - rho)
    for s in range(0, n, _CHUNK // 4):
        m = min(_CHUNK // 4, n - s)
        g = rng.standard_normal((m, nb))
        z = a * np.repeat(g, block, axis=1) + b * rng.standard_normal((m, d))
        out[s:s + m] = beta25_ppf(ndtr(z))
    return out


def normalized_mixture(n, d, n_comp, scale, data_seed, rows_seed=None):
    """x = mu_c + scale * N(0, I), mu ~ N(0, I), then x / ||x||."""
    crng = np.random.Generator(np.random.PCG64(data_seed))
    centres = _mixture_centres(crng, n_comp, d, 1.0)
    rrng = crng if rows_seed is None else np.random.Generator(np.random.PCG64(rows_seed))
    out = np.empty((n, d), np.float32)
    for s in range(0, n, _CHUNK):
        m = min(_CHUNK, n - s)
        lab = rrng.integers(0, n_comp, size=m)
        x = centres[lab] + scale * rrng.standard_normal((m, d))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[s:s + m] = x
    return out


# --------------------------------------------------------------------------
# torch/GPU variants of the two largest shapes (same law, torch's stream)
# --------------------------------------------------------------------------

def _torch_beta_copula(n, d, seed, device, block=32, rho=0.5):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    nb = d // block
    out = torch.empty((n, d), dtype=torch.float32, device=device)
    a, b = math.sqrt(rho), math.sqrt(1.0 - rho)
    step = 1 << 16
    for s in range(0, n, step):
        m = min(step, n - s)
        gb = torch.randn((m, nb), generator=g, device=device, dtype=torch.float64)
        z = a * gb.repeat_interleave(block, dim=1) + b * torch.randn(
            (m, d), generator=g, device=device, dtype=torch.float64)
        out[s:s + m] = beta25_ppf(torch.special.ndtr(z), xp=torch).float()
    return out


def _torch_normalized_mixture(n, d, n_comp, scale, data_seed, device, rows_seed=None):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(data_seed)
    centres = torch.randn((n_comp, d), generator=g, device=device, dtype=torch.float64)
    if rows_seed is not None:
        g = torch.Generator(device=device)
        g.manual_seed(rows_seed)
    out = torch.empty((n, d), dtype=torch.float32, device=device)
    step = 1 << 20
    for s in range(0, n, step):
        m = min(step, n - s)
        lab = torch.randint(0, n_comp, (m,), generator=g, device=device)
        x = centres[lab] + scale * torch.randn((m, d), generator=g, device=device,
                                               dtype=torch.float64)
        out[s:s + m] = (x / x.norm(dim=1, keepdim=True)).float()
    return out


# --------------------------------------------------------------------------
# config-level entry points
# --------------------------------------------------------------------------

def make_data(cfg: Config, n=None, device=None):
    """Data set of ``cfg`` (first ``n`` rows if given).  Returns a float32
    numpy array, or a torch tensor when ``device`` is given (C3/C4 only use
    torch's generator there; the others are generated on the host and moved)."""
    n = cfg.n if n is None else n
    if device is not None and cfg.name in ("C3", "C4"):
        if cfg.name == "C3":
            return _torch_beta_copula(n, cfg.d, cfg.data_seed, device)
        return _torch_normalized_mixture(n, cfg.d, 1024, 0.3, cfg.data_seed, device)
    x = _host_rows(cfg, n, cfg.data_seed, None)
    if device is not None:
        import torch
        return torch.from_numpy(x).to(device)
    return x


def make_queries(cfg: Config, nq=None, device=None):
    """Query set drawn from the same generator as the data (same mixture
    centres where there is a mixture) with the query seed."""
    nq = cfg.nq if nq is None else nq
    if device is not None and cfg.name in ("C3", "C4"):
        if cfg.name == "C3":
            return _torch_beta_copula(nq, cfg.d, cfg.query_seed, device)
        return _torch_normalized_mixture(nq, cfg.d, 1024, 0.3, cfg.data_seed, device,
                                         rows_seed=cfg.query_seed)
    q = _host_rows(cfg, nq, cfg.data_seed, cfg.query_seed)
    if device is not None:
        import torch
        return torch.from_numpy(q).to(device)
    return q


def _host_rows(cfg, n, data_seed, rows_seed):
    seed = data_seed if rows_seed is None else rows_seed
    if cfg.name == "C1":
        return gaussian_mixture(n, cfg.d, 32, 10.0, 1.0, data_seed, rows_seed)
    if cfg.name == "C2":
        return sift_like(n, cfg.d, seed)
    if cfg.name == "C3":
        return beta_copula(n, cfg.d, seed)
    if cfg.name == "C4":
        return normalized_mixture(n, cfg.d, 1024, 0.3, data_seed, rows_seed)
    if cfg.name == "C5":
        return gaussian_mixture(n, cfg.d, 256, 5.0, 1.0, data_seed, rows_seed)
    raise KeyError(cfg.name)


# --------------------------------------------------------------------------
# serving request stream
# --------------------------------------------------------------------------

def request_stream(nreq: int, pool: int, seed: int, max_nq: int = 256, ks=(1, 10, 100), cs=(1.5, 2.0)):
    """Seeded serving requests: nq = floor(exp(U(0, ln(max_nq+1)))) clamped to
    [1, max_nq] (log-uniform, mean about 46 for 256), k and c uniform over
    their sets, a start row q0 uniform in the query pool, and unit-rate
    exponential inter-arrival gaps (scale them by 1/rate for Poisson arrivals).
    Returns a dict of numpy arrays."""
    rng = np.random.default_rng(seed)
    nq = np.floor(np.exp(rng.uniform(0.0, np.log(max_nq + 1), nreq))).astype(np.int64)
    nq = np.clip(nq, 1, max_nq)
    k = rng.choice(np.asarray(ks, np.int64), nreq)
    c = rng.choice(np.asarray(cs, np.float64), nreq)
    q0 = rng.integers(0, pool - nq + 1)
    gaps = rng.exponential(1.0, nreq)
    return {"nq": nq, "k": k, "c": c, "q0": q0, "gaps": gaps}
