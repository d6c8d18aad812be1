"""Seeded synthetic inputs shared by the oracle-side tests and the GPU side.

This module holds no arithmetic of the method itself: it only draws the
matrices that both sides receive (the data A, the Gaussian test matrices
Omega, the initial factors), from NumPy's PCG64 with fixed seeds.  It
imports nothing but NumPy, so the oracle tests can use it without touching
the HIP library.

Recipes (the paper's synthetic NMF experiment, Section 5.1 and its figure
caption, with the dense density delta = 1):
  * NMF data:   A = W H + N, W ~ U[0,1)^{m x r}, H ~ U[0,1)^{r x n},
                N = |sigma Z|, Z standard normal (sigma is a standard
                deviation; the absolute value keeps A >= 0).
  * Separable:  A = W [I_r  H'] P + noise Z, W ~ U[0,1)^{m x r}, the columns
                of H' are Dirichlet(1) draws scaled by s_j ~ U(0, 1], P a
                seeded column permutation; the planted (extreme) columns are
                where the identity columns land after P.
  * Sparse NMF data (the same figure's sparse case): entries of W (m x r)
                and H (r x n) are U[0,1) with probability delta and 0
                otherwise, N is standard normal with probability delta^2
                and 0 otherwise, A = W H + N (n = 0.75 m and delta = 1e-2
                in the paper), returned in compressed-row form.
  * Test matrices Omega: iid N(0, 1) (Section 2).
  * Initial factors: c * U[0,1) with c = sqrt(4 mean(A) / r), so that
    E[U V] = mean(A).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "WORKLOADS", "nmf_matrix", "separable_matrix", "separable_on_device", "gaussian",
           "init_factors", "make_inputs", "sparse_nmf_matrix"]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def nmf_matrix(m: int, n: int, r: int, sigma: float, seed: int, dtype=np.float64) -> np.ndarray:
    """A = W H + |sigma Z| with W, H uniform on [0, 1).  Built in float64 and
    rounded once to ``dtype``."""
    g = _rng(seed)
    W = g.random((m, r))
    H = g.random((r, n))
    A = W @ H
    if sigma:
        # draw the noise in row blocks to bound peak memory
        for i0 in range(0, m, 8192):
            blk = A[i0:i0 + 8192]
            blk += np.abs(sigma * g.standard_normal(blk.shape))
    return A.astype(dtype, copy=False)


def separable_matrix(m: int, n: int, r: int, noise: float, seed: int, dtype=np.float64):
    """Near-separable A = W [I_r H'] P + noise * Z.  Returns (A, planted) with
    ``planted`` the sorted 0-based column indices of the identity columns."""
    g = _rng(seed)
    W = g.random((m, r))
    Hp = g.dirichlet(np.ones(r), size=n - r).T          # r x (n - r), columns on the simplex
    s = 1.0 - g.random(n - r)                            # U(0, 1]
    Hp *= s[None, :]
    Hfull = np.concatenate([np.eye(r), Hp], axis=1)      # r x n
    perm = g.permutation(n)                              # column j of A is column perm[j] of W Hfull
    A = (W @ Hfull)[:, perm]
    if noise:
        for i0 in range(0, m, 4096):
            blk = A[i0:i0 + 4096]
            blk += noise * g.standard_normal(blk.shape)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    planted = np.sort(inv[:r])
    return A.astype(dtype, copy=False), planted


def separable_on_device(m: int, n: int, r: int, noise: float, seed: int, device):
    """The near-separable recipe of separable_matrix, drawn on a torch device
    with torch's seeded generator (for sizes whose host copy would be slow):
    A = W [I_r H'] P + noise * Z in FP32, H' columns Dirichlet(1) (normalised
    Exponential(1) draws) scaled by U(0, 1].  Returns (A, planted indices)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    W = torch.rand(m, r, device=device, generator=g)
    E = -torch.log1p(-torch.rand(r, n - r, device=device, dtype=torch.float64, generator=g))
    Hp = E / E.sum(dim=0, keepdim=True)
    Hp *= 1.0 - torch.rand(1, n - r, device=device, dtype=torch.float64, generator=g)
    H = torch.cat([torch.eye(r, device=device, dtype=torch.float64), Hp], dim=1).float()
    perm = torch.randperm(n, device=device, generator=g)
    A = (W @ H)[:, perm].contiguous()
    if noise:
        A += noise * torch.randn(m, n, device=device, generator=g)
    planted = torch.nonzero(perm < r).flatten().cpu().numpy()
    return A, np.sort(planted)


def sparse_nmf_matrix(m: int, n: int, r: int, delta: float, seed: int, dtype=np.float64):
    """The sparse synthetic recipe: (rowptr int64, colind int32, values, dense)
    of A = W H + N in compressed-row form (column indices ascending within
    each row), and the dense copy for the oracle side."""
    g = _rng(seed)
    W = np.where(g.random((m, r)) < delta, g.random((m, r)), 0.0)
    H = np.where(g.random((r, n)) < delta, g.random((r, n)), 0.0)
    N = np.where(g.random((m, n)) < delta * delta, g.standard_normal((m, n)), 0.0)
    A = (W @ H + N).astype(dtype)
    mask = A != 0
    rowptr = np.zeros(m + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(mask.sum(axis=1))
    rows, cols = np.nonzero(mask)            # row-major order, columns ascending
    return rowptr, cols.astype(np.int32), A[rows, cols], A


def gaussian(rows: int, cols: int, seed: int) -> np.ndarray:
    """iid N(0, 1) test matrix (Section 2), float64."""
    return _rng(seed).standard_normal((rows, cols))


def init_factors(mean_a: float, m: int, n: int, r: int, seed: int):
    """U1 (m x r), V1 (r x n) = c U[0,1) with c = sqrt(4 mean(A) / r)."""
    g = _rng(seed)
    c = math.sqrt(4.0 * float(mean_a) / r)
    return c * g.random((m, r)), c * g.random((r, n))


@dataclass(frozen=True)
class Workload:
    name: str
    index: int            # seed base: data 100*index, Omega 100*index+1, init 100*index+2
    m: int
    n: int
    r: int
    k: int
    q: int
    iters: int
    dtype: str            # storage / pass precision of A on the GPU
    sigma: float = 0.0    # |N(0, sigma)| additive noise for NMF data
    separable: bool = False
    sep_noise: float = 0.0
    extra: dict = field(default_factory=dict)


# Workload table.  The first entry is small enough for the oracle to run in
# about a second; the others are the full-size cases.
WORKLOADS = {
    "plain_fp64_1000x500": Workload("plain_fp64_1000x500", 1, 1000, 500, 10, 20, 4, 100, "f64", sigma=0.01),
    "nmf_fp32_20000x5000": Workload("nmf_fp32_20000x5000", 2, 20000, 5000, 50, 60, 4, 200, "f32", sigma=0.05),
    "separable_fp32_10000x100000": Workload("separable_fp32_10000x100000", 3, 10000, 100000, 20, 30, 2, 0,
                                            "f32", separable=True, sep_noise=1e-3),
    "precision_100000x20000": Workload("precision_100000x20000", 4, 100000, 20000, 100, 120, 4, 0, "f32",
                                       sigma=0.05),
}


def make_inputs(w: Workload, *, m=None, n=None, storage=None, two_sided=True, want_init=True):
    """Draw every input of a workload (optionally at a reduced size).

    Returns a dict with float64 arrays: A (rounded to the storage precision
    and cast back, so both sides see the same values), Omega_L (n x k),
    Omega_R (m x k), U1, V1, and for separable data the planted indices.
    """
    m = w.m if m is None else m
    n = w.n if n is None else n
    storage = storage or ("f64" if w.dtype == "f64" else "f32")
    sdt = np.float64 if storage == "f64" else np.float32
    out = {}
    if w.separable:
        A, planted = separable_matrix(m, n, w.r, w.sep_noise, 100 * w.index, dtype=sdt)
        out["planted"] = planted
    else:
        A = nmf_matrix(m, n, w.r, w.sigma, 100 * w.index, dtype=sdt)
    out["A"] = A
    g = _rng(100 * w.index + 1)
    out["Omega_L"] = g.standard_normal((n, w.k))
    if two_sided:
        out["Omega_R"] = g.standard_normal((m, w.k))
    if want_init:
        mean_a = float(np.mean(A, dtype=np.float64))
        out["U1"], out["V1"] = init_factors(mean_a, m, n, w.r, 100 * w.index + 2)
    return out


# Serving workload: a stream of uneven factorisation requests.
SERVING = dict(count=2000, m=(500, 20000), n=(200, 8000), r=(5, 64), oversample=10, q=2, iters=100, sigma=0.05)


def serving_requests(count: int = SERVING["count"], qps: float = 0.0, seed: int = 500):
    """Shapes and arrival times of the serving workload: m and n log-uniform
    on their ranges, r uniform on [5, 64], k = r + 10; Poisson arrivals at
    `qps` requests per second (all at t = 0 when qps == 0).  Returns int64
    arrays m, n, r, k and float64 arrival times in seconds."""
    g = _rng(seed)
    lo_m, hi_m = SERVING["m"]
    lo_n, hi_n = SERVING["n"]
    m = np.rint(np.exp(g.uniform(math.log(lo_m), math.log(hi_m), count))).astype(np.int64)
    n = np.rint(np.exp(g.uniform(math.log(lo_n), math.log(hi_n), count))).astype(np.int64)
    r = g.integers(SERVING["r"][0], SERVING["r"][1] + 1, count).astype(np.int64)
    k = r + SERVING["oversample"]
    t = np.cumsum(g.exponential(1.0 / qps, count)) if qps > 0 else np.zeros(count)
    return m, n, r, k, t


def expected_rms(r: int, sigma: float) -> float:
    """Root mean square of an entry of W H + |sigma Z| with W, H uniform on
    [0, 1): E[(sum_l w_l h_l)^2] = r / 9 + r (r - 1) / 16, plus the noise's
    second moment sigma^2 (cross terms neglected)."""
    return math.sqrt(r / 9.0 + r * (r - 1) / 16.0 + sigma * sigma)
