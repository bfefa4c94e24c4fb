"""Seeded synthetic inputs: planted-cluster time series and tie-heavy similarity matrices.

This module only draws random numbers. It holds none of the TMFG arithmetic, so both the
GPU path and the CPU oracle can consume its outputs.

The paper evaluates on UCR time-series datasets (Section 5, Table 1: n from 930 to 19412
series, lengths 46 to 2709), with the similarity matrix being the Pearson correlation of
every pair of series. Those datasets are not used here; seeded random-walk series with
planted clusters stand in for them, at the same scale.

Recipe (every input is generated in float64 and cast once to float32):
  * prototype k: a Gaussian random walk, P_k[t] = sum_{s<=t} e_s with e_s ~ N(0, 1);
  * member i of cluster k: X_i = P_k + sigma_i * N(0, 1)^L;
  * pure-noise series: N(0, 1)^L;
  * cluster sizes: equal, or 1 + Multinomial(n_clustered - K, pi) with pi ~ Dirichlet(1_K)
    so that every cluster has at least one member;
  * finally a seeded permutation of the rows.
The random generator is numpy's PCG64 seeded through SeedSequence.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        ss = seed
    else:
        ss = np.random.SeedSequence(seed)
    return np.random.Generator(np.random.PCG64(ss))


@dataclasses.dataclass
class Series:
    X: np.ndarray          # (n, L) float32, row-major
    labels: np.ndarray     # (n,) int32; -1 marks a pure-noise series
    name: str


def dirichlet_sizes(rng: np.random.Generator, n_clustered: int, k: int) -> np.ndarray:
    """Cluster sizes 1 + Multinomial(n_clustered - k, pi), pi ~ Dirichlet(1_k)."""
    if k < 1 or n_clustered < k:
        raise ValueError("need at least one member per cluster")
    pi = rng.dirichlet(np.ones(k))
    return 1 + rng.multinomial(n_clustered - k, pi)


def planted_clusters(n: int, L: int, sizes: Sequence[int], sigma, n_noise: int = 0,
                     seed=0, name: str = "planted") -> Series:
    """Random-walk prototypes plus i.i.d. Gaussian noise per member.

    ``sigma`` is either a scalar or a pair (lo, hi) for a per-series U(lo, hi) draw.
    """
    sizes = np.asarray(sizes, dtype=np.int64)
    if int(sizes.sum()) + n_noise != n:
        raise ValueError("cluster sizes plus noise series must add up to n")
    rng = _rng(seed)
    k = len(sizes)
    protos = np.cumsum(rng.standard_normal((k, L)), axis=1)
    n_cl = int(sizes.sum())
    labels = np.repeat(np.arange(k, dtype=np.int32), sizes)
    if np.isscalar(sigma):
        sig = np.full(n_cl, float(sigma))
    else:
        lo, hi = sigma
        sig = rng.uniform(lo, hi, size=n_cl)
    X = protos[labels] + sig[:, None] * rng.standard_normal((n_cl, L))
    if n_noise:
        X = np.concatenate([X, rng.standard_normal((n_noise, L))], axis=0)
        labels = np.concatenate([labels, np.full(n_noise, -1, dtype=np.int32)])
    perm = rng.permutation(n)
    return Series(X=np.ascontiguousarray(X[perm].astype(np.float32)),
                  labels=labels[perm].astype(np.int32), name=name)


# ---------------------------------------------------------------------------------------
# The five workloads. C1 is the small case the oracle finishes in well under a second;
# C2 and C3 are the single-build sizes; C4 is the batched mix; C5 the serving trace.
# ---------------------------------------------------------------------------------------

def config_c1() -> Series:
    """n=200, L=128: 5 equal clusters of 40, sigma=0.5."""
    return planted_clusters(200, 128, [40] * 5, 0.5, seed=np.random.SeedSequence(1), name="C1")


def config_c2() -> Series:
    """n=5000, L=512: 20 clusters with Dirichlet(1) sizes, sigma_i ~ U(0.3, 1.0)."""
    ss = np.random.SeedSequence(2)
    size_rng, data_ss = [_rng(s) if i == 0 else s for i, s in enumerate(ss.spawn(2))]
    sizes = dirichlet_sizes(size_rng, 5000, 20)
    return planted_clusters(5000, 512, sizes, (0.3, 1.0), seed=data_ss, name="C2")


def config_c3() -> Series:
    """n=20000, L=1024: 18000 clustered (50 Dirichlet clusters) plus 2000 white-noise series."""
    ss = np.random.SeedSequence(3)
    size_rng, data_ss = [_rng(s) if i == 0 else s for i, s in enumerate(ss.spawn(2))]
    sizes = dirichlet_sizes(size_rng, 18000, 50)
    return planted_clusters(20000, 1024, sizes, (0.3, 1.0), n_noise=2000, seed=data_ss,
                            name="C3")


def batch_instance(ss: np.random.SeedSequence, n_lo: int = 64, n_hi: int = 4096,
                   L: Optional[int] = None, L_lo: int = 64, L_hi: int = 512) -> Series:
    """One instance of the uneven batch: n log-uniform in [n_lo, n_hi], L uniform, K in 2..30."""
    rng = _rng(ss)
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    n = max(n, 4)
    if L is None:
        L = int(rng.integers(L_lo, L_hi + 1))
    k = int(rng.integers(2, 31))
    k = min(k, n)
    sizes = dirichlet_sizes(rng, n, k)
    data_ss = np.random.SeedSequence(int(rng.integers(0, 2**63 - 1)))
    return planted_clusters(n, L, sizes, (0.3, 1.0), seed=data_ss, name="C4")


def config_c4(count: int = 512) -> List[Series]:
    """512 independent instances, n log-uniform over 64..4096, L uniform over 64..512."""
    return [batch_instance(s) for s in np.random.SeedSequence(4).spawn(count)]


@dataclasses.dataclass
class Request:
    t_arrival: float       # seconds after the start of the trace
    series: Series


def serving_trace(qps: float, count: int, seed: int = 5, n_lo: int = 100, n_hi: int = 8000,
                  L: int = 256) -> List[Request]:
    """Poisson arrivals (exponential gaps of mean 1/qps) of rolling-window requests.

    Each request is a fresh window of n log-uniform in [n_lo, n_hi] correlated random-walk
    series of length L.
    """
    ss = np.random.SeedSequence(seed)
    gap_ss, *req_ss = ss.spawn(count + 1)
    gaps = _rng(gap_ss).exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps) - gaps[0]
    return [Request(float(t[i]), batch_instance(req_ss[i], n_lo, n_hi, L=L))
            for i in range(count)]


# ---------------------------------------------------------------------------------------
# Similarity matrices given directly (not through series).
# ---------------------------------------------------------------------------------------

def grid_symmetric(n: int, seed, levels: int = 8, lo: float = -1.0, hi: float = 1.0,
                   diag: float = 1.0) -> np.ndarray:
    """A symmetric float32 matrix whose off-diagonal entries sit on a coarse grid.

    Entries are multiples of (hi - lo) / levels, so many sums tie exactly; such matrices
    exercise every tie rule.
    """
    rng = _rng(seed)
    steps = rng.integers(0, levels + 1, size=(n, n))
    A = lo + steps * ((hi - lo) / levels)
    A = np.triu(A, 1)
    A = A + A.T
    np.fill_diagonal(A, diag)
    return np.ascontiguousarray(A.astype(np.float32))


def random_symmetric(n: int, seed, scale: float = 1.0) -> np.ndarray:
    """A symmetric float32 matrix with continuous entries in [-scale, scale]."""
    rng = _rng(seed)
    A = rng.uniform(-scale, scale, size=(n, n)).astype(np.float32)
    A = np.triu(A, 1)
    A = A + A.T
    np.fill_diagonal(A, np.float32(1.0))
    return np.ascontiguousarray(A)
