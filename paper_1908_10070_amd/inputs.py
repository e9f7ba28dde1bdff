"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers only: interferometers, squeezing vectors, output
patterns, random symmetric matrices and arrival times. It holds none of the
method's arithmetic (no B matrix, no hafnian, no probability), so both the GPU
path and the CPU oracle can take their inputs from it.

Recipes (numpy ``default_rng`` / PCG64):

* Haar unitary: Z = (N + iN)/sqrt(2), Z = QR, U = Q diag(R_ii/|R_ii|).
  The paper draws its interferometers at random with m = n^2 modes (Sec. III E)
  without stating the measure; this is the usual Haar recipe.
* Collision-free output pattern: a uniformly random n-subset of [m], as a sorted
  mode list (x_1 < ... < x_n), drawn as the n smallest of m uniform keys.
* Random complex-symmetric matrix: M = (a + ib)/sqrt(2), a, b ~ N(0, 1), A = (M + M^t)/2.
* Arrivals: exponential inter-arrival times at rate lam (a Poisson stream).
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Sequence

import numpy as np


def haar_unitary(m: int, rng: np.random.Generator) -> np.ndarray:
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def random_symmetric(n: int, batch: int, rng: np.random.Generator) -> np.ndarray:
    a = rng.standard_normal((batch, n, n))
    b = rng.standard_normal((batch, n, n))
    mm = (a + 1j * b) / np.sqrt(2.0)
    return np.ascontiguousarray((mm + np.swapaxes(mm, 1, 2)) / 2.0)


def bipartite(k: int, rng: np.random.Generator):
    """(W, A): a k x k complex Gaussian W = (a + ib)/sqrt(2) and the 2k x 2k block matrix
    A = [[0, W], [W^t, 0]] (whose hafnian is the permanent of W)."""
    W = (rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) / np.sqrt(2.0)
    A = np.block([[np.zeros((k, k)), W], [W.T, np.zeros((k, k))]])
    return W, np.ascontiguousarray(A)


def collision_free_patterns(m: int, n: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """count x n int32 array; each row a sorted uniformly random n-subset of range(m)."""
    if n > m:
        raise ValueError("n > m")
    out = np.empty((count, n), dtype=np.int32)
    step = 8192
    for s in range(0, count, step):
        e = min(count, s + step)
        keys = rng.random((e - s, m))
        if n:
            out[s:e] = np.sort(np.argpartition(keys, n - 1, axis=1)[:, :n], axis=1)
    return out


def all_patterns(m: int, n: int) -> np.ndarray:
    """All C(m, n) collision-free patterns in lexicographic order."""
    return np.array(list(itertools.combinations(range(m), n)), dtype=np.int32).reshape(-1, n)


def pack(patterns: Sequence[Sequence[int]]):
    """Mode lists -> (modes int32 flat, offsets int64 of length batch+1)."""
    lens = np.fromiter((len(p) for p in patterns), dtype=np.int64, count=len(patterns))
    offsets = np.zeros(len(patterns) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    modes = np.empty(int(offsets[-1]), dtype=np.int32)
    for i, p in enumerate(patterns):
        modes[offsets[i]:offsets[i + 1]] = p
    return modes, offsets


def poisson_arrivals(rate: float, count: int, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream."""
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# --------------------------------------------------------------- workloads


@dataclasses.dataclass
class GBSSetup:
    U: np.ndarray
    r: np.ndarray


def gbs_setup(m: int, r: float, seed: int) -> GBSSetup:
    rng = np.random.default_rng(seed)
    return GBSSetup(haar_unitary(m, rng), np.full(m, float(r)))


def config1():
    """m = 16, r = 0.5, every collision-free 8-photon pattern (lexicographic) plus the vacuum."""
    st = gbs_setup(16, 0.5, 1001)
    return st, all_patterns(16, 8)


def config2(batch: int = 4096, n: int = 24):
    """4096 independent complex-symmetric 24x24 matrices."""
    return random_symmetric(n, batch, np.random.default_rng(1002))


def config3(count: int = 100000, n: int = 20):
    """m = 50, r = 0.88, uniformly random collision-free 20-photon patterns."""
    st = gbs_setup(50, 0.88, 1003)
    pats = collision_free_patterns(50, n, count, np.random.default_rng(2003))
    return st, pats


def config4_requests(count: int, rate: float, seed: int = 3004) -> tuple:
    """Served stream on the config-3 state: (arrival times, list of mode lists).

    Photon numbers are even and uniform in {8, ..., 32}; each request a random
    collision-free pattern of that size.
    """
    rng = np.random.default_rng(seed)
    t = poisson_arrivals(rate, count, rng)
    ns = 2 * rng.integers(4, 17, size=count)
    pats: List[np.ndarray] = []
    for n in ns:
        pats.append(collision_free_patterns(50, int(n), 1, rng)[0])
    return t, pats


def config5(count: int = 64):
    """m = 60, r = 0.88; pattern sizes cycling 36, 40, 44 (B_S submatrices of large size)."""
    st = gbs_setup(60, 0.88, 1005)
    rng = np.random.default_rng(2005)
    sizes = [36, 40, 44]
    pats = [collision_free_patterns(60, sizes[i % 3], 1, rng)[0] for i in range(count)]
    return st, pats
