"""Gaussian boson sampling by the chain rule over marginal probabilities (Sec. III, Alg. 1).

Step 1 draws the photon number n from P_n truncated at ``nmax`` and renormalised (the library's
``gbs_photon_number_pmf``). The positions x_1..x_n are then drawn one at a time: for every sample
with the same n, one ``gbs_sample_step`` call evaluates the m marginals q_n(x_1..x_{k-1}, l) on the
device (Theorem 1) and draws x_k by inverse CDF from a uniform the caller's generator supplies, so
a run is reproducible from its seed. The output configuration s counts the photons per mode.

All samples that share n advance together, so each step is one batched library call.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import gbs


@dataclass
class Sample:
    n: int
    positions: List[int]       # x_1..x_n in draw order
    configuration: np.ndarray  # s_j = number of photons in mode j


def truncated_photon_pmf(m: int, r: float, nmax: int) -> np.ndarray:
    """P_0..P_nmax renormalised over the truncation (odd n have probability 0)."""
    p = gbs.photon_number_pmf(m, r, nmax)
    tot = p.sum()
    if not tot > 0:
        raise ValueError("truncated photon-number distribution has no mass")
    return p / tot


class Sampler:
    def __init__(self, ctx: gbs.Context, state: gbs.State, m: int, r: float):
        self.ctx, self.state, self.m, self.r = ctx, state, int(m), float(r)

    def positions(self, n: int, count: int, rng: np.random.Generator, keep_weights: bool = False):
        """Draw `count` position sequences of n photons; optionally the per-step weights
        (list over k of (count, m) arrays)."""
        import torch
        dev = self.ctx.torch_device
        if n > gbs.GBS_MARGINAL_KMAX:
            raise ValueError(f"n = {n} exceeds the marginal limit {gbs.GBS_MARGINAL_KMAX}")
        x = np.zeros((count, n), dtype=np.int32)
        weights = []
        for k in range(n):
            u = torch.from_numpy(rng.random(count)).to(dev)
            w = torch.empty((count, self.m), dtype=torch.float64, device=dev) if keep_weights else None
            nxt = self.ctx.sample_step(self.state, n, (x[:, :k].reshape(-1), np.arange(count + 1, dtype=np.int64) * k),
                                       u, weights_out=w)
            x[:, k] = nxt.cpu().numpy()
            if keep_weights:
                weights.append(w.cpu().numpy())
        return (x, weights) if keep_weights else x

    def sample(self, count: int, rng: np.random.Generator, nmax: int, n: Optional[int] = None) -> List[Sample]:
        """`count` samples: n from the truncated P_n (or fixed), then the positions."""
        if n is None:
            pmf = truncated_photon_pmf(self.m, self.r, nmax)
            ns = rng.choice(len(pmf), size=count, p=pmf)
        else:
            ns = np.full(count, int(n))
        out: List[Optional[Sample]] = [None] * count
        for nv in np.unique(ns):
            idx = np.nonzero(ns == nv)[0]
            xs = self.positions(int(nv), len(idx), rng) if nv > 0 else np.zeros((len(idx), 0), dtype=np.int32)
            for i, row in zip(idx, xs):
                out[i] = Sample(int(nv), [int(v) for v in row], np.bincount(row, minlength=self.m))
        return out


class BruteForceSampler:
    """Brute-force sampling of output patterns (App. I): the probabilities of every n-photon pattern
    are evaluated once (gbs_prob_sweep, sub-hafnians shared across patterns), then each sample is the
    pattern whose interval of the cumulative distribution holds a uniform (gbs_sweep_sample). Exact
    for p_n(s) / sum_s p_n(s); memory and time grow with C(m + n - 1, n)."""

    def __init__(self, ctx, state, n: int, collisions: bool = True):
        import itertools
        self.ctx = ctx
        self.n = n
        self.m = state.m
        self.collisions = collisions
        self.prob = ctx.prob_sweep(state, n, collisions)
        gen = itertools.combinations_with_replacement if collisions else itertools.combinations
        self._gen = lambda: gen(range(self.m), n)

    def sample_indices(self, count: int, rng):
        import torch
        u = torch.from_numpy(rng.random(count)).to(self.ctx.torch_device)
        idx, total = self.ctx.sweep_sample(self.prob, u)
        return idx.cpu().numpy(), float(total.cpu()[0])

    def patterns(self, indices):
        """Mode lists of the given pattern indices (lexicographic order)."""
        import itertools
        want = sorted(set(int(i) for i in indices))
        out, j = {}, 0
        for i, p in enumerate(self._gen()):
            if j < len(want) and i == want[j]:
                out[i] = p
                j += 1
                if j == len(want):
                    break
        return [out[int(i)] for i in indices]
