"""CPU oracle for marginal probabilities of the position sequence -- TEST INFRASTRUCTURE ONLY.

Follows Sec. III of the paper (Wu et al., arXiv:1908.10070) for identical squeezing on every mode,
where the distribution of the photon positions x = (x_1, ..., x_n) in [m]^n is

    q_n(x) = |Haf(W_x)|^2 / f_n,   W = U U^t,   W_x(i, j) = W(x_i, x_j),
    f_n = n! C((m + n)/2 - 1, n/2)                               (Sec. III B, Eq. EqDisE),

and the marginal of a prefix is the sum over the remaining positions (Eq. marginal_definition).

* ``q_sequence``      -- q_n(x) from the definition.
* ``marginal_brute``  -- the marginal by summing q_n over all m^(n-k) completions.
* ``marginal_thm1``   -- Theorem 1 written out: sums over j1, j2, a, a', mu, A, B of
                         Haf(R_a) Haf(R*_a') F Per(S_{A,B}) Haf(R_e) Haf(R*_e'), with
                         F = (n-k)!/f_n C((n-k+mu+m)/2 - 1, k - j1 - j2 + m/2 - 1).
                         Reading: B ranges over mu-subsets of X_k minus a' (as the proof uses it);
                         ``b_excludes="a"`` takes the statement's literal X_k minus a instead.
* ``marginal_split``  -- the same sum regrouped: for fixed A the sum over a is
                         G_j(C) = sum over 2j-subsets a of C of Haf(R_a) Haf(R_{C minus a}) with
                         C = X_k minus A (likewise for a', B), so
                         q = sum_{mu, A, B} Per(S_{A,B}) sum_{j1, j2} F G_{j1}(X_k - A) conj G_{j2}(X_k - B).

Hafnians come from ``oracle.haf_enum`` (the matching sum), permanents of the 0/1 matrices from
their definition; no blocking or reordering beyond what the formulas state.
"""
from __future__ import annotations

import itertools
import math
from typing import Sequence

import numpy as np

from . import oracle as _o


def haf_sub(W: np.ndarray, modes: Sequence[int]) -> complex:
    """Haf of W restricted to the mode list (rows and columns repeated for repeated modes)."""
    if len(modes) == 0:
        return 1.0 + 0.0j
    if len(modes) % 2:
        return 0.0j
    idx = np.asarray(modes, dtype=np.int64)
    return complex(_o.haf_enum(W[np.ix_(idx, idx)]))


def q_sequence(W: np.ndarray, x: Sequence[int], n: int | None = None) -> float:
    """q_n(x) = |Haf(W_x)|^2 / f_n for a full sequence x of n positions (Eq. EqDisE)."""
    m = W.shape[0]
    n = len(x) if n is None else n
    return abs(haf_sub(W, x)) ** 2 / _o.f_n(m, n)


def marginal_brute(W: np.ndarray, prefix: Sequence[int], n: int) -> float:
    """q_n(x_1..x_k): q_n summed over every completion x_{k+1..n} in [m]^(n-k)."""
    m = W.shape[0]
    k = len(prefix)
    tot = 0.0
    for rest in itertools.product(range(m), repeat=n - k):
        tot += abs(haf_sub(W, list(prefix) + list(rest))) ** 2
    return tot / _o.f_n(m, n)


def per01(S: np.ndarray) -> int:
    """Permanent of a small 0/1 matrix: the sum over permutations, expanded row by row (row i picks
    an unused column j with S[i, j] = 1), memoised on the set of columns already used."""
    r = S.shape[0]
    rows = [[j for j in range(r) if S[i, j]] for i in range(r)]
    memo = {}

    def rec(i, used):
        if i == r:
            return 1
        key = (i, used)
        if key not in memo:
            memo[key] = sum(rec(i + 1, used | (1 << j)) for j in rows[i] if not used >> j & 1)
        return memo[key]

    return rec(0, 0)


def F_weight(m: int, n: int, k: int, mu: int, j1: int, j2: int) -> float:
    """F_j^(mu) = (n - k)! / f_n * C((n - k + mu + m)/2 - 1, k - j1 - j2 + m/2 - 1) (Theorem 1).
    Both binomial arguments may be half-integers (odd m): the generalized binomial
    Gamma(a + 1) / (Gamma(b + 1) Gamma(a - b + 1)), zero when b < 0 or a - b is a negative integer."""
    a = (n - k + mu + m) / 2 - 1
    b = k - j1 - j2 + m / 2 - 1
    if b < 0:
        return 0.0
    d = a - b
    if d < 0 and float(d).is_integer():
        return 0.0
    c = math.exp(math.lgamma(a + 1) - math.lgamma(b + 1) - math.lgamma(d + 1))
    sign = 1.0
    for v in (a + 1, b + 1, d + 1):  # signs of Gamma at negative non-integer arguments
        if v < 0 and math.floor(v) % 2 == 1:
            sign = -sign
    return math.factorial(n - k) / _o.f_n(m, n) * sign * c


def _j_range(k: int, n: int):
    return range(max(0, math.ceil(k - n / 2)), k // 2 + 1)


def _mu_range(k: int, n: int, j1: int, j2: int):
    lo = max(0, 3 * k - 2 * (j1 + j2) - n)
    hi = k - 2 * max(j1, j2)
    return [mu for mu in range(lo, hi + 1) if (mu - k) % 2 == 0]


def marginal_thm1(W: np.ndarray, prefix: Sequence[int], n: int, b_excludes: str = "a_prime") -> float:
    """Theorem 1, term by term (see the module docstring for the reading of B's range)."""
    m = W.shape[0]
    x = list(prefix)
    k = len(x)
    X = list(range(k))  # positions 1..k of the prefix
    tot = 0.0 + 0.0j
    for j1 in _j_range(k, n):
        for j2 in _j_range(k, n):
            for a in itertools.combinations(X, 2 * j1):
                ha = haf_sub(W, [x[i] for i in a])
                rest_a = [i for i in X if i not in a]
                for a2 in itertools.combinations(X, 2 * j2):
                    ha2 = np.conj(haf_sub(W, [x[i] for i in a2]))
                    rest_a2 = [i for i in X if i not in a2]
                    pool_b = rest_a2 if b_excludes == "a_prime" else rest_a
                    for mu in _mu_range(k, n, j1, j2):
                        F = F_weight(m, n, k, mu, j1, j2)
                        if F == 0.0:
                            continue
                        for A in itertools.combinations(rest_a, mu):
                            e = [i for i in rest_a if i not in A]
                            he = haf_sub(W, [x[i] for i in e])
                            for B in itertools.combinations(pool_b, mu):
                                S = np.array([[int(x[Ai] == x[Bj]) for Bj in B] for Ai in A], dtype=np.int64)
                                per = per01(S.reshape(mu, mu))
                                if per == 0:
                                    continue
                                e2 = [i for i in X if i not in a2 and i not in B]
                                he2 = np.conj(haf_sub(W, [x[i] for i in e2]))
                                tot += ha * ha2 * F * per * he * he2
    return float(tot.real)


def split_sums(W: np.ndarray, prefix: Sequence[int], C: Sequence[int], memo: dict | None = None) -> dict:
    """G_j(C) = sum over a subset of C with |a| = 2j of Haf(R_a) Haf(R_{C minus a}), for every j.
    ``memo`` caches Haf(R_a) by position tuple (each evaluated once, same value either way)."""
    x = list(prefix)

    def h(pos):
        if memo is None:
            return haf_sub(W, [x[i] for i in pos])
        key = tuple(pos)
        if key not in memo:
            memo[key] = haf_sub(W, [x[i] for i in pos])
        return memo[key]

    G = {}
    for j in range(len(C) // 2 + 1):
        g = 0.0j
        for a in itertools.combinations(C, 2 * j):
            e = [i for i in C if i not in a]
            g += h(a) * h(e)
        G[j] = g
    return G


def marginal_split(W: np.ndarray, prefix: Sequence[int], n: int) -> float:
    """Theorem 1 with the sum over a (and a') taken inside, for fixed A (and B)."""
    m = W.shape[0]
    x = list(prefix)
    k = len(x)
    X = list(range(k))
    Gs = {}
    memo: dict = {}
    for r in range(k + 1):
        for A in itertools.combinations(X, r):
            C = tuple(i for i in X if i not in A)
            Gs[A] = split_sums(W, x, C, memo)
    tot = 0.0 + 0.0j
    for mu in range(k + 1):
        # Per(S_{A,B}) vanishes unless A and B carry the same multiset of modes (otherwise a mode
        # has more rows than matching columns), so only pairs within one multiset are formed.
        by_modes: dict = {}
        for A in itertools.combinations(X, mu):
            by_modes.setdefault(tuple(sorted(x[i] for i in A)), []).append(A)
        pairs = [(A, B) for group in by_modes.values() for A in group for B in group]
        for A, B in pairs:
            S = np.array([[int(x[Ai] == x[Bj]) for Bj in B] for Ai in A], dtype=np.int64)
            per = per01(S.reshape(mu, mu))
            if per == 0:
                continue
            GA, GB = Gs[A], Gs[B]
            for j1 in _j_range(k, n):
                for j2 in _j_range(k, n):
                    if mu not in _mu_range(k, n, j1, j2):
                        continue
                    F = F_weight(m, n, k, mu, j1, j2)
                    if F == 0.0 or j1 not in GA or j2 not in GB:
                        continue
                    tot += F * per * GA[j1] * np.conj(GB[j2])
    return float(tot.real)
