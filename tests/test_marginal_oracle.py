"""Pins for the marginal-probability oracle (Theorem 1 of Sec. III D) against the definition.

The marginal q_n(x_1..x_k) is defined as q_n summed over all completions (Eq. marginal_definition),
so brute force over [m]^(n-k) is the reference; closed forms: q = 1 for the empty prefix and 1/m for
one photon; consistency: summing the last position of a prefix gives the shorter prefix's marginal.
"""
import math

import numpy as np
import pytest

from oracle import marginal as M
from paper_1908_10070_amd import inputs

# (m, n, prefix) cases; several with repeated modes (collisions)
CASES = [
    (3, 4, [1, 0]), (3, 4, [2, 0, 0]), (3, 4, [1, 2, 0, 2]),
    (4, 4, [1, 2, 2]), (4, 4, [0, 0, 2]), (4, 4, [3, 1]),
    (5, 6, [2, 2, 1, 3]), (5, 6, [1, 2, 1, 1, 0]), (5, 6, [2, 1, 4]),
    (3, 6, [1, 1, 1, 1]), (3, 6, [2, 2, 0, 0, 2]), (6, 6, [0, 3, 5]),
]


def W_of(m, seed=11):
    U = inputs.haar_unitary(m, np.random.default_rng(seed + m))
    return U @ U.T


@pytest.mark.parametrize("m,n,prefix", CASES)
def test_theorem1_equals_brute_force(m, n, prefix):
    W = W_of(m)
    b = M.marginal_brute(W, prefix, n)
    assert abs(M.marginal_thm1(W, prefix, n) - b) <= 1e-12 * b
    assert abs(M.marginal_split(W, prefix, n) - b) <= 1e-12 * b


def test_statement_reading_of_B_fails_with_collisions():
    """Taking B from X_k minus a (the statement's literal range) instead of X_k minus a' (the
    proof's) changes the result once modes repeat -- the pin that fixes the reading."""
    W = W_of(4)
    for prefix in ([1, 2, 2], [0, 0, 2]):
        b = M.marginal_brute(W, prefix, 4)
        assert abs(M.marginal_thm1(W, prefix, 4, b_excludes="a") - b) > 1e-3 * b
    # without collisions the two readings agree
    b = M.marginal_brute(W, [0, 1, 2], 4)
    assert abs(M.marginal_thm1(W, [0, 1, 2], 4, b_excludes="a") - b) <= 1e-12 * b


@pytest.mark.parametrize("m,n", [(3, 4), (5, 6), (8, 8), (16, 10)])
def test_closed_forms_k0_k1(m, n):
    W = W_of(m)
    assert abs(M.marginal_split(W, [], n) - 1.0) < 1e-12
    for x1 in (0, m - 1):
        assert abs(M.marginal_split(W, [x1], n) - 1.0 / m) < 1e-12


def test_full_prefix_is_the_sequence_probability():
    W = W_of(5)
    x = [3, 0, 4, 0, 1, 2]
    assert abs(M.marginal_split(W, x, 6) - M.q_sequence(W, x)) <= 1e-12 * M.q_sequence(W, x)


@pytest.mark.parametrize("m,n,prefix", [(6, 8, [2, 5, 2]), (7, 8, [0, 3, 6, 1]), (5, 10, [4, 4, 1, 0, 4])])
def test_chain_consistency(m, n, prefix):
    """sum over x_k of q(x_1..x_k) = q(x_1..x_{k-1}) (the conditionals of Eq. ConPro normalise)."""
    W = W_of(m)
    parent = M.marginal_split(W, prefix[:-1], n)
    kids = sum(M.marginal_split(W, prefix[:-1] + [l], n) for l in range(m))
    assert abs(kids - parent) <= 1e-12 * parent


def test_planted_mistakes_break_the_brute_force_pin(monkeypatch):
    """A dropped (n-k)!, a conjugate left off a' and a shifted binomial each break equality."""
    W = W_of(5)
    prefix, n = [2, 2, 1, 3], 6
    b = M.marginal_brute(W, prefix, n)
    good = M.F_weight

    monkeypatch.setattr(M, "F_weight", lambda m, n, k, mu, j1, j2: good(m, n, k, mu, j1, j2) / math.factorial(n - k))
    assert abs(M.marginal_thm1(W, prefix, n) - b) > 1e-3 * b
    monkeypatch.setattr(M, "F_weight", lambda m, n, k, mu, j1, j2: good(m, n, k, mu + 2, j1, j2))
    assert abs(M.marginal_thm1(W, prefix, n) - b) > 1e-3 * b
    monkeypatch.setattr(M, "F_weight", good)
    conj = np.conj
    monkeypatch.setattr(M.np, "conj", lambda z: z)
    try:
        assert abs(M.marginal_thm1(W, prefix, n) - b) > 1e-3 * b
    finally:
        monkeypatch.setattr(M.np, "conj", conj)


def test_per01_is_the_permutation_sum():
    import itertools
    rng = np.random.default_rng(0)
    for r in range(0, 7):
        for _ in range(10):
            S = (rng.random((r, r)) < 0.6).astype(int)
            brute = sum(all(S[i, p[i]] for i in range(r)) for p in itertools.permutations(range(r)))
            assert M.per01(S) == brute
    # all-ones block of size c has permanent c!
    assert M.per01(np.ones((5, 5), dtype=int)) == 120
