"""Pins for the CPU oracle: each check ties it to something other than itself.

Closed forms, textbook special cases, invariants of the hafnian and the paper's
own probability identities. Hafnian definition: Sec. II C (Eq. HafMatch);
probabilities: Eq. ProOri, Eq. Eqdistribution, Sec. III B and App. A/B.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1908_10070_amd import inputs

HAFS = {
    "enum": oracle.haf_enum,
    "pt": oracle.haf_pt,
    "pt_ld": oracle.haf_pt_ld,
}


def dfact(n):
    return math.prod(range(n - 1, 0, -2)) if n > 0 else 1


def rand_sym(n, rng):
    return inputs.random_symmetric(n, 1, rng)[0]


def perm_brute(W):
    W = np.asarray(W)
    k = W.shape[0]
    return sum(math.prod(W[i, p[i]] for i in range(k)) for p in itertools.permutations(range(k)))


def perm_ryser(W):
    """Ryser's inclusion-exclusion formula (textbook), independent of the hafnian code."""
    W = np.asarray(W, dtype=np.complex128)
    k = W.shape[0]
    tot = 0j
    for mask in range(1, 1 << k):
        cols = [j for j in range(k) if mask >> j & 1]
        rows = W[:, cols].sum(axis=1)
        tot += (-1) ** len(cols) * np.prod(rows)
    return (-1) ** k * tot


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ------------------------------------------------------------ hafnian pins


@pytest.mark.parametrize("name", list(HAFS))
def test_empty_and_odd(name):
    f = HAFS[name]
    assert f(np.zeros((0, 0))) == 1
    rng = np.random.default_rng(1)
    for n in (1, 3, 5):
        assert f(rand_sym(n, rng)) == 0


@pytest.mark.parametrize("name", list(HAFS) + ["py"])
def test_n2_n4_worked_example(name):
    """n = 4: V12 V34 + V13 V24 + V14 V23 (the paper's worked example, Sec. II C)."""
    f = HAFS.get(name, oracle.haf_py)
    rng = np.random.default_rng(2)
    A = rand_sym(2, rng)
    assert abs(f(A) - A[0, 1]) < 1e-15 * abs(A[0, 1])
    V = rand_sym(4, rng)
    ref = V[0, 1] * V[2, 3] + V[0, 2] * V[1, 3] + V[0, 3] * V[1, 2]
    assert rel(f(V), ref) < 1e-14


@pytest.mark.parametrize("name", list(HAFS))
def test_all_ones_double_factorial(name):
    f = HAFS[name]
    top = 18 if name == "enum" else 16
    for n in range(2, top + 1, 2):
        assert f(np.ones((n, n))) == dfact(n), n


@pytest.mark.parametrize("name", list(HAFS))
def test_rank_one(name):
    """Every matching of v v^t contributes prod v_i, so Haf = (n-1)!! prod v_i."""
    f = HAFS[name]
    rng = np.random.default_rng(3)
    for n in (2, 6, 10, 12):
        v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        assert rel(f(np.outer(v, v)), dfact(n) * np.prod(v)) < 1e-12, n


@pytest.mark.parametrize("name", list(HAFS))
def test_bipartite_is_permanent(name):
    """Haf([[0, W], [W^t, 0]]) = Per(W)."""
    f = HAFS[name]
    rng = np.random.default_rng(4)
    for k in range(1, 7):
        W = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
        A = np.block([[np.zeros((k, k)), W], [W.T, np.zeros((k, k))]])
        ref = perm_brute(W) if k <= 5 else perm_ryser(W)
        assert rel(f(A), ref) < 1e-12, k


@pytest.mark.parametrize("name", list(HAFS))
def test_block_diagonal_factorises(name):
    f = HAFS[name]
    rng = np.random.default_rng(5)
    for a, c in [(2, 4), (4, 6), (6, 6), (2, 10)]:
        A, C = rand_sym(a, rng), rand_sym(c, rng)
        Z = np.zeros((a, c))
        full = np.block([[A, Z], [Z.T, C]])
        assert rel(f(full), f(A) * f(C)) < 1e-12


@pytest.mark.parametrize("name", list(HAFS))
def test_invariants(name):
    """Haf(P A P^t) = Haf(A) (App. B); Haf(cA) = c^(n/2) Haf(A); Haf(conj A) = conj Haf(A)."""
    f = HAFS[name]
    rng = np.random.default_rng(6)
    for n in (6, 10, 12):
        A = rand_sym(n, rng)
        h = f(A)
        p = rng.permutation(n)
        assert rel(f(A[np.ix_(p, p)]), h) < 1e-12
        c = 0.7 - 0.4j
        assert rel(f(c * A), c ** (n // 2) * h) < 1e-12
        assert rel(f(np.conj(A)), np.conj(h)) < 1e-12


@pytest.mark.parametrize("name", list(HAFS))
def test_diagonal_ignored(name):
    f = HAFS[name]
    rng = np.random.default_rng(7)
    A = rand_sym(10, rng)
    B = A.copy()
    np.fill_diagonal(B, rng.standard_normal(10) * 5)
    # exact in real arithmetic; the power-trace route cancels the diagonal only up to rounding
    assert rel(f(B), f(A)) < (1e-15 if name == "enum" else 1e-10)


def test_power_trace_matches_enumeration():
    rng = np.random.default_rng(8)
    for n in (2, 4, 6, 8, 10, 12, 14, 16):
        for _ in range(3):
            A = rand_sym(n, rng)
            e = oracle.haf_enum(A)
            assert rel(oracle.haf_pt(A), e) < 1e-11, n
            assert rel(oracle.haf_pt_ld(A), e) < 1e-12, n


def test_python_matches_c_enumeration():
    rng = np.random.default_rng(9)
    for n in (2, 4, 6, 8):
        A = rand_sym(n, rng)
        assert rel(oracle.haf_py(A), oracle.haf_enum(A)) < 1e-13


def test_batch_wrappers():
    rng = np.random.default_rng(10)
    As = inputs.random_symmetric(8, 5, rng)
    one = np.array([oracle.haf_enum(a) for a in As])
    assert np.array_equal(oracle.haf_enum_batch(As), one)
    assert np.array_equal(oracle.haf_pt_batch(As), np.array([oracle.haf_pt(a) for a in As]))


def test_enum_memo_n20():
    """Memoised enumeration at a config-3 size agrees with the long-double power trace."""
    rng = np.random.default_rng(11)
    A = rand_sym(20, rng)
    assert rel(oracle.haf_enum(A), oracle.haf_pt_ld(A)) < 1e-11


# --------------------------------------------------------- probability pins


def test_vacuum_probability():
    """p(0) = 1 / prod cosh r_i (Eq. Eqdistribution at n = 0)."""
    st, _ = inputs.config1()
    p0 = oracle.prob_ref(st.U, st.r, [])
    assert abs(p0 - 0.1463386077562255) < 1e-15
    assert abs(p0 - 1 / math.cosh(0.5) ** 16) < 1e-16
    assert oracle.prob_ref(st.U, st.r, [0, 1, 2]) == 0.0


def test_paper_formula_equals_B_reading():
    """Eq. ProOri with W_s (column/row repetition) equals |Haf(B_x)|^2/(s! prod cosh r)."""
    rng = np.random.default_rng(12)
    U = inputs.haar_unitary(6, rng)
    r = 0.6
    for s in [(1, 1, 0, 2, 0, 0), (0, 2, 0, 0, 0, 0), (1, 1, 1, 1, 0, 0), (3, 0, 1, 0, 0, 0), (0, 0, 0, 0, 0, 0)]:
        modes = [j for j, c in enumerate(s) for _ in range(c)]
        a = oracle.prob_paper(U, r, s)
        b = oracle.prob_ref(U, np.full(6, r), modes)
        assert rel(b, a) < 1e-13, s


def test_W_s_example_layout():
    """The 6-mode example s = (1,1,0,2,0,0) of Sec. II C."""
    W = np.arange(36).reshape(6, 6)
    Ws = oracle.W_s_paper(W, (1, 1, 0, 2, 0, 0))
    idx = [0, 1, 3, 3]
    assert np.array_equal(Ws, W[np.ix_(idx, idx)])


@pytest.mark.parametrize("m,nmax", [(3, 8), (4, 6), (5, 6)])
def test_sum_over_configurations_is_Pn(m, nmax):
    """sum_{|s| = n} p(s) = P_n, all configurations with collisions (Eq. Eqdistribution)."""
    rng = np.random.default_rng(13 + m)
    U = inputs.haar_unitary(m, rng)
    r = 0.7
    for n in range(0, nmax + 1):
        pats = list(oracle.multisets(m, n))
        tot = float(np.sum(oracle.prob_ref_patterns(U, np.full(m, r), pats))) if n else \
            oracle.prob_ref(U, np.full(m, r), [])
        assert abs(tot - oracle.photon_number_prob(m, n, r)) < 1e-14, (m, n)


def test_nonuniform_squeezing_total_is_one():
    """Per-mode r_i: the total over all configurations with n <= N tends to 1."""
    rng = np.random.default_rng(14)
    U = inputs.haar_unitary(3, rng)
    r = np.array([0.2, 0.35, 0.1])
    tot = 0.0
    for n in range(0, 15, 2):
        pats = list(oracle.multisets(3, n))
        tot += float(np.sum(oracle.prob_ref_patterns(U, r, pats))) if n else oracle.prob_ref(U, r, [])
    assert abs(1 - tot) < 1e-8


def test_identity_interferometer_is_product_of_single_modes():
    """U = I: p(s) = prod_j |c_{s_j}(r_j)|^2 (single-mode squeezed states, Sec. II A)."""
    r = np.array([0.3, 0.5, 0.8, 0.2])
    U = np.eye(4, dtype=np.complex128)
    for s in [(2, 0, 0, 0), (2, 2, 0, 0), (0, 4, 2, 0), (1, 1, 0, 0), (2, 0, 2, 2), (0, 0, 0, 0)]:
        modes = [j for j, c in enumerate(s) for _ in range(c)]
        ref = math.prod(oracle.smss_prob(c, rr) for c, rr in zip(s, r))
        assert abs(oracle.prob_ref(U, r, modes) - ref) < 1e-15, s


@pytest.mark.parametrize("m,n", [(3, 2), (4, 4), (5, 4), (3, 6)])
def test_normalisation_f_n(m, n):
    """App. A: sum over x in [m]^n of |Haf(W_x)|^2 = f_n for W = U U^t."""
    rng = np.random.default_rng(15)
    U = inputs.haar_unitary(m, rng)
    W = U @ U.T
    xs = np.array(list(itertools.product(range(m), repeat=n)))
    mats = W[xs[:, :, None], xs[:, None, :]]
    tot = float(np.sum(np.abs(oracle.haf_enum_batch(mats)) ** 2))
    assert abs(tot - oracle.f_n(m, n)) < 1e-11 * oracle.f_n(m, n)


def test_single_mode_closed_form_normalised():
    for r in (0.3423, 0.8814):
        assert abs(sum(oracle.smss_prob(s, r) for s in range(0, 400, 2)) - 1) < 1e-12
        assert abs(sum(oracle.photon_number_prob(36, n, r) for n in range(0, 2000, 2)) - 1) < 1e-10


def test_config1_full_sweep_is_P8():
    """Config-1 state: the 490,314 eight-photon configurations sum to P_8 = 0.1004360452105159."""
    st, _ = inputs.config1()
    pats = np.array(list(oracle.multisets(16, 8)), dtype=np.int64)
    assert len(pats) == math.comb(23, 8)
    tot = 0.0
    step = 50000
    for s in range(0, len(pats), step):
        tot += float(np.sum(oracle.prob_ref_patterns(st.U, st.r, pats[s:s + step])))
    assert abs(tot - 0.1004360452105159) < 1e-14
    assert abs(tot - oracle.photon_number_prob(16, 8, 0.5)) < 1e-14


# ------------------------------------------- planted mistakes are caught


def _single_mode_convolution(r, n):
    """n-photon probability of independent single-mode squeezers r_i (Sec. II A): a passive
    interferometer conserves photon number, so this is the n-photon total of the GBS state."""
    dist = np.zeros(n + 1)
    dist[0] = 1.0
    for ri in r:
        dist = np.convolve(dist, [oracle.smss_prob(s, ri) for s in range(n + 1)])[: n + 1]
    return dist[n]


def _n_photon_total(B, r, n, with_sfact=True):
    m = B.shape[0]
    tot = 0.0
    for p in oracle.multisets(m, n):
        h = oracle.haf_enum(B[np.ix_(p, p)])
        sf = math.prod(math.factorial(c) for c in np.bincount(p, minlength=m)) if with_sfact else 1
        tot += abs(h) ** 2 / (sf * float(np.prod(np.cosh(r))))
    return tot


def test_nonuniform_n_photon_total_is_convolution():
    """Per-mode r_i: sum of p over all n-photon patterns = the single-mode convolution."""
    rng = np.random.default_rng(17)
    m, n = 4, 4
    U = inputs.haar_unitary(m, rng)
    r = np.array([0.3, 0.5, 0.7, 0.9])
    B = oracle.state_B(U, r)
    assert abs(_n_photon_total(B, r, n) - _single_mode_convolution(r, n)) < 1e-14


def test_pins_catch_planted_mistakes():
    """A conjugate transpose instead of a transpose, a dropped s!, or a dropped tanh each break a
    photon-number pin. (With one r on every mode U tanh(r) U^dagger = tanh(r) I is itself a valid
    state, so the conjugate-transpose plant needs per-mode squeezing to show.)"""
    rng = np.random.default_rng(16)
    m, n, r = 4, 4, 0.7
    U = inputs.haar_unitary(m, rng)
    Pn = oracle.photon_number_prob(m, n, r)
    ru = np.full(m, r)
    D = np.diag(np.tanh(ru))
    assert abs(_n_photon_total(U @ D @ U.T, ru, n) - Pn) < 1e-14
    assert abs(_n_photon_total(U @ D @ U.T, ru, n, with_sfact=False) - Pn) > 1e-3
    assert abs(_n_photon_total(U @ U.T, ru, n) - Pn) > 1e-3
    rv = np.array([0.3, 0.5, 0.7, 0.9])
    Dv = np.diag(np.tanh(rv))
    conv = _single_mode_convolution(rv, n)
    assert abs(_n_photon_total(U @ Dv @ U.T, rv, n) - conv) < 1e-14
    assert abs(_n_photon_total(U @ Dv @ U.conj().T, rv, n) - conv) > 1e-3


# ------------------------------------------------------------------ cancellation statistics


def _rank_one_terms(v):
    """Subset terms of the power-trace formula for A = v v^t in closed form: M_Z = X A_Z has rank one
    with eigenvalue t = v_Z^t X v_Z = 2 sum_{i in Z} v_{2i} v_{2i+1}, so det(I - lambda M_Z)^(-1/2) =
    (1 - lambda t)^(-1/2) and c_k = C(2k, k) / 4^k t^k; the term is (-1)^(k-|Z|) c_k."""
    k = len(v) // 2
    p = np.array([v[2 * i] * v[2 * i + 1] for i in range(k)])
    terms = []
    for Z in range(1, 1 << k):
        idx = [i for i in range(k) if Z >> i & 1]
        t = 2 * p[idx].sum()
        terms.append((-1) ** (k - len(idx)) * math.comb(2 * k, k) / 4 ** k * t ** k)
    return np.array(terms)


@pytest.mark.parametrize("n", [4, 8, 12])
def test_kappa_closed_form_rank_one(n):
    """kappa = sum |t_Z| / |Haf| and kappa2 = sqrt(sum |t_Z|^2) / |Haf| against the rank-one closed form
    of every term (whose sum is (n-1)!! prod v_i)."""
    rng = np.random.default_rng(600 + n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A = np.outer(v, v)
    terms = _rank_one_terms(v)
    haf = dfact(n) * np.prod(v)
    assert abs(terms.sum() - haf) <= 1e-10 * abs(haf)
    for f in (oracle.haf_pt_kappa, oracle.haf_pt_ld_kappa):
        h, kappa, kappa2 = f(A)
        assert abs(h - haf) <= 1e-10 * abs(haf)
        assert abs(kappa - np.abs(terms).sum() / abs(haf)) <= 1e-10 * kappa
        assert abs(kappa2 - np.sqrt((np.abs(terms) ** 2).sum()) / abs(haf)) <= 1e-10 * kappa2


@pytest.mark.parametrize("n", [2, 6, 10, 14])
def test_kappa_invariants(n):
    """kappa >= 1 (triangle inequality), kappa2 <= kappa <= sqrt(N) kappa2 over the N = 2^(n/2) - 1
    subset terms (Cauchy-Schwarz); a single term (n = 2) gives kappa = kappa2 = 1."""
    A = inputs.random_symmetric(n, 1, np.random.default_rng(700 + n))[0]
    h, kappa, kappa2 = oracle.haf_pt_kappa(A)
    N = 2 ** (n // 2) - 1
    assert kappa >= 1 - 1e-12
    assert kappa2 <= kappa * (1 + 1e-12) and kappa <= np.sqrt(N) * kappa2 * (1 + 1e-12)
    if n == 2:
        assert abs(kappa - 1) < 1e-15 and abs(kappa2 - 1) < 1e-15
