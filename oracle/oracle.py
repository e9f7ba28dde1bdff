"""CPU oracle: hafnians and GBS output probabilities -- TEST INFRASTRUCTURE ONLY.

Follows the paper (Wu, Cheng, Zhang, Yung, Sun, "Speedup in classical simulation
of Gaussian boson sampling", arXiv:1908.10070):

* ``haf_enum``   -- Haf(V) as the sum over perfect matchings (Sec. II C, Eq. HafMatch).
* ``haf_pt``     -- the power-trace hafnian formula the paper cites for its
                    O(n^3 2^(n/2)) cost (Sec. II C); ``haf_pt_ld`` in long double.
* ``haf_py``     -- the matching sum in pure Python, for tiny n only.
* ``prob_paper`` -- Eq. ProOri verbatim for identical squeezing r:
                    p(s) = tanh^n r / (s_1!...s_m! cosh^m r) |Haf(W_s)|^2,
                    W = U U^t (Sec. II C) and W_s built by repeating the j-th
                    column and then the j-th row s_j times.
* ``prob_ref``   -- the same probability for per-mode squeezing r_i, read as
                    |Haf(B_x)|^2 / (prod_j s_j! prod_i cosh r_i) with
                    B = U diag(tanh r_i) U^t and B_x(i, j) = B(x_i, x_j) (Sec. III B,
                    the position-sequence matrix W_x, and App. B for its hafnian
                    being that of W_s). Equal to ``prob_paper`` when all r_i agree.
* closed forms  -- single-mode squeezed-state photon statistics |c_s(r)|^2
                    (Sec. II A), the photon-number distribution P_n (Eq. Eqdistribution)
                    and the normalisation f_n (Sec. III B, App. A).
"""
from __future__ import annotations

import ctypes
import itertools
import math
from typing import Iterable, Sequence

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.build()
        lib = ctypes.CDLL(str(path))
        dp = ctypes.POINTER(ctypes.c_double)
        for name in ("orc_haf_enum", "orc_haf_pt", "orc_haf_pt_ld"):
            f = getattr(lib, name)
            f.argtypes = [dp, ctypes.c_int, dp]
            f.restype = ctypes.c_int
        for name in ("orc_haf_enum_batch", "orc_haf_pt_batch", "orc_haf_pt_ld_batch"):
            f = getattr(lib, name)
            f.argtypes = [dp, ctypes.c_int, ctypes.c_long, dp]
            f.restype = ctypes.c_int
        for name in ("orc_haf_pt_kappa", "orc_haf_pt_ld_kappa"):
            f = getattr(lib, name)
            f.argtypes = [dp, ctypes.c_int, dp, dp]
            f.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _as_c128(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    return A


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _call_single(fname: str, A) -> complex:
    A = _as_c128(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    out = np.zeros(2, dtype=np.float64)
    rc = getattr(_lib(), fname)(_ptr(A), n, _ptr(out))
    if rc:
        raise RuntimeError(f"{fname} failed with code {rc} (n={n})")
    return complex(out[0], out[1])


def _call_batch(fname: str, As) -> np.ndarray:
    As = _as_c128(As)
    if As.ndim != 3 or As.shape[1] != As.shape[2]:
        raise ValueError("batch of square matrices expected")
    b, n, _ = As.shape
    out = np.zeros(2 * b, dtype=np.float64)
    rc = getattr(_lib(), fname)(_ptr(As), n, b, _ptr(out))
    if rc:
        raise RuntimeError(f"{fname} failed with code {rc} (n={n})")
    return out.view(np.complex128).copy()


# ------------------------------------------------------------------ hafnians


def haf_enum(A) -> complex:
    """Sum over perfect matchings (Eq. HafMatch); memoised on the remaining set for n <= 24."""
    return _call_single("orc_haf_enum", A)


def haf_enum_batch(As) -> np.ndarray:
    return _call_batch("orc_haf_enum_batch", As)


def haf_pt(A) -> complex:
    """Power-trace formula in double precision (the O(n^3 2^(n/2)) method cited in Sec. II C)."""
    return _call_single("orc_haf_pt", A)


def haf_pt_ld(A) -> complex:
    """Power-trace formula evaluated in long double (64-bit mantissa)."""
    return _call_single("orc_haf_pt_ld", A)


def _call_kappa(fname: str, A):
    A = _as_c128(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    out = np.zeros(2, dtype=np.float64)
    stats = np.zeros(2, dtype=np.float64)
    rc = getattr(_lib(), fname)(_ptr(A), n, _ptr(out), _ptr(stats))
    if rc:
        raise RuntimeError(f"{fname} failed with code {rc} (n={n})")
    h = complex(out[0], out[1])
    if h == 0:
        return h, float("inf"), float("inf")
    return h, float(stats[0]) / abs(h), float(np.sqrt(stats[1])) / abs(h)


def haf_pt_kappa(A):
    """(Haf, kappa, kappa2) by the power-trace formula in double: with t_Z the subset terms,
    kappa = sum_Z |t_Z| / |Haf| is the cancellation of the subset sum (a worst-case rounding error
    of an FP64 evaluation is about kappa u) and kappa2 = sqrt(sum_Z |t_Z|^2) / |Haf| its
    root-sum-square counterpart (the size of independent per-term rounding errors added up)."""
    return _call_kappa("orc_haf_pt_kappa", A)


def haf_pt_ld_kappa(A):
    """(Haf, kappa, kappa2) as haf_pt_kappa, evaluated in long double."""
    return _call_kappa("orc_haf_pt_ld_kappa", A)


def haf_pt_batch(As) -> np.ndarray:
    return _call_batch("orc_haf_pt_batch", As)


def haf_pt_ld_batch(As) -> np.ndarray:
    return _call_batch("orc_haf_pt_ld_batch", As)


def haf_py(A) -> complex:
    """Pure-Python sum over perfect matchings, for n <= 10 (Eq. HafMatch)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    if n % 2:
        return 0j

    def rec(rem: tuple) -> complex:
        if not rem:
            return 1 + 0j
        i, rest = rem[0], rem[1:]
        tot = 0j
        for pos, j in enumerate(rest):
            tot += complex(A[i, j]) * rec(rest[:pos] + rest[pos + 1:])
        return tot

    return rec(tuple(range(n)))


# ------------------------------------------------------------- probabilities


def state_B(U, r) -> np.ndarray:
    """B = U diag(tanh r_i) U^t -- transpose, not conjugate transpose (W = U U^t, Sec. II C)."""
    U = np.asarray(U, dtype=np.complex128)
    r = np.broadcast_to(np.asarray(r, dtype=np.float64), (U.shape[0],))
    return U @ np.diag(np.tanh(r)) @ U.T


def occupation(modes: Sequence[int], m: int) -> np.ndarray:
    """Configuration s = (s_1..s_m) read off a position sequence x (Sec. III B)."""
    s = np.zeros(m, dtype=np.int64)
    for x in modes:
        s[int(x)] += 1
    return s


def pattern_matrix(B: np.ndarray, modes: Sequence[int]) -> np.ndarray:
    """B_x(i, j) = B(x_i, x_j) (Sec. III B)."""
    x = np.asarray(modes, dtype=np.int64)
    return B[np.ix_(x, x)]


def W_s_paper(W: np.ndarray, s: Sequence[int]) -> np.ndarray:
    """W_s as constructed in Sec. II C: s_j copies of column j, then s_j copies of row j."""
    cols = [W[:, j] for j, sj in enumerate(s) for _ in range(sj)]
    Wc = np.stack(cols, axis=1) if cols else np.zeros((W.shape[0], 0), dtype=W.dtype)
    rows = [Wc[j, :] for j, sj in enumerate(s) for _ in range(sj)]
    return np.stack(rows, axis=0) if rows else np.zeros((0, 0), dtype=W.dtype)


def prob_paper(U, r: float, s: Sequence[int], haf=None) -> float:
    """Eq. ProOri for identical squeezing r on all m modes, configuration s."""
    haf = haf or haf_enum
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    W = U @ U.T
    n = int(sum(s))
    Ws = W_s_paper(W, s)
    sfact = math.prod(math.factorial(int(v)) for v in s)
    return math.tanh(r) ** n / (sfact * math.cosh(r) ** m) * abs(haf(Ws)) ** 2


def prob_ref(U, r, modes: Sequence[int], haf=None, B=None) -> float:
    """p = |Haf(B_x)|^2 / (prod_j s_j! prod_i cosh r_i) for one output pattern (mode list x)."""
    haf = haf or haf_enum
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    r = np.broadcast_to(np.asarray(r, dtype=np.float64), (m,))
    if B is None:
        B = state_B(U, r)
    n = len(modes)
    if n % 2:
        return 0.0
    h = haf(pattern_matrix(B, modes)) if n else 1.0
    sfact = math.prod(math.factorial(int(v)) for v in occupation(modes, m))
    return abs(h) ** 2 / (sfact * float(np.prod(np.cosh(r))))


def haf_ref_patterns(U, r, patterns: Iterable[Sequence[int]], haf_batch=None) -> np.ndarray:
    """Hafnians of B_x for many equal-length patterns (batched oracle call)."""
    haf_batch = haf_batch or haf_enum_batch
    B = state_B(U, r)
    pats = np.asarray(list(patterns), dtype=np.int64)
    if pats.shape[1] == 0:
        return np.ones(pats.shape[0], dtype=np.complex128)
    mats = B[pats[:, :, None], pats[:, None, :]]
    return haf_batch(mats)


def prob_ref_patterns(U, r, patterns, haf_batch=None) -> np.ndarray:
    """Probabilities of many equal-length patterns; collisions handled by the s! divisor."""
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    r = np.broadcast_to(np.asarray(r, dtype=np.float64), (m,))
    pats = np.asarray(list(patterns), dtype=np.int64)
    n = pats.shape[1]
    if n % 2:
        return np.zeros(pats.shape[0])
    h = haf_ref_patterns(U, r, pats, haf_batch)
    sfact = np.array([math.prod(math.factorial(int(c)) for c in np.bincount(p, minlength=m)) for p in pats],
                     dtype=np.float64)
    return np.abs(h) ** 2 / (sfact * float(np.prod(np.cosh(r))))


# -------------------------------------------------------------- closed forms


def log_gbinom(a: float, b: int) -> float:
    return math.lgamma(a + 1) - math.lgamma(b + 1) - math.lgamma(a - b + 1)


def gbinom(a: float, b: int) -> float:
    """Binomial coefficient with a Gamma-function top argument (needed for odd m)."""
    return math.exp(log_gbinom(a, b))


def smss_prob(s: int, r: float) -> float:
    """|c_s(r)|^2 of a single-mode squeezed state (Sec. II A); zero for odd s."""
    if s % 2:
        return 0.0
    if s == 0:
        return 1.0 / math.cosh(r)
    log_ratio = math.lgamma(s + 1) - 2 * math.lgamma(s // 2 + 1)  # log(s! / ((s/2)!)^2)
    return math.exp(-math.log(math.cosh(r)) + s * math.log(math.tanh(r) / 2) + log_ratio)


def photon_number_prob(m: int, n: int, r: float) -> float:
    """P_n = C((m+n)/2 - 1, n/2) tanh^n r / cosh^m r for even n, 0 for odd n (Eq. Eqdistribution)."""
    if n % 2:
        return 0.0
    if n == 0:
        return 1.0 / math.cosh(r) ** m
    return math.exp(log_gbinom((m + n) / 2 - 1, n // 2) + n * math.log(math.tanh(r)) - m * math.log(math.cosh(r)))


def f_n(m: int, n: int) -> float:
    """f_n = n! C((m+n)/2 - 1, n/2) (Sec. III B; App. A)."""
    return math.factorial(n) * gbinom((m + n) / 2 - 1, n // 2)


def multisets(m: int, n: int):
    """All configurations with n photons in m modes, as sorted mode lists (with repeats)."""
    return itertools.combinations_with_replacement(range(m), n)


__all__ = [
    "haf_enum", "haf_enum_batch", "haf_pt", "haf_pt_ld", "haf_pt_batch", "haf_pt_ld_batch", "haf_py",
    "haf_pt_kappa", "haf_pt_ld_kappa",
    "state_B", "occupation", "pattern_matrix", "W_s_paper", "prob_paper", "prob_ref",
    "haf_ref_patterns", "prob_ref_patterns", "gbinom", "smss_prob", "photon_number_prob", "f_n",
    "multisets",
]
