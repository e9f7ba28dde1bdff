"""Error bounds of FP64 power-trace hafnians against stored oracle values.

With t_Z the subset terms (Haf = sum_Z t_Z), one term's first-order rounding error is at most about
n^2 u |t_Z| (u = 2^-53): k = n/2 chained products of inner length d <= n, then the k-step coefficient
recursion, (k d + k^2) u <= n^2 u. Summed over the terms:

* worst case, every error aligned:  |err| / |Haf| <= n^2 u kappa,   kappa = sum_Z |t_Z| / |Haf|;
* independent errors (the probabilistic analysis of rounding, in which sums of m rounding errors
  grow like sqrt(m) rather than m):  |err| / |Haf| <~ n^2 u kappa2,   kappa2 = sqrt(sum_Z |t_Z|^2) / |Haf|.

kappa and kappa2 come with every stored value (oracle haf_pt_kappa / haf_pt_ld_kappa). Against a
double-precision oracle value both sides round, so the bound doubles; a long-double value's own
error is negligible.
"""
U53 = 2.0 ** -53


def worst_case_bound(n, kappa, oracle_prec="long double"):
    return n * n * U53 * kappa * (2.0 if oracle_prec == "double" else 1.0)


def rss_bound(n, kappa2, oracle_prec="long double"):
    return n * n * U53 * kappa2 * (2.0 if oracle_prec == "double" else 1.0)


def bound(n, rec_kappa, rec_kappa2=None, oracle_prec="long double"):
    """The tighter of the two bounds available for a stored value."""
    b = worst_case_bound(n, rec_kappa, oracle_prec)
    if rec_kappa2 is not None:
        b = min(b, rss_bound(n, rec_kappa2, oracle_prec))
    return b
