"""Write general_haf.json: oracle hafnians of general complex-symmetric matrices, n = 26..46.

Inputs: the config-2 recipe (M = (a + ib)/sqrt(2), a, b ~ N(0, 1), A = (M + M^t)/2), drawn with
inputs.random_symmetric(n, count, default_rng(7000 + n)); record i is matrix i of that draw.
Each value is the oracle's power-trace formula (haf_pt_ld_kappa in long double up to n = 40,
haf_pt_kappa in double above, where long double would take many hours) together with
kappa = sum_Z |term(Z)| / |Haf|, the cancellation of the subset sum, and its root-sum-square
counterpart kappa2 = sqrt(sum_Z |term(Z)|^2) / |Haf|. Only oracle/ and the seeded
input generators are used. The file is rewritten as each record finishes, largest n first.

With --blockdiag it writes blockdiag46_haf.json instead: the n = 46 block-diagonal matrix of two
config-5 pattern matrices (the exact value is the product of the blocks' matching sums) with its kappa.
With --bipartite it writes bipartite_haf.json: the bipartite block matrices [[0, W], [W^t, 0]] of
inputs.bipartite(k, default_rng(300 + k)), k = 17..23 (hafnian = permanent of W), with the same
oracle precisions and kappa, kappa2.

Usage: python tests/golden/make_general_golden.py [--jobs 6] [--nmax 46] [--blockdiag | --bipartite]
n = 46 in double takes a few CPU-hours (2^23 subsets with plain repeated multiplication).
"""
import argparse
import json
import multiprocessing as mp
import os
import pathlib
import sys
import time

HERE = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(HERE.parents[1]))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1908_10070_amd import inputs  # noqa: E402

OUT = HERE / "general_haf.json"
LD_MAX_N = 40


def matrices(n: int, count: int) -> np.ndarray:
    return inputs.random_symmetric(n, count, np.random.default_rng(7000 + n))


def jobs(nmax: int):
    out = []
    for n in range(26, nmax + 1, 2):
        count = 2 if n <= 38 else 1
        out += [(n, i, count) for i in range(count)]
    return sorted(out, key=lambda j: -j[0])


def one(job):
    n, i, count = job
    A = matrices(n, count)[i]
    t0 = time.time()
    if n <= LD_MAX_N:
        h, kappa, kappa2 = oracle.haf_pt_ld_kappa(A)
        prec = "long double"
    else:
        h, kappa, kappa2 = oracle.haf_pt_kappa(A)
        prec = "double"
    rec = {"n": n, "index": i, "count": count, "seed": 7000 + n, "haf": [h.real, h.imag], "kappa": kappa,
           "kappa2": kappa2, "oracle": prec, "seconds": time.time() - t0}
    print(json.dumps(rec), flush=True)
    return rec


def write(recs):
    out = {"source": "oracle haf_pt_ld_kappa (n <= 40) / haf_pt_kappa (n > 40) on "
                     "inputs.random_symmetric(n, count, default_rng(7000 + n))",
           "records": sorted(recs, key=lambda r: (r["n"], r["index"]))}
    tmp = OUT.with_suffix(".tmp")
    tmp.write_text(json.dumps(out, indent=1) + "\n")
    os.replace(tmp, OUT)


def blockdiag46():
    """The n = 46 block-diagonal matrix of two config-5 pattern matrices (sizes 24 and 22, modes from a
    seeded permutation of the 60 modes): its hafnian is the product of the blocks' (matching sums),
    and its kappa (double power trace) sets its error bound."""
    st, _ = inputs.config5()
    B = oracle.state_B(st.U, st.r)
    modes = np.random.default_rng(46).permutation(60)
    A1 = oracle.pattern_matrix(B, sorted(modes[:24]))
    A2 = oracle.pattern_matrix(B, sorted(modes[24:46]))
    A = np.zeros((46, 46), dtype=np.complex128)
    A[:24, :24] = A1
    A[24:, 24:] = A2
    return A, A1, A2


def write_blockdiag():
    A, A1, A2 = blockdiag46()
    t0 = time.time()
    h, kappa, kappa2 = oracle.haf_pt_kappa(A)
    exact = complex(oracle.haf_enum(A1)) * complex(oracle.haf_enum(A2))
    rec = {"n": 46, "haf_pt": [h.real, h.imag], "kappa": kappa, "kappa2": kappa2,
           "haf_blocks": [exact.real, exact.imag], "seconds": time.time() - t0}
    (HERE / "blockdiag46_haf.json").write_text(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec), flush=True)


def one_bipartite(k):
    _, A = inputs.bipartite(k, np.random.default_rng(300 + k))
    n = 2 * k
    t0 = time.time()
    if n <= LD_MAX_N:
        h, kappa, kappa2 = oracle.haf_pt_ld_kappa(A)
        prec = "long double"
    else:
        h, kappa, kappa2 = oracle.haf_pt_kappa(A)
        prec = "double"
    rec = {"k": k, "n": n, "seed": 300 + k, "haf": [h.real, h.imag], "kappa": kappa, "kappa2": kappa2,
           "oracle": prec, "seconds": time.time() - t0}
    print(json.dumps(rec), flush=True)
    return rec


def write_bipartite(jobs_n):
    path = HERE / "bipartite_haf.json"
    recs = json.loads(path.read_text())["records"] if path.exists() else []
    have = {r["k"] for r in recs}
    todo = [k for k in range(23, 16, -1) if k not in have]
    with mp.get_context("fork").Pool(jobs_n) as pool:
        for rec in pool.imap_unordered(one_bipartite, todo, chunksize=1):
            recs.append(rec)
            out = {"source": "oracle haf_pt_ld_kappa (n <= 40) / haf_pt_kappa (n > 40) on "
                             "inputs.bipartite(k, default_rng(300 + k))",
                   "records": sorted(recs, key=lambda r: r["k"])}
            tmp = path.with_suffix(".tmp")
            tmp.write_text(json.dumps(out, indent=1) + "\n")
            os.replace(tmp, path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(6, os.cpu_count() or 1))
    ap.add_argument("--nmax", type=int, default=46)
    ap.add_argument("--blockdiag", action="store_true", help="write blockdiag46_haf.json instead")
    ap.add_argument("--bipartite", action="store_true", help="write bipartite_haf.json instead")
    args = ap.parse_args()
    if args.blockdiag:
        write_blockdiag()
        return
    if args.bipartite:
        write_bipartite(args.jobs)
        return
    recs = []
    if OUT.exists():
        recs = json.loads(OUT.read_text())["records"]
    recs = [r for r in recs if "kappa2" in r]  # records from before kappa2 was stored are redone
    have = {(r["n"], r["index"]) for r in recs}
    todo = [j for j in jobs(args.nmax) if (j[0], j[1]) not in have]
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for rec in pool.imap_unordered(one, todo, chunksize=1):
            recs.append(rec)
            write(recs)


if __name__ == "__main__":
    main()
