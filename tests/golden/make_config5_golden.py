"""Write config5_haf.json: oracle hafnians of config-5 pattern matrices, with their cancellation kappa.

Config 5: m = 60 Haar interferometer (seed 1005), r = 0.88 on every mode, patterns of sizes cycling
36, 40, 44 (pattern seed 2005; index i has n = (36, 40, 44)[i % 3]). The oracle builds
B = U diag(tanh r) U^t and the pattern matrices itself and evaluates the power-trace formula:
every n = 36 record in long double (haf_pt_ld_kappa), the others in double (haf_pt_kappa; some also
hold a long-double value from an earlier run). Each record carries kappa = sum_Z |term(Z)| / |Haf|
and kappa2 = sqrt(sum_Z |term(Z)|^2) / |Haf|.
Only oracle/ and the seeded input generators are used. Existing records are kept and completed; the
file is rewritten as each record finishes.

Usage: python tests/golden/make_config5_golden.py [--jobs 2] [--all]
Runs for hours (n = 44 is ~2^22 subsets with plain repeated multiplication). --all extends the set
to all 64 patterns (the n = 40 and n = 44 ones in double).
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

import oracle  # noqa: E402
from paper_1908_10070_amd import inputs  # noqa: E402

OUT = HERE / "config5_haf.json"
# every n = 36 matrix, the first six n = 40 ones and the first three n = 44 ones
INDICES = sorted(list(range(0, 64, 3)) + [1, 4, 7, 10, 13, 16] + [2, 5, 8])


def matrix(idx):
    st, pats = inputs.config5()
    B = oracle.state_B(st.U, st.r)
    return pats[idx], oracle.pattern_matrix(B, pats[idx])


def one(job):
    idx, rec = job
    p, A = matrix(idx)
    rec = dict(rec) if rec else {"index": idx, "n": len(p), "modes": [int(v) for v in p]}
    t0 = time.time()
    if len(p) == 36:
        h, kappa, kappa2 = oracle.haf_pt_ld_kappa(A)
        rec["haf_pt_ld"] = [h.real, h.imag]
        rec["seconds_pt_ld"] = time.time() - t0
    else:
        h, kappa, kappa2 = oracle.haf_pt_kappa(A)
        if "haf_pt" in rec:
            assert rec["haf_pt"] == [h.real, h.imag], "double oracle not reproducible"
        rec["haf_pt"] = [h.real, h.imag]
        rec["seconds_pt"] = time.time() - t0
    rec["kappa"] = kappa
    rec["kappa2"] = kappa2
    print(json.dumps(rec), flush=True)
    return rec


def write(recs):
    out = {"source": "oracle haf_pt_kappa / haf_pt_ld_kappa on config-5 pattern matrices "
                     "(m=60, r=0.88, seeds 1005/2005)",
           "records": sorted(recs.values(), key=lambda r: r["index"])}
    tmp = OUT.with_suffix(".tmp")
    tmp.write_text(json.dumps(out, indent=1) + "\n")
    os.replace(tmp, OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=2)
    ap.add_argument("--all", action="store_true", help="all 64 patterns")
    args = ap.parse_args()
    indices = list(range(64)) if args.all else INDICES
    recs = {}
    if OUT.exists():
        recs = {r["index"]: r for r in json.loads(OUT.read_text())["records"]}
    todo = [(i, recs.get(i)) for i in indices if i not in recs or "kappa2" not in recs[i]]
    todo.sort(key=lambda j: -(36, 40, 44)[j[0] % 3])  # longest first
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for rec in pool.imap_unordered(one, todo, chunksize=1):
            recs[rec["index"]] = rec
            write(recs)


if __name__ == "__main__":
    main()
