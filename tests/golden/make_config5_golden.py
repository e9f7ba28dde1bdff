"""Write config5_haf.json: oracle hafnians of a few large config-5 pattern matrices.

Config 5: m = 60 Haar interferometer (seed 1005), r = 0.88 on every mode, patterns of sizes cycling
36, 40, 44 (pattern seed 2005). The oracle builds B = U diag(tanh r) U^t and the pattern matrices
itself and evaluates the power-trace formula in double (haf_pt) and, where listed, in long double
(haf_pt_ld). Only oracle/ and the seeded input generators are used.

Usage: python tests/golden/make_config5_golden.py [--jobs 8]
Runs for hours on a few cores (n = 44 is ~2^22 subsets with plain repeated multiplication).
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

# (pattern index in config 5, evaluate in long double too)
JOBS = [(0, True), (3, True), (1, False), (4, False), (2, False)]


def one(job):
    idx, with_ld = job
    st, pats = inputs.config5()
    B = oracle.state_B(st.U, st.r)
    p = pats[idx]
    A = oracle.pattern_matrix(B, p)
    t0 = time.time()
    h = oracle.haf_pt(A)
    t1 = time.time()
    rec = {"index": idx, "n": len(p), "modes": [int(v) for v in p], "haf_pt": [h.real, h.imag],
           "seconds_pt": t1 - t0}
    if with_ld:
        hl = oracle.haf_pt_ld(A)
        rec["haf_pt_ld"] = [hl.real, hl.imag]
        rec["seconds_pt_ld"] = time.time() - t1
    print(json.dumps(rec), flush=True)
    return rec


def add_ld(rec):
    """Fill in the long-double value of an existing record."""
    if "haf_pt_ld" in rec:
        return rec
    st, pats = inputs.config5()
    B = oracle.state_B(st.U, st.r)
    A = oracle.pattern_matrix(B, pats[rec["index"]])
    t0 = time.time()
    hl = oracle.haf_pt_ld(A)
    rec = dict(rec, haf_pt_ld=[hl.real, hl.imag], seconds_pt_ld=time.time() - t0)
    print(json.dumps(rec), flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--ld-all", action="store_true", help="add long-double values to an existing file")
    args = ap.parse_args()
    if args.ld_all:
        old = json.loads((HERE / "config5_haf.json").read_text())
        with mp.get_context("fork").Pool(args.jobs) as pool:
            recs = pool.map(add_ld, old["records"], chunksize=1)
    else:
        with mp.get_context("fork").Pool(args.jobs) as pool:
            recs = pool.map(one, JOBS, chunksize=1)
    out = {
        "source": "oracle haf_pt / haf_pt_ld on config-5 pattern matrices (m=60, r=0.88, seeds 1005/2005)",
        "records": sorted(recs, key=lambda r: r["index"]),
    }
    (HERE / "config5_haf.json").write_text(json.dumps(out, indent=1) + "\n")


if __name__ == "__main__":
    main()
