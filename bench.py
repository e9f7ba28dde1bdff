"""Benchmark: batched complex128 hafnians on one MI355X, against the per-pattern GPU path and the
CPU oracle, plus the latency of served probability requests.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one haf_batch call over 4096 random complex-symmetric 24x24 matrices (resident in HBM),
i.e. one pass of the whole hot path: planning, staging, the subset engine and the finalize kernel,
replayed from a HIP graph. Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "n=24 complex128 hafnians/s + p50/p99 prob-request latency vs per-pattern path"
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 (matrix and vector)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_haf_batch_n24_b4096.json")


def kernel_source_hash() -> str:
    """Hash of the device sources; counter-derived traffic is reported only for the kernels it was
    measured on."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1908_10070_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(chunk_small, chunk_large, shape):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, or None when the
    summary is missing or was taken on other kernel sources or another launch shape."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    if (t.get("chunk_small"), t.get("chunk_large"), t.get("engine_shape")) != (chunk_small, chunk_large, shape):
        return None
    return t.get("hbm_bytes_per_launch")


def _oracle_worker(args):
    import oracle
    mats, = args
    t0 = time.perf_counter()
    vals = [oracle.haf_pt(a) for a in mats]
    return time.perf_counter() - t0, vals


def host_info():
    """Core count and CPU model of this host (the oracle's baseline runs here)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "host_cores": os.cpu_count() or 1, "usable_cores": usable}


def cpu_baseline(A, n_per_core=12, max_cores=16):
    """The oracle's power-trace hafnian (plain C, -O2, one matrix per call) timed on the host cores over
    a bounded sample, plus a one-core rate. Returns (record, oracle values of the sample)."""
    import multiprocessing as mp
    info = host_info()
    # worker processes: all usable cores, at most max_cores (the GPU machine grants 16 per GPU)
    cores = max(1, min(max_cores, info["usable_cores"]))
    sample = A[: cores * n_per_core]
    idx = [list(range(i, len(sample), cores)) for i in range(cores)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(sample[ix],) for ix in idx])
    wall = time.perf_counter() - t0
    vals = np.zeros(len(sample), dtype=np.complex128)
    for ix, (_, v) in zip(idx, res):
        vals[ix] = v
    one_t, _ = _oracle_worker((A[:n_per_core],))
    rec = {"value": len(sample) / wall, "unit": "hafnians/s", "cores": cores, "kind": "oracle",
           "one_core_value": n_per_core / one_t,
           "sample": f"oracle haf_pt (FP64 power trace, plain C at -O2, no SIMD or threads inside) on the first "
                     f"{len(sample)} of the 4096 matrices, {cores} worker processes, {wall:.1f} s wall; one-core "
                     f"rate from the first {n_per_core} on one process",
           **info}
    return rec, vals


def rel_errs(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return np.abs(x - ref) / np.maximum(np.abs(ref), 1e-300)


def _timed(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _kappa_bound(n, kappa, double_ref):
    """n^2 u kappa: the stated FP64 error bound where the subset sum cancels by kappa (the worst case
    with kappa = sum |term| / |Haf|; the root-sum-square kappa2 gives the typical size). Doubled when
    the reference is itself a double-precision power trace."""
    return n * n * kappa * 2.0 ** -53 * (2.0 if double_ref else 1.0)


def config5_extra(gbs, torch, dev, ctx):
    """Config 5: 64 B_S matrices of n = 36/40/44 (m = 60, r = 0.88), one gbs_prob_batch call, against the
    stored oracle values (with kappa) of the ones that have them."""
    import pathlib
    from paper_1908_10070_amd import inputs
    st_in, pats = inputs.config5()
    st = ctx.state(torch.from_numpy(st_in.U).to(dev), st_in.r)
    prob = torch.empty(len(pats), dtype=torch.float64, device=dev)
    haf = torch.empty(len(pats), dtype=torch.complex128, device=dev)
    ctx.prob_batch(st, pats, prob_out=prob, haf_out=haf)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.prob_batch(st, pats, prob_out=prob, haf_out=haf)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flops = sum(gbs.haf_flops(len(p)) for p in pats)
    out = {"hafnians": len(pats), "seconds": dt, "hafnians_per_s": len(pats) / dt, "tflops": flops / dt / 1e12,
           "frac_fp64_peak": flops / dt / 1e12 / FP64_PEAK_TFLOPS}
    gold = ROOT + "/tests/golden/config5_haf.json"
    try:
        recs = json.loads(pathlib.Path(gold).read_text())["records"]
    except (OSError, ValueError):
        recs = []
    h = haf.cpu().numpy()
    rows = []
    for r in recs:
        ld = "haf_pt_ld" in r
        ref = complex(*(r["haf_pt_ld"] if ld else r["haf_pt"]))
        e = float(rel_errs(h[r["index"]], ref))
        row = {"index": r["index"], "n": r["n"], "rel_err": e, "ref": "long double" if ld else "double"}
        if "kappa" in r:
            row["kappa"] = r["kappa"]
            row["err_over_kappa_u"] = e / (r["kappa"] * 2.0 ** -53)
            row["within_n2_kappa_u"] = e <= _kappa_bound(r["n"], r["kappa"], not ld)
        if "kappa2" in r:
            row["kappa2"] = r["kappa2"]
            row["err_over_kappa2_u"] = e / (r["kappa2"] * 2.0 ** -53)
            row["within_n2_kappa2_u"] = e <= _kappa_bound(r["n"], r["kappa2"], not ld)
        rows.append(row)
    out["vs_oracle"] = rows
    out["max_rel_err"] = max((r["rel_err"] for r in rows), default=None)
    out["double_double"] = config5_dd(gbs, torch, dev, ctx, st_in, pats, h, recs)
    return out


def config5_dd(gbs, torch, dev, ctx, st_in, pats, h_fp64, recs, sample=6):
    """The double-double accuracy mode on the first `sample` config-5 patterns (two each of n = 36, 40,
    44): its time against FP64 on the same patterns, its error against the stored oracle values, and
    how far the FP64 results lie from it."""
    sel = [list(map(int, p)) for p in pats[:sample]]
    c = gbs.Context(0)
    c.set_precision("dd")
    st = c.state(torch.from_numpy(st_in.U).to(dev), st_in.r)
    haf = torch.empty(len(sel), dtype=torch.complex128, device=dev)
    c.prob_batch(st, [sel[0][:4]], want_haf=True)  # plan and graph machinery warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.prob_batch(st, sel, haf_out=haf)
    torch.cuda.synchronize()
    t_dd = time.perf_counter() - t0
    st64 = ctx.state(torch.from_numpy(st_in.U).to(dev), st_in.r)
    t_fp = _timed(lambda: ctx.prob_batch(st64, sel), reps=2)
    hd = haf.cpu().numpy()
    rows = []
    for r in recs:
        if r["index"] >= sample:
            continue
        ld = "haf_pt_ld" in r
        ref = complex(*(r["haf_pt_ld"] if ld else r["haf_pt"]))
        rows.append({"index": r["index"], "n": r["n"], "ref": "long double" if ld else "double",
                     "dd_rel_err": float(rel_errs(hd[r["index"]], ref)),
                     "fp64_rel_err": float(rel_errs(h_fp64[r["index"]], ref))})
    return {"patterns": sample, "ns": [len(p) for p in sel], "seconds": t_dd, "fp64_seconds": t_fp,
            "cost_factor": t_dd / t_fp, "vs_oracle": rows,
            "max_fp64_vs_dd": float(np.max(rel_errs(h_fp64[:sample], hd))),
            "note": "gbs_ctx_set_precision(GBS_PREC_DD): double-double subset sum on the VALU; the oracle "
                    "values' own error (long double, n^2 2^-64 kappa2) bounds what dd_rel_err can show"}


def extras(gbs, torch, dev, args):
    """Probability throughput (configs 1, 3, 5) with oracle errors, and served-request latency (config 4)."""
    import oracle
    from paper_1908_10070_amd import inputs, serve

    out = {}
    ctx = gbs.Context(0)
    # config 1: m = 16, all 12,870 eight-photon patterns plus the vacuum
    st1_in, pats1 = inputs.config1()
    st1 = ctx.state(torch.from_numpy(st1_in.U).to(dev), st1_in.r)
    from paper_1908_10070_amd.gbs import pack_patterns
    allp = pack_patterns([[]] + [list(p) for p in pats1])  # the vacuum and every 8-photon pattern
    t = _timed(lambda: ctx.prob_batch(st1, allp))
    p1 = ctx.prob_batch(st1, allp).cpu().numpy()
    sel = np.linspace(0, len(pats1) - 1, 64).astype(int)
    ref1 = oracle.prob_ref_patterns(st1_in.U, st1_in.r, pats1[sel])
    out["config1"] = {"probs_per_s": (len(pats1) + 1) / t, "ms": t * 1e3, "patterns": int(len(pats1) + 1),
                      "max_rel_err": float(np.max(rel_errs(p1[1 + sel], ref1))), "err_sample": len(sel)}
    # config 3: m = 50, r = 0.88, 100,000 twenty-photon patterns
    st3_in, pats3 = inputs.config3()
    st3 = ctx.state(torch.from_numpy(st3_in.U).to(dev), st3_in.r)
    prob = torch.empty(len(pats3), dtype=torch.float64, device=dev)
    t = _timed(lambda: ctx.prob_batch(st3, pats3, prob_out=prob))
    f20 = gbs.haf_flops(20)
    sel = np.linspace(0, len(pats3) - 1, 48).astype(int)
    ref3 = oracle.prob_ref_patterns(st3_in.U, st3_in.r, pats3[sel])
    out["config3"] = {"probs_per_s": len(pats3) / t, "ms": t * 1e3, "patterns": int(len(pats3)),
                      "tflops": f20 * len(pats3) / t / 1e12, "frac_fp64_peak": f20 * len(pats3) / t / 1e12 / FP64_PEAK_TFLOPS,
                      "max_rel_err": float(np.max(rel_errs(prob.cpu().numpy()[sel], ref3))), "err_sample": len(sel)}
    # the whole config-1 output space with stored sub-hafnians (App. D) and the brute-force sampler (App. I)
    t_cf = _timed(lambda: ctx.prob_sweep(st1, 8, collisions=False))
    p_all = ctx.prob_sweep(st1, 8, collisions=True)
    t_all = _timed(lambda: ctx.prob_sweep(st1, 8, collisions=True, prob_out=p_all))
    u = torch.from_numpy(np.random.default_rng(6).random(1 << 20)).to(dev)
    t_smp = _timed(lambda: ctx.sweep_sample(p_all, u))
    _, tot = ctx.sweep_sample(p_all, u)
    out["config1_sweep"] = {
        "collision_free_patterns": int(len(pats1)), "collision_free_ms": t_cf * 1e3,
        "speedup_vs_batched_power_trace": out["config1"]["ms"] / (t_cf * 1e3),
        "all_configurations": int(p_all.numel()), "all_configurations_ms": t_all * 1e3,
        "total_probability": float(tot.cpu()[0]), "P8_closed_form": 0.1004360452105159,
        "sampler_draws": int(u.numel()), "sampler_ms": t_smp * 1e3,
        "note": "gbs_prob_sweep (every n-photon pattern, hafnians from stored sub-hafnians) and gbs_sweep_sample "
                "(prefix sum + binary search over all 490,314 configurations)"}
    if not args.no_config5:
        out["config5"] = config5_extra(gbs, torch, dev, ctx)
    # config 4: served mixed stream on the config-3 state
    nreq, warm = args.serve_requests, args.serve_warmup
    mix_rng = np.random.default_rng(3004)
    mix = [inputs.collision_free_patterns(50, int(2 * mix_rng.integers(4, 17)), 1, mix_rng)[0] for _ in range(2000)]
    cap_ctx = gbs.Context(0)
    cap_ctx.set_streams(args.serve_streams)
    t = _timed(lambda: cap_ctx.prob_batch(st3, mix), reps=2)
    capacity = len(mix) / t
    srv_out = {"batched_capacity_req_s": capacity,
               "streams_per_step": args.serve_streams,
               "note": "capacity = 2000 mixed requests in one gbs_prob_batch call; latency = scheduled arrival to "
                       "result on the host; statistics over the requests after the warm-up ones; Python's cyclic "
                       "garbage collector is held off during both servers' streams (serve.hold_gc)"}
    for load in args.serve_loads:
        rate = load * capacity
        arr, pats = inputs.config4_requests(nreq + warm, rate)
        # every step has a new shape, so the server's context captures no graphs (nothing to replay)
        sctx = gbs.Context(0, use_graph=False)
        be = serve.GpuBackend(sctx, st3, pool_entries=1 << 16, lanes=1, streams_per_call=args.serve_streams)
        be.warmup(range(8, 33, 2))
        cont = serve.Server(be, pool_entries=1 << 16, step_flops=args.step_flops, max_slice=4096,
                            hold_gc=True, adaptive=not args.serve_fixed_budget).start()
        serve.replay(cont, arr, pats)
        cont.stop(timeout=600)
        lat_c = np.array(cont.latencies_by_rid(warm)) * 1e3
        res = {"arrival_rate_req_s": rate, "requests": nreq, "warmup_requests": warm,
               "continuous": {"p50_ms": float(np.percentile(lat_c, 50)), "p99_ms": float(np.percentile(lat_c, 99)),
                              "mean_ms": float(lat_c.mean()), "throughput_req_s": cont.completion_rate(warm),
                              "steps": cont.steps,
                              "host_ms_per_step": {k: v for k, v in cont.stats().items() if k.startswith("host_")}}}
        if not args.no_fifo:
            pp = gbs.Context(0, use_graph=False, persistent=False)
            for n in range(8, 33, 2):  # load every kernel the stream uses
                pp.prob_batch(st3, [list(range(n))])
            torch.cuda.synchronize()
            fifo = serve.FifoServer(pp, st3).start()
            serve.hold_gc()
            serve.replay(fifo, arr, pats)
            fifo.stop(timeout=900)
            serve.release_gc()
            lat_f = np.array(fifo.latencies_by_rid(warm)) * 1e3
            res["fifo_per_pattern"] = {"p50_ms": float(np.percentile(lat_f, 50)),
                                       "p99_ms": float(np.percentile(lat_f, 99)), "mean_ms": float(lat_f.mean()),
                                       "throughput_req_s": fifo.completion_rate(warm)}
        srv_out[f"load_{load}"] = res
    out["config4_serving"] = srv_out
    if not args.no_sampler:
        # chain-rule sampler (Theorem-1 marginals) at the paper's mode count m = n^2, r = 0.88
        from paper_1908_10070_amd import sampler
        smp_out = {}
        for n_ph, count in ((12, 8), (16, 2), (18, 1)):
            m_s = n_ph * n_ph
            U_s = inputs.haar_unitary(m_s, np.random.default_rng(4000 + n_ph))
            st_s = ctx.state(torch.from_numpy(U_s).to(dev), np.full(m_s, 0.88))
            smp = sampler.Sampler(ctx, st_s, m_s, 0.88)
            srng = np.random.default_rng(5)
            smp.positions(min(n_ph, 8), 1, srng)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            smp.positions(n_ph, count, srng)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            smp_out[f"n{n_ph}_m{m_s}"] = {"seconds_per_sample": dt / count, "samples": count}
        smp_out["context"] = ("paper (CPU, other hardware): 18 photons about 20 h on a laptop; 20 photons about "
                              "36 h on a 256-core server")
        out["sampler"] = smp_out
    return out


def run_config3(args):
    """--workload config3 / config5: only that probability batch (config 3: m = 50, r = 0.88, 100,000
    twenty-photon patterns; config 5: m = 60, r = 0.88, 64 patterns of n = 36/40/44), one
    gbs_prob_batch call per step, timed like the headline; for profiling those paths."""
    import torch
    from paper_1908_10070_amd import gbs, inputs
    dev = torch.device("cuda", 0)
    ctx = gbs.Context(0)
    if args.streams:
        ctx.set_streams(args.streams)
    c5 = args.workload == "config5"
    st_in, pats = inputs.config5() if c5 else inputs.config3()
    st = ctx.state(torch.from_numpy(st_in.U).to(dev), st_in.r)
    from paper_1908_10070_amd.gbs import pack_patterns
    packed = pack_patterns(pats)
    prob = torch.empty(len(pats), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        ctx.prob_batch(st, packed, prob_out=prob)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.prob_batch(st, packed, prob_out=prob)
        e1.record(stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = [a.elapsed_time(b) for a, b in evs]
    kern_ms = float(np.mean(gpu_ms))
    flops = sum(gbs.haf_flops(len(p)) for p in pats)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    name = "config5" if c5 else "config3"
    print(json.dumps({
        "metric": f"{name} probabilities/s", "value": len(pats) / (wall / args.steps), "unit": "probabilities/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "complex128", "data": "synthetic",
        "config": {"workload": ("config5: m = 60, r = 0.88, 64 patterns of n = 36/40/44 (seeds 1005/2005)" if c5 else
                                "config3: m = 50, r = 0.88, 100,000 collision-free 20-photon patterns (seeds 1003/2003)")
                               + ", gbs_prob_batch"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "flops_per_launch": flops,
                     "kernel_ms": kern_ms, "kernel_ms_min": float(np.min(gpu_ms))}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-per-pattern", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the probability and serving measurements")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-warmup", type=int, default=1000)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.8],
                    help="arrival rates as fractions of the measured batched capacity")
    ap.add_argument("--step-flops", type=float, default=1.6e12, help="modelled work per server step")
    ap.add_argument("--no-fifo", action="store_true", help="skip the FIFO per-pattern server")
    ap.add_argument("--streams", type=int, default=0,
                    help="streams of the headline context (gbs_ctx_set_streams; 0 = the library's default)")
    ap.add_argument("--serve-streams", type=int, default=4,
                    help="streams a mixed batch's kernels are spread over (gbs_ctx_set_streams), for the batched "
                         "capacity and each server step")
    ap.add_argument("--serve-fixed-budget", action="store_true",
                    help="server steps of --step-flops only (no growth with the backlog)")
    ap.add_argument("--no-config5", action="store_true")
    ap.add_argument("--no-sampler", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner here instead of using the built-in table (which is its output)")
    ap.add_argument("--no-tune", action="store_true", help="the built-in launch-shape table (the default)")
    ap.add_argument("--chunks", type=str, default="",
                    help="fixed chunk sizes 'small,large' instead of tuning (profiling runs)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM traffic counters)")
    ap.add_argument("--workload", choices=("config2", "config3", "config5"), default="config2",
                    help="config3 / config5: time only that probability batch (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload in ("config3", "config5"):
        run_config3(args)
        return

    from paper_1908_10070_amd import inputs

    n, batch = 24, 4096
    A_host = inputs.config2(batch=batch, n=n)
    # The CPU leg runs first, in worker processes forked before anything touches the GPU; its oracle
    # values of the sampled matrices also check the timed run's output.
    cpu, cpu_vals = (None, None) if args.no_cpu else cpu_baseline(A_host)

    import torch
    from paper_1908_10070_amd import gbs

    dev = torch.device("cuda", 0)
    A = torch.from_numpy(A_host).to(dev)
    out = torch.empty(batch, dtype=torch.complex128, device=dev)
    if args.copy_calib_mib:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = gbs.Context(0, use_graph=True, persistent=True)
    if args.streams:
        ctx.set_streams(args.streams)
    stream = torch.cuda.current_stream()
    # launch shape: the built-in table (the autotuner's output for every n), or tuned here with --tune
    from paper_1908_10070_amd import autotune
    tune_log = []
    if args.chunks:
        cs, cl = (int(v) for v in args.chunks.split(","))
        ctx.set_tuning(n, cs, cl)
        chunks = ctx.get_tuning(n)
    elif args.tune:
        chunks = autotune.tune(ctx, n, A, reps=1, small=(256, 512, 1024, 2048), large=(64, 128, 256, 512),
                               cache=None, log=tune_log)
    else:
        chunks = ctx.get_tuning(n)
    shape = ctx.get_shape(n)

    for _ in range(args.warmup):
        ctx.haf_batch(A, out=out)
    torch.cuda.synchronize()
    # no cyclic-GC pause inside the timed region (it would stall the host that feeds the device)
    import gc
    gc.collect()
    gc.disable()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.haf_batch(A, out=out)
        e1.record(stream)
        step_ms.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    gpu_ms = [a.elapsed_time(b) for a, b in step_ms]
    ms_per_step = wall * 1e3 / args.steps
    value = batch / (wall / args.steps)

    flops_per_haf = gbs.haf_flops(n)
    kern_ms = float(np.mean(gpu_ms))
    achieved = flops_per_haf * batch / (kern_ms * 1e-3) / 1e12

    # error of the timed run's output against the oracle (the CPU leg's sample; else a small one)
    h_timed = out.cpu().numpy()
    if cpu_vals is None:
        import oracle
        cpu_vals = np.array([oracle.haf_pt(a) for a in A_host[:16]])
    errs = rel_errs(h_timed[: len(cpu_vals)], cpu_vals)

    res = {
        "metric": METRIC, "value": value, "unit": "hafnians/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "complex128", "data": "synthetic",
        "config": {"workload": "config2: 4096 random complex-symmetric 24x24 matrices (seed 1002), haf_batch, "
                               "persistent launch replayed from a HIP graph", "n": n, "batch": batch,
                   "chunk_small": int(chunks[0]), "chunk_large": int(chunks[1]), "engine_shape": int(shape),
                   "streams": ctx.streams,
                   "launch_shape_from": "chunks given" if args.chunks else ("autotuned here" if args.tune else
                                                                             "built-in table (autotuner output)")},
        "max_rel_err": float(errs.max()), "median_rel_err": float(np.median(errs)),
        "err_sample": f"timed run's output of the first {len(cpu_vals)} matrices vs the oracle's haf_pt (FP64 power "
                      f"trace); the stated tolerance is 1e-9",
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(int(chunks[0]), int(chunks[1]),
                                                                                       int(shape)),
                     "flops_per_launch": flops_per_haf * batch, "kernel_ms": kern_ms,
                     "kernel_ms_median": float(np.median(gpu_ms)), "kernel_ms_min": float(np.min(gpu_ms)),
                     "kernel_ms_max": float(np.max(gpu_ms)),
                     "algorithmic_bytes_per_launch": batch * n * n * 16 + batch * 16},
    }

    if not args.no_per_pattern:
        pp = gbs.Context(0, use_graph=False, persistent=False)
        cnt = 256
        for i in range(4):
            pp.haf_batch(A[i:i + 1], out=out[i:i + 1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(cnt):
            pp.haf_batch(A[i:i + 1], out=out[i:i + 1])
        torch.cuda.synchronize()
        pp_rate = cnt / (time.perf_counter() - t1)
        res["per_pattern"] = {"value": pp_rate, "unit": "hafnians/s", "sample": f"{cnt} one-launch-per-matrix calls",
                              "speedup_batched": value / pp_rate}

    if cpu is not None:
        res["cpu_baseline"] = cpu

    if not args.no_extras:
        res["extras"] = extras(gbs, torch, dev, args)

    print(json.dumps(res))


if __name__ == "__main__":
    main()
