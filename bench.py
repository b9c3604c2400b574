"""Benchmark: Schroedinger-Feynman path sum on one MI355X.

Default workload: 7x8 grid (56 qubits), depth 1+40+1, vertical cut 28+28
(k = 35 crossing CZs, 2 GiB complex64 block states), one seeded aligned block
of 1024 paths (one GPU's share of the path space, at the shape of the paper's
56-qubit run), 1e6 uniformly random bitstrings.  One "step" is one full
run_paths call over the block with inputs (bitstrings, workspace, output)
already resident in HBM.

Prints one JSON line with paths/s (value), amps/s, the roofline of the
dominant kernel measured with HIP events on the launch stream, the plain
one-path-per-launch GPU form on a subset of paths, the FP64 CPU oracle on a
bounded sample of the same workload, shorter lines for the other
configurations (4x4 FP64 sweeps, 5x6 all paths, a 6x7 sample, the iSWAP
variant), measured bandwidth ceilings, and the serving mix.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid7x8_d40")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-paths", type=int, default=64)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=500, help="jobs in the serving mix (0 = skip)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving mix and print its JSON")
    ap.add_argument("--serve-policies", default="oldest",
                    help="comma-separated scheduling policies of the served runs (oldest, round_robin, least_work)")
    ap.add_argument("--no-sampling", action="store_true", help="skip the rejection-sampling measurement")
    ap.add_argument("--no-iswap", action="store_true", help="skip the iSWAP-variant measurement")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the lines of the other configurations and the bandwidth ceilings")
    ap.add_argument("--bitstrings", type=int, default=0,
                    help="number of requested bitstrings instead of the workload's (amplitude-count scaling)")
    ap.add_argument("--chunk-paths", type=int, default=0,
                    help="split a step into run_paths calls of at most this many paths (accumulated; one progress "
                         "line each), for workloads whose step takes minutes")
    ap.add_argument("--max-paths", type=int, default=0,
                    help="time only the first N paths of the request (a bounded sample, for profiling)")
    ap.add_argument("--tuning", default="",
                    help="fixed tuning R,leaf_batch,waves_per_cu[,dense_qubits[,no_leaf_fold[,fold_levels[,chain_passes[,no_row_skip[,no_defer[,no_chain_merge[,jit[,no_tail_move]]]]]]]]]] "
                         "(skips autotune)")
    ap.add_argument("--no-interpreted", action="store_true",
                    help="with compiled passes (tuning jit), skip timing the same request with interpreted passes "
                         "(profiles then hold the compiled kernels only)")
    ap.add_argument("--ceilings-only", action="store_true",
                    help="only measure the bandwidth ceilings (and the read rate per buffer size) and print them")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (known HBM traffic for counter scaling)")
    return ap.parse_args()


def progress(msg):
    """One line on stderr per phase, so a long run shows it is moving."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def prepare(workload, n_bits=0, max_paths=0, tuning="", autotune=True, n_measure=4, ws_frac=0.85, jit=1):
    """Set up one request the way the benchmark times it: circuit and cut, path ids (all,
    an aligned block or a seeded f-sample), bitstrings, output and workspace resident on the
    device, and the tuning (fixed, autotuned on this request, or the library default).  jit: the
    passes run kernels compiled for their programs (tuning jit; compiled by the first step, which
    the warm-up covers)."""
    import torch
    from paper_1807_10749_amd import binding as sf
    from workload import CONFIGS, make_workload, workload_block

    cfg = CONFIGS[workload]
    w = make_workload(workload, n_bits=n_bits or None)
    gates, bits = w["gates"], w["bitstrings"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    c = sf.Circuit(cfg.rows, cfg.cols, gates, cfg.cut_mask())
    if cfg.paths == "all":
        ids, begin, npaths = None, 0, 1 << c.k
    elif cfg.paths == "block":
        begin, npaths = workload_block(workload)
        ids = None
    else:
        ids = sf.sample_paths(c.k, cfg.f, cfg.path_seed)
        begin, npaths = 0, ids.size
    full_paths = npaths
    if 0 < max_paths < npaths:
        npaths = max_paths
        if ids is not None:
            ids = ids[:npaths]
    flags_base = sf.SF_FP64_SWEEPS if cfg.fp64_sweeps else 0
    d_bits = torch.from_numpy(bits.view(np.int64)).cuda()
    d_amps = torch.zeros(2 * bits.size, dtype=torch.float64, device="cuda")
    # room for every tuning the autotuner may try, materialised leaf states included
    sf.set_tuning(c.handle, no_leaf_fold=1)
    ws_bytes = sf.workspace_size(c.handle, npaths, bits.size, flags_base)
    sf.set_tuning(c.handle)
    free_b, _ = torch.cuda.mem_get_info()
    ws_bytes = max(min(ws_bytes, int(free_b * ws_frac)), 1 << 28)     # run_paths takes at least 256 MiB
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    flags = flags_base | sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    tuned = None
    if tuning:
        vals = [int(v) for v in tuning.split(",")]
        r, lb, wpc = vals[:3]
        dense = vals[3] if len(vals) > 3 else 0
        nofold = vals[4] if len(vals) > 4 else 0
        flev = vals[5] if len(vals) > 5 else 0
        chain = vals[6] if len(vals) > 6 else 0
        sf.set_tuning(c.handle, reg_qubits=r, leaf_batch=lb, waves_per_cu=wpc, dense_qubits=dense,
                      no_leaf_fold=nofold, fold_levels=flev, chain_passes=chain,
                      no_row_skip=vals[7] if len(vals) > 7 else 0, no_defer=vals[8] if len(vals) > 8 else 0,
                      no_chain_merge=vals[9] if len(vals) > 9 else 0, jit=vals[10] if len(vals) > 10 else jit,
                      no_tail_move=vals[11] if len(vals) > 11 else 0)
        tuned = sf.get_tuning(c.handle)
    elif autotune:
        sf.set_tuning(c.handle, jit=jit)
        tuned = sf.autotune(c.handle, ids, begin, npaths, d_bits, bits.size, d_amps, flags, stream, ws, ws_bytes,
                            n_measure=n_measure)
    return {"cfg": cfg, "c": c, "gates": gates, "bits": bits, "ids": ids, "begin": begin, "npaths": npaths,
            "full_paths": full_paths, "d_bits": d_bits, "d_amps": d_amps, "ws": ws, "ws_bytes": ws_bytes,
            "flags": flags, "stream": stream, "tuning": tuned}


def run_step(req, extra=0, chunk_paths=0):
    """One pass over the whole request (in run_paths calls of at most chunk_paths paths,
    accumulated); returns the summed run statistics of its calls."""
    from paper_1807_10749_amd import binding as sf
    c, ids, npaths = req["c"], req["ids"], req["npaths"]
    chunk = chunk_paths if 0 < chunk_paths < npaths else npaths
    tot = None
    for off in range(0, max(npaths, 1), max(chunk, 1)):
        n = min(chunk, npaths - off)
        acc = sf.SF_ACCUMULATE if off else 0
        sf.run_paths(c.handle, None if ids is None else ids[off:off + n], req["begin"] + off if ids is None else 0,
                     n, req["d_bits"], req["bits"].size, req["d_amps"], req["flags"] | extra | acc, req["stream"],
                     req["ws"], req["ws_bytes"])
        st = c.stats()
        tot = st if tot is None else {k: tot[k] + st[k] if k != "a_groups" else st[k] for k in st}
        if chunk < npaths:
            progress(f"  paths {off + n}/{npaths}")
    return tot


def time_steps(req, steps, warmup, chunk_paths=0, label=""):
    """Warm-up steps, then `steps` timed steps bracketed by device synchronisation; per-kernel
    times come from the library's HIP events on the launch stream (SF_TIMING)."""
    import torch
    from paper_1807_10749_amd import binding as sf
    jit_ms = 0.0
    for i in range(warmup):
        progress(f"{label}warm-up step {i + 1}/{warmup}")
        jit_ms += run_step(req, chunk_paths=chunk_paths)["jit_compile_ms"]
    torch.cuda.synchronize()
    keys = ("ms_sweep", "ms_gather", "ms_other", "ms_total", "ms_plan", "n_sweep_launches", "n_gather_launches",
            "sweep_bytes", "gather_bytes", "gather_row_bytes", "n_chained_passes", "n_jit_passes", "jit_compile_ms")
    tot = {k: 0 for k in keys}
    st = None
    t0 = time.perf_counter()
    for i in range(steps):
        progress(f"{label}timed step {i + 1}/{steps}")
        st = run_step(req, sf.SF_TIMING, chunk_paths)
        for k in keys:
            tot[k] += st[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tot["elapsed_s"] = elapsed
    tot["jit_compile_ms_warmup"] = jit_ms
    tot["a_groups"] = st["a_groups"] if st else 0
    tot["gather_ws_bytes"] = st["gather_ws_bytes"] if st else 0
    return tot


def compiled_passes(req, tot, steps, warmup, chunk_paths=0, compare=True):
    """With tuning jit: passes run by kernels compiled for their programs per step, the warm-up's
    compile time, and (compare) the same request timed with interpreted passes (tuning jit = 0)."""
    from paper_1807_10749_amd import binding as sf
    t = req["tuning"]
    if not t or not t.get("jit"):
        return None
    out = {"per_step": tot["n_jit_passes"] / steps, "compile_s_in_warmup": tot["jit_compile_ms_warmup"] / 1e3}
    if not compare:
        return out
    sf.set_tuning(req["c"].handle, **dict(t, jit=0))
    it = time_steps(req, steps, max(warmup, 1), chunk_paths, label="interpreted passes: ")
    sf.set_tuning(req["c"].handle, **t)
    return dict(out, interpreted_ms_per_step=1e3 * it["elapsed_s"] / steps,
                interpreted_ms_sweep_per_step=it["ms_sweep"] / steps)


def dominant(req, tot, steps):
    """The kernel category with the most measured time, its algorithmic bytes per launch and
    average launch duration."""
    from paper_1807_10749_amd import binding as sf
    plan_text = sf.describe_plan(req["c"].handle)
    folded = "folded" in plan_text
    if tot["ms_sweep"] >= tot["ms_gather"]:
        dom, ms, n, by = "pass_kernel (gate sweep)", tot["ms_sweep"], tot["n_sweep_launches"], tot["sweep_bytes"]
    elif folded and "iSWAP gates" in plan_text:
        dom, ms, n, by = ("fold_iswap_kernel (last levels + path sum)", tot["ms_gather"], tot["n_gather_launches"],
                          tot["gather_bytes"])
    elif folded:
        dom, ms, n, by = "fold_kernel (last level + path sum)", tot["ms_gather"], tot["n_gather_launches"], tot["gather_bytes"]
    else:
        dom, ms, n, by = "gather_kernel (path sum)", tot["ms_gather"], tot["n_gather_launches"], tot["gather_bytes"]
    avg_ms = ms / max(n, 1)
    achieved = (by / max(n, 1)) / (avg_ms * 1e-3) / 1e9 if n else 0.0
    return dom, avg_ms, n / steps, by / max(n, 1), achieved


def plain_form(req, n_paths):
    """The plain one-path-per-launch GPU form on the first n_paths paths of the request."""
    import torch
    from paper_1807_10749_amd import binding as sf
    plain_n = min(n_paths, req["npaths"])
    if plain_n <= 0:
        return None
    c, ids = req["c"], req["ids"]
    plain_ids = ids[:plain_n] if ids is not None else None
    args = (req["d_bits"], req["bits"].size, req["d_amps"], req["flags"] | sf.SF_PLAIN, req["stream"], req["ws"],
            req["ws_bytes"])
    sf.run_paths(c.handle, plain_ids, req["begin"], plain_n, *args)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    sf.run_paths(c.handle, plain_ids, req["begin"], plain_n, *args)
    torch.cuda.synchronize()
    return {"paths_per_s": plain_n / (time.perf_counter() - tp), "paths": plain_n}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path sum would shard "
              "aligned path blocks across GPUs with one final reduction, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": x.numel(), "calibrate_copy_bytes_written": y.numel()}))
        return
    from paper_1807_10749_amd import binding as sf
    if args.ceilings_only:
        out = measure_ceilings()
        buf = torch.ones(1 << 32, dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        sweep = {}
        for shift in range(21, 33):
            nbytes = 1 << shift
            reps = max(4, (1 << 36) // nbytes // 4)
            sweep[f"{nbytes >> 20} MiB"] = nbytes * reps / (sf.read_bandwidth(buf, nbytes, reps, 0, stream) * 1e-3) / 1e9
        out["read_GB_per_s_by_buffer_size"] = sweep
        print(json.dumps({"ceilings": out}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(args.serve_jobs, policies=tuple(args.serve_policies.split(",")))}),
              flush=True)
        return

    progress(f"{args.workload}: set-up" + ("" if args.tuning or args.no_autotune else " and autotune"))
    req = prepare(args.workload, n_bits=args.bitstrings, max_paths=args.max_paths, tuning=args.tuning,
                  autotune=not args.no_autotune)
    cfg, c, bits, npaths = req["cfg"], req["c"], req["bits"], req["npaths"]
    n = cfg.n_qubits
    progress(f"{args.workload}: k={c.k}, {npaths} paths, {bits.size} bitstrings, "
             f"workspace {req['ws_bytes'] / 2**30:.1f} GiB, tuning {req['tuning']}")
    tot = time_steps(req, args.steps, args.warmup, args.chunk_paths)
    live_paths = c.stats()["n_paths_live"] if not args.chunk_paths else None
    elapsed = tot["elapsed_s"]
    ms_per_step = 1e3 * elapsed / args.steps
    paths_per_s = npaths * args.steps / elapsed
    amps_per_s = bits.size * args.steps / elapsed
    dom, avg_launch_ms, launches_per_step, bytes_per_launch, achieved = dominant(req, tot, args.steps)
    traffic = measured_traffic(args.workload, dom.split(" ")[0])
    plain = plain_form(req, args.plain_paths)
    if plain:
        plain["speedup_of_batched"] = paths_per_s / plain["paths_per_s"]
    compiled = compiled_passes(req, tot, args.steps, args.warmup, args.chunk_paths, not args.no_interpreted)
    progress("timed steps done")
    # rejection sampling and the validation protocol need the full output distribution: they run
    # on an all-paths request (this one, or the 5x6 line's)
    sampling = None
    if not args.no_sampling and cfg.paths == "all":
        sampling = sampling_bench(c, req["ids"], req["begin"], npaths, bits.size, req["ws"], req["ws_bytes"],
                                  req["stream"])
    validation = None
    if not args.no_sampling and cfg.paths == "all":
        run_step(req)                # exact amplitudes again (the plain-form runs overwrote them)
        torch.cuda.synchronize()
        validation = validation_bench(c, bits, req["d_amps"], cfg.bits_seed, req["ws"], req["ws_bytes"], req["stream"])
    tuning = req["tuning"] or sf.get_tuning(c.handle)
    gates = req["gates"]
    ids, begin = req["ids"], req["begin"]
    run_stats = dict(tot)
    full_paths = req["full_paths"]
    del req
    c_keep = c
    torch.cuda.empty_cache()

    extra = None
    ceilings = None
    if not args.no_extra:
        extra = {}
        progress("bandwidth ceilings")
        ceilings = extra["ceilings"] = measure_ceilings()
        for name in ("grid4x4_d16", "grid5x6_d24", "grid6x7_d32"):
            if name == args.workload:
                continue
            progress(f"extra configuration {name}")
            extra[name] = config_line(name, extra["ceilings"], max_paths=131072 if name == "grid6x7_d32" else 0,
                                      with_sampling=name == "grid5x6_d24" and not args.no_sampling
                                      and sampling is None)
            torch.cuda.empty_cache()
    iswap = None
    if not args.no_iswap and args.workload != "grid5x6_d24_iswap":
        progress("iSWAP variant")
        iswap = iswap_bench(torch.cuda.current_stream())
        torch.cuda.empty_cache()
    serving = None
    if args.serve_jobs > 0:
        progress(f"serving mix, {args.serve_jobs} jobs")
        serving = serving_bench(args.serve_jobs, policies=tuple(args.serve_policies.split(",")))

    # the dominant kernel's roof: HBM for the gate sweeps; for a dominant path sum, the measured
    # read ceiling of the memory level that holds its working set
    if dom.startswith("pass_kernel"):
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    else:
        if ceilings is None:
            progress("bandwidth ceilings")
            ceilings = measure_ceilings()
        roof = gather_roofline(dom, achieved, run_stats["gather_ws_bytes"], ceilings)

    cpu = None
    if not args.no_cpu:
        progress("CPU oracle sample")
        cpu = cpu_baseline(cfg, gates, bits, c_keep.k, ids, begin, npaths, args.cpu_seconds)

    out = {
        "metric": "Feynman paths/s at fidelity f (amps/s, HBM GB/s % peak alongside)",
        "value": paths_per_s,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if cfg.fp64_sweeps else "c64 sweeps, f64 path sum",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": f"{cfg.rows}x{cfg.cols}", "depth": f"1+{cfg.depth}+1",
                   "cut": f"{bin(cfg.cut_mask()).count('1')}+{n - bin(cfg.cut_mask()).count('1')}",
                   "k": c_keep.k, "paths": npaths,
                   "f": cfg.f if cfg.paths == "sample" else npaths / 2.0 ** c_keep.k,
                   "bitstrings": int(bits.size), "tuning": tuning,
                   **({"path_block": [int(begin), int(begin + npaths)]} if cfg.paths == "block" else {}),
                   **({"paths_sample": f"first {npaths} of {full_paths} paths"} if npaths < full_paths else {})},
        "amps_per_s": amps_per_s,
        "live_paths": live_paths,
        "path_amp_contributions_per_s": npaths * bits.size * args.steps / elapsed,
        "plain_form": plain,
        "kernel_ms_per_step": {"sweep": run_stats["ms_sweep"] / args.steps,
                               "gather": run_stats["ms_gather"] / args.steps,
                               "other": run_stats["ms_other"] / args.steps},
        "run_paths_wall_ms_per_step": run_stats["ms_total"] / args.steps,
        "host_plan_ms_per_step": run_stats["ms_plan"] / args.steps,
        "compiled_passes": compiled,
        "roofline": dict(roof, traffic=traffic, avg_launch_ms=avg_launch_ms, launches_per_step=launches_per_step,
                         bytes_per_launch=bytes_per_launch),
        "sweep_roofline": {"kernels": "pass_kernel + dense_kernel (gate sweeps, all levels written)", "bound": "hbm",
                           "achieved": (run_stats["sweep_bytes"] / max(run_stats["ms_sweep"], 1e-9)) / 1e6,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": (run_stats["sweep_bytes"] / max(run_stats["ms_sweep"], 1e-9)) / 1e6 / HBM_PEAK_GBS,
                           "bytes_per_step": run_stats["sweep_bytes"] / args.steps,
                           "launches_per_step": run_stats["n_sweep_launches"] / args.steps,
                           "note": "time of one event pair around each run of sweep launches, gaps included"},
        "gather": {"ms_per_step": run_stats["ms_gather"] / args.steps,
                   "bytes_per_step": run_stats["gather_bytes"] / args.steps,
                   "row_bytes_per_step": run_stats["gather_row_bytes"] / args.steps,
                   "launches_per_step": run_stats["n_gather_launches"] / args.steps},
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "extra": extra,
        "serving": serving,
        "sampling": sampling,
        "validation": validation,
        "iswap": iswap,
    }
    print(json.dumps(out), flush=True)
    c_keep.close()


# The paper's own figures for the closest runs (all on CPUs, single-precision complex): context,
# not targets; the circuits differ (the paper's benchmark files vs the seeded generator here).
PAPER_CONTEXT = {
    "7x8 56q 1+40+1, 28+28 cut, k=35, f=1/196, 1e6 amps": {
        "paths": 175304832, "wall_h": 140.7, "paths_per_s_cluster": 346,
        "paths_per_s_per_process": 0.224,
        "hardware": "625 n1-highmem-32 VMs (Skylake 2.0 GHz, 16 cores each), 4 processes x 8 threads per VM"},
    "5x6 30q 1+26+1, 15+15 cut, k=17, f=1, 1e3 amps": {
        "paths": 131072, "wall_s": 12.95, "paths_per_s": 10121,
        "hardware": "one Xeon Platinum 8124M (18 cores, 72 threads)"},
    "7x6 42q 1+25+1, 24+18 cut, k=18, f=1, 1e6 amps": {
        "paths": 262144, "wall_h": 6.0, "paths_per_s": 12.1, "hardware": "one n1-highcpu-96 VM (48 cores)"},
}


def config_line(name, ceilings, max_paths=0, steps=3, warmup=1, with_sampling=False):
    """A short line for another configuration: paths/s, amps/s and kernel times, autotuned, on
    the whole request or on its first max_paths paths (with_sampling: also rejection sampling and
    the validation protocol on it)."""
    import torch
    req = prepare(name, max_paths=max_paths, n_measure=3)
    tot = time_steps(req, steps, warmup, label=f"{name}: ")
    live = req["c"].stats()["n_paths_live"]
    el = tot["elapsed_s"]
    dom, avg_ms, lps, bpl, ach = dominant(req, tot, steps)
    out = {"paths": req["npaths"], "live_paths": live, "bitstrings": int(req["bits"].size), "k": req["c"].k,
           "paths_per_s": req["npaths"] * steps / el, "amps_per_s": req["bits"].size * steps / el,
           "ms_per_step": 1e3 * el / steps,
           "kernel_ms_per_step": {"sweep": tot["ms_sweep"] / steps, "gather": tot["ms_gather"] / steps,
                                  "other": tot["ms_other"] / steps},
           "dominant": {"kernel": dom, "avg_launch_ms": avg_ms, "launches_per_step": lps,
                        "bytes_per_launch": bpl, "GB_per_s": ach},
           "sweep_launches_per_step": tot["n_sweep_launches"] / steps,
           "chained_passes_per_step": tot["n_chained_passes"] / steps,
           "compiled_passes_per_step": tot["n_jit_passes"] / steps,
           "compile_s_in_warmup": tot["jit_compile_ms_warmup"] / 1e3,
           "sweep_GB_per_s": tot["sweep_bytes"] / max(tot["ms_sweep"], 1e-9) / 1e6,
           "sweep_frac_of_hbm_peak": tot["sweep_bytes"] / max(tot["ms_sweep"], 1e-9) / 1e6 / HBM_PEAK_GBS,
           "tuning": req["tuning"], "dtype": "c128" if req["cfg"].fp64_sweeps else "c64 sweeps, f64 path sum"}
    if req["npaths"] < req["full_paths"]:
        out["paths_sample"] = f"first {req['npaths']} of {req['full_paths']} paths"
    if tot["ms_gather"] > 0:
        # the path sum as path x bitstring contributions per second, and its row reads (each
        # requested bitstring reads one row of both blocks per path, or 2^|S| rows per folded
        # parent) against the measured read ceiling of a cache-resident buffer
        rows = tot["gather_row_bytes"] / steps
        out["gather"] = {"contributions_per_s": req["npaths"] * req["bits"].size / (tot["ms_gather"] / steps * 1e-3),
                         "row_bytes_per_step": rows, "ms_per_step": tot["ms_gather"] / steps,
                         "row_GB_per_s": rows / (tot["ms_gather"] / steps * 1e-3) / 1e9}
        if ceilings and tot["ms_gather"] >= tot["ms_sweep"]:
            out["roofline"] = dict(gather_roofline(dom, ach, tot["gather_ws_bytes"], ceilings),
                                   bytes_per_launch=bpl, avg_launch_ms=avg_ms,
                                   contributions_per_s=out["gather"]["contributions_per_s"])
    if req["tuning"] is not None and tot["n_sweep_launches"] > steps:
        # the same request and tuning with the passes of small tree levels chained into
        # persistent cooperative launches (grid barriers instead of kernel boundaries)
        from paper_1807_10749_amd import binding as sf
        sf.set_tuning(req["c"].handle, **dict(req["tuning"], chain_passes=1))
        ch = time_steps(req, steps, warmup, label=f"{name} chained: ")
        sf.set_tuning(req["c"].handle, **req["tuning"])
        out["chained_passes"] = {"ms_sweep_per_step": ch["ms_sweep"] / steps,
                                 "sweep_launches_per_step": ch["n_sweep_launches"] / steps,
                                 "chained_passes_per_step": ch["n_chained_passes"] / steps,
                                 "ms_per_step": 1e3 * ch["elapsed_s"] / steps}
    if with_sampling:
        c, bits = req["c"], req["bits"]
        out["sampling"] = sampling_bench(c, req["ids"], req["begin"], req["npaths"], bits.size, req["ws"],
                                         req["ws_bytes"], req["stream"])
        run_step(req)               # exact amplitudes again
        torch.cuda.synchronize()
        out["validation"] = validation_bench(c, bits, req["d_amps"], req["cfg"].bits_seed, req["ws"],
                                             req["ws_bytes"], req["stream"])
    req["c"].close()
    del req
    torch.cuda.empty_cache()
    return out


def gather_roofline(dom, achieved, ws, ceilings):
    """Roofline of a dominant path-sum kernel.  Its block-B rows are read at random over the
    block-B state of the level it reads (the working set ws); the smallest level of the memory
    hierarchy that holds it serves the reads, and that level's measured read ceiling is the roof:
    an XCD's 4 MB L2, the 256 MB Infinity Cache, else HBM."""
    level, key = (("l2", "l2_read_GB_per_s") if ws <= 4 << 20 else
                  ("mall", "mall_read_GB_per_s") if ws <= 256 * 10 ** 6 else ("hbm", "hbm_read_GB_per_s"))
    peak = ceilings[key]
    return {"kernel": dom, "bound": level, "achieved": achieved, "peak": peak, "unit": "GB/s", "frac": achieved / peak,
            "peak_kind": f"measured {key.replace('_GB_per_s', '')} ceiling (read_bandwidth)", "working_set_bytes": ws}


def measure_ceilings():
    """Measured bandwidth ceilings on this GPU: a 2 GiB device-to-device copy (HBM read + write,
    torch), and the library's streaming read (read_bandwidth) of buffers sized for each level:
    4 GiB (HBM), 128 MiB (fits the 256 MB Infinity Cache, not an XCD's 4 MB L2) and 2 MiB
    (fits every XCD's L2)."""
    import torch
    from paper_1807_10749_amd import binding as sf
    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    x = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    out["hbm_copy_GB_per_s"] = 2 * x.numel() * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    buf = torch.ones(1 << 32, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for key, nbytes, reps in (("hbm_read_GB_per_s", 1 << 32, 4), ("mall_read_GB_per_s", 1 << 27, 200),
                              ("l2_read_GB_per_s", 1 << 21, 20000)):
        ms = sf.read_bandwidth(buf, nbytes, reps, 0, stream)
        out[key] = nbytes * reps / (ms * 1e-3) / 1e9
    del buf
    torch.cuda.empty_cache()
    out["note"] = ("copy: torch copy_, read + write bytes; reads: the library's read_bandwidth streaming kernel "
                   "(32 workgroups per compute unit less one, 8 loads of 16 B in flight per thread), bytes read "
                   "per second")
    return out


def library_source_sha256():
    """SHA-256 over the library's sources (kernels, planner, executor): the counters of a
    profile hold only while the kernels and the launch plan they were taken on are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1807_10749_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        h.update(name.encode())
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of
    this workload, or None if there is none or the library's sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if library_source_sha256() != rec.get("library_source_sha256"):
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes_per_launch"]


def sampling_bench(c, ids, begin, npaths, n_candidates, ws, ws_bytes, stream, m_prime=10.0, reps=3):
    """Frugal rejection sampling (Algorithm 2) on the benchmark request: n_candidates = l M'
    uniform candidates, their amplitudes over the same paths, acceptance on the device; and the
    acceptance step alone on 1e7 Porter-Thomas-distributed amplitudes resident in HBM."""
    import torch
    from paper_1807_10749_amd import binding as sf
    torch.cuda.synchronize()
    best = None
    for r in range(reps):
        t0 = time.perf_counter()
        out, err = sf.frugal_sample(c.handle, ids, begin, npaths, n_candidates, m_prime, 9000 + r, 9100 + r, 0,
                                    stream, ws, ws_bytes)
        dt = time.perf_counter() - t0
        if best is None or dt < best[0]:
            best = (dt, out.size, err)
    # acceptance step alone: 1e7 candidates
    n = 10_000_000
    t = torch.empty(n, dtype=torch.float64, device="cuda").exponential_(1.0, generator=torch.Generator("cuda").manual_seed(3))
    amps = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    amps[0::2] = torch.sqrt(t / 2.0 ** c.n)
    acc = torch.empty(n, dtype=torch.int32, device="cuda")
    rws = torch.empty(sf.rejection_workspace_size(n), dtype=torch.uint8, device="cuda")
    sf.rejection_accept(amps, n, c.n, m_prime, 1, acc, 0, stream, rws, rws.numel())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for r in range(reps):
        n_acc, _ = sf.rejection_accept(amps, n, c.n, m_prime, 2 + r, acc, 0, stream, rws, rws.numel())
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"m_prime": m_prime, "candidates": n_candidates, "samples": best[1],
            "samples_per_s": best[1] / best[0], "ms": best[0] * 1e3, "batch_error_estimate": best[2],
            "accept_only": {"candidates": n, "ms": ms, "candidates_per_s": n / (ms * 1e-3),
                            "accepted_fraction": n_acc / n,
                            "bytes_per_candidate": 34, "GB_per_s": 34 * n / (ms * 1e-3) / 1e9}}


def validation_bench(c, bits, d_amps, index_seed, ws, ws_bytes, stream, f1=0.25, delta=0.05):
    """The Verifier's side of the validation protocol on the benchmark circuit: the benchmark's
    own exact amplitudes (its bitstrings are the protocol's seeded indices) as the honest claim,
    a fidelity-f1 simulation on the same indices, the overlap estimate and the test."""
    from paper_1807_10749_amd import binding as sf
    if not np.array_equal(sf.sample_bitstrings(c.n, bits.size, index_seed), bits):
        return None
    claim = d_amps.cpu().numpy().view(np.complex128)
    best = None
    for r in range(2):
        t0 = time.perf_counter()
        fe, ok = sf.verify_claim(c.handle, claim, index_seed, f1, 3005 + r, delta, 0, stream, ws, ws_bytes)
        dt = time.perf_counter() - t0
        if best is None or dt < best[0]:
            best = (dt, fe, ok)
    return {"indices": int(bits.size), "f1": f1, "delta": delta, "f_e": best[1], "passed": best[2],
            "ms": best[0] * 1e3}


def iswap_bench(stream, steps=3, warmup=1, jit=1):
    """The harder variant (every CZ of the default circuit an iSWAP, Eq. (4way): four terms and
    two path bits per crossing gate, k = 30): one seeded aligned block of 2^18 paths, 1e5
    bitstrings, autotuned, compiled passes (jit), timed like the headline step."""
    import torch
    from paper_1807_10749_amd import binding as sf
    from workload import make_workload, workload_block
    w = make_workload("grid5x6_d24_iswap")
    cfg, bits = w["cfg"], w["bitstrings"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    begin, npaths = workload_block(cfg.name)
    d_bits = torch.from_numpy(bits.view(np.int64)).cuda()
    d_amps = torch.zeros(2 * bits.size, dtype=torch.float64, device="cuda")
    # the bound assumes every leaf resident at once; the library batches leaves within what it gets
    free_b, _ = torch.cuda.mem_get_info()
    ws_bytes = min(sf.workspace_size(c.handle, npaths, bits.size, 0), 64 << 30, int(free_b * 0.5))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    flags = sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    sf.set_tuning(c.handle, jit=jit)
    tuning = sf.autotune(c.handle, None, begin, npaths, d_bits, bits.size, d_amps, flags, stream, ws, ws_bytes,
                         n_measure=4)
    compile_ms = 0.0
    for _ in range(warmup):
        sf.run_paths(c.handle, None, begin, npaths, d_bits, bits.size, d_amps, flags, stream, ws, ws_bytes)
        compile_ms += c.stats()["jit_compile_ms"]
    torch.cuda.synchronize()
    tot = {"ms_sweep": 0.0, "ms_gather": 0.0, "ms_other": 0.0, "sweep_bytes": 0, "n_sweep_launches": 0}
    t0 = time.perf_counter()
    for _ in range(steps):
        sf.run_paths(c.handle, None, begin, npaths, d_bits, bits.size, d_amps, flags | sf.SF_TIMING, stream, ws,
                     ws_bytes)
        st = c.stats()
        for key in tot:
            tot[key] += st[key]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    sweep_gbs = tot["sweep_bytes"] / (tot["ms_sweep"] * 1e-3) / 1e9 if tot["ms_sweep"] else 0.0
    out = {"workload": cfg.name, "k": c.k, "paths": npaths, "bitstrings": int(bits.size),
           "paths_per_s": npaths / dt, "ms_per_step": dt * 1e3,
           "kernel_ms_per_step": {"sweep": tot["ms_sweep"] / steps, "gather": tot["ms_gather"] / steps,
                                  "other": tot["ms_other"] / steps},
           "sweep_launches_per_step": tot["n_sweep_launches"] / steps,
           "sweep_GB_per_s": sweep_gbs, "sweep_frac_of_hbm_peak": sweep_gbs / HBM_PEAK_GBS,
           "compile_s_in_warmup": compile_ms / 1e3, "tuning": tuning}
    c.close()
    return out


def serving_bench(n_jobs, workers=4, chunk_paths=16384, seed=5005, policies=("oldest",)):
    """Serving mix: Poisson arrivals at 0.7 of the sequential service rate.

    Jobs (grid 4x5..6x6, depth 1+16+1..1+32+1, 1e3..1e5 bitstrings, f in
    {0.01, 0.1, 1}) are served by the library's server (continuous batching over
    `workers` streams, one served run per scheduling policy).  Latency runs from
    the entry to server_submit to the job's completion.  References on the same
    jobs: the batched form run one job at a time (its throughput, and the
    latencies a FIFO queue of those measured run times gives under the submit
    times the served run recorded), and the plain one-path-per-launch form run
    one job at a time (timed on up to 8 paths per job and scaled to the job's
    path count).  A last served run submits every job at once, for the
    throughput of a saturated server.
    """
    import math
    from paper_1807_10749_amd import binding as sf
    from workload import SplitMix64, grid_circuit, random_bitstrings, serving_mix

    pol_id = {"oldest": sf.SF_SERVE_OLDEST_FIRST, "round_robin": sf.SF_SERVE_ROUND_ROBIN,
              "least_work": sf.SF_SERVE_LEAST_WORK}
    specs = serving_mix(n_jobs, seed)
    inputs = []
    for j in specs:
        g = grid_circuit(j["rows"], j["cols"], j["depth"], j["circuit_seed"])
        b = random_bitstrings(j["rows"] * j["cols"], j["n_bits"], j["bits_seed"])
        inputs.append((g, b))
    arena = 32 << 30

    def submit(srv, i):
        j = specs[i]
        g, b = inputs[i]
        return sf.server_submit(srv, j["rows"], j["cols"], g, b, f=j["f"], path_seed=j["path_seed"])

    # one job at a time (batched form): service time from submission to completion
    progress("serving: one job at a time")
    srv = sf.server_create(arena, None, 1, chunk_paths)
    seq_res, seq_t, n_paths = [], [], []
    for i in range(n_jobs):
        jid = submit(srv, i)
        sf.server_drain(srv)
        done, a, info = sf.server_poll(srv, jid, specs[i]["n_bits"])
        seq_res.append(a.copy())
        seq_t.append(info["t_done"] - info["t_submit"])
        n_paths.append(info["n_paths"])
        sf.server_release(srv, jid)
    sf.server_destroy(srv)
    total_paths = sum(n_paths)
    mean_s = sum(seq_t) / n_jobs

    # plain form, one job at a time, timed on a few paths per job
    progress("serving: plain form sample")
    plain_total = 0.0
    for i, j in enumerate(specs):
        g, b = inputs[i]
        c = sf.Circuit(j["rows"], j["cols"], g)
        m = min(8, n_paths[i])
        ids = (np.arange(m, dtype=np.uint64) if j["f"] >= 1 else sf.sample_paths(c.k, j["f"], j["path_seed"])[:m])
        t0 = time.perf_counter()
        c.amplitudes(b, path_ids=ids, flags=sf.SF_PLAIN)
        plain_total += (time.perf_counter() - t0) / m * n_paths[i]
        c.close()

    # served: Poisson arrivals at 0.7 of the sequential service rate
    rate = 0.7 / mean_s
    rng = SplitMix64(seed + 1)
    arrivals, t = [], 0.0
    for _ in range(n_jobs):
        u = ((rng.next() >> 11) + 1) * (1.0 / (1 << 53))
        t += -math.log(u) / rate
        arrivals.append(t)

    def served(arr, policy):
        """Submit job i at arr[i] seconds (all at once when arr is all zeros), drain, and return
        the latencies, submit times, first submit and last completion, the largest relative
        difference from the one-at-a-time results, and the server's counters."""
        srv = sf.server_create(arena, None, workers, chunk_paths)
        sf.server_set_policy(srv, pol_id[policy])
        t0 = time.perf_counter()
        jids = []
        for i in range(n_jobs):
            dt = arr[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            jids.append(submit(srv, i))
        sf.server_drain(srv)
        lat, sub, first, last, dev = [], [], 1e300, 0.0, 0.0
        for i, jid in enumerate(jids):
            done, a, info = sf.server_poll(srv, jid, specs[i]["n_bits"])
            lat.append(info["t_done"] - info["t_submit"])
            sub.append(info["t_submit"])
            first, last = min(first, info["t_submit"]), max(last, info["t_done"])
            ref = seq_res[i]
            dev = max(dev, float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300)))
        st = sf.server_stats(srv)
        sf.server_destroy(srv)
        return lat, sub, first, last, dev, st

    def pct(lat, q):
        s_ = sorted(lat)
        return s_[min(len(s_) - 1, int(math.ceil(q * len(s_))) - 1)]

    def fifo(sub):
        """The one-at-a-time form under the recorded submit times: a FIFO queue whose service
        times are the measured one-at-a-time times of the same jobs."""
        order = sorted(range(n_jobs), key=lambda i: sub[i])
        out, free = [0.0] * n_jobs, 0.0
        for i in order:
            start = max(sub[i], free)
            free = start + seq_t[i]
            out[i] = free - sub[i]
        return out

    res = {"jobs": n_jobs, "workers": workers, "chunk_paths": chunk_paths, "arrival_rate_jobs_per_s": rate,
           "total_paths": total_paths, "sequential_paths_per_s": total_paths / sum(seq_t),
           "sequential_mean_service_ms": 1e3 * mean_s,
           "plain_sequential_paths_per_s": total_paths / plain_total, "plain_extrapolated": True,
           "policies": {}}
    for pol in policies:
        progress(f"serving: Poisson arrivals, policy {pol}")
        lat, sub, first, last, dev, st = served(arrivals, pol)
        ff = fifo(sub)
        res["policies"][pol] = {
            "p50_latency_ms": 1e3 * pct(lat, 0.50), "p99_latency_ms": 1e3 * pct(lat, 0.99),
            "mean_latency_ms": 1e3 * sum(lat) / n_jobs,
            "served_paths_per_s": total_paths / (last - first), "makespan_s": last - first,
            "sequential_fifo_p50_latency_ms": 1e3 * pct(ff, 0.50),
            "sequential_fifo_p99_latency_ms": 1e3 * pct(ff, 0.99),
            "sequential_fifo_mean_latency_ms": 1e3 * sum(ff) / n_jobs,
            "submit_lag_max_ms": 1e3 * max(s_ - a_ for s_, a_ in zip(sub, arrivals)),
            "max_concurrent_chunks": st["max_concurrent_chunks"], "peak_arena_bytes": st["peak_bytes"],
            "alone_vs_mix_max_rel_diff": dev}
    # saturated: every job submitted at once, so the device always has admitted work queued
    progress("serving: saturated")
    sat_lat, _, sat_first, sat_last, sat_dev, sat_st = served([0.0] * n_jobs, policies[0])
    res["saturated"] = {"policy": policies[0], "paths_per_s": total_paths / (sat_last - sat_first),
                        "makespan_s": sat_last - sat_first,
                        "p50_latency_ms": 1e3 * pct(sat_lat, 0.50), "p99_latency_ms": 1e3 * pct(sat_lat, 0.99),
                        "max_concurrent_chunks": sat_st["max_concurrent_chunks"],
                        "alone_vs_mix_max_rel_diff": sat_dev}
    return res


def host_info():
    """CPU model, host threads and RAM of this machine (for the CPU-baseline record)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = 0
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = int(line.split()[1]) * 1024
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_threads": os.cpu_count(), "ram_GiB": round(ram / 2 ** 30, 1)}


def cpu_baseline(cfg, gates, bits, k, ids, begin, npaths, budget_s):
    """The FP64 oracle's path sum on a bounded, time-boxed sample of the same workload.

    Blocks of up to 24 qubits: whole paths (the first ones of the request) over all bitstrings,
    until the budget is spent.  Larger blocks (a single 28-qubit path takes minutes): one path
    of the request run on two prefixes of the gate list (every gate up to cycle 9, and up to
    cycle 17; the path id keeps its bits of the crossing gates in the prefix), each over all
    bitstrings; the first prefix's time plus the remaining gates at the rate between the two
    gives the time of one path."""
    import oracle
    from oracle.build import build
    if not os.path.exists(oracle.lib_path()):
        build()
    q_a = bin(cfg.cut_mask()).count("1")
    q_max = max(q_a, cfg.n_qubits - q_a)
    info = {"cores": oracle.num_threads(), "kind": "oracle", "unit": "paths/s", **host_info()}
    if q_max <= 24:
        chunk = 16
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s and done < npaths:
            m = min(chunk, npaths - done)
            sel = ids[done:done + m] if ids is not None else np.arange(begin + done, begin + done + m, dtype=np.uint64)
            oracle.path_sum(cfg.n_qubits, gates, cfg.cut_mask(), sel, bits)
            done += m
            chunk = min(chunk * 2, 4096)
        el = time.perf_counter() - t0
        return {"value": done / el, **info,
                "sample": f"first {done} of {npaths} paths x all {bits.size} bitstrings, {el:.1f} s"}
    first = int(ids[0]) if ids is not None else int(begin)
    pts = []
    for last_cycle in (9, 17):
        pre = gates[gates["cycle"] <= last_cycle]
        kp = oracle.num_cut(cfg.n_qubits, pre, cfg.cut_mask())
        pid = np.array([first >> (k - kp)], dtype=np.uint64)
        t0 = time.perf_counter()
        oracle.path_sum(cfg.n_qubits, pre, cfg.cut_mask(), pid, bits)
        pts.append((pre.size, time.perf_counter() - t0))
    (g1, t1), (g2, t2) = pts
    # the time of the first prefix (opening H layer, allocation, the final gather) plus the rest of
    # the gates at the rate of cycles 10-17 (a steady mix of one-qubit gates, CZs and projectors)
    rate = (t2 - t1) / max(g2 - g1, 1)
    per_path = t1 + rate * (gates.size - g1)
    return {"value": 1.0 / per_path, **info, "extrapolated": True, "s_per_path": per_path,
            "sample": (f"path {first}: gates of cycles 0-9 ({g1} gates, {t1:.1f} s) and 0-17 ({g2} gates, "
                       f"{t2:.1f} s), all {bits.size} bitstrings; the remaining {gates.size - g1} gates at the "
                       f"rate of cycles 10-17")}


if __name__ == "__main__":
    main()
