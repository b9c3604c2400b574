"""Benchmark: Schroedinger-Feynman path sum on one MI355X.

Default workload: 5x6 grid (30 qubits), depth 1+24+1, vertical cut 15+15
(k = 15 crossing CZs), all 2^15 paths (f = 1), 1e5 uniformly random
bitstrings.  One "step" is one full run_paths call over all paths with
inputs (bitstrings, workspace, output) already resident in HBM.

Prints one JSON line with paths/s (value), amps/s, the roofline of the
dominant kernel measured with HIP events on the launch stream, the plain
one-path-per-launch GPU form on a subset of paths, and the FP64 CPU oracle
on a bounded sample of the same workload.
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid5x6_d24")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-paths", type=int, default=64)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=24, help="jobs in the serving mix (0 = skip)")
    ap.add_argument("--no-sampling", action="store_true", help="skip the rejection-sampling measurement")
    ap.add_argument("--no-iswap", action="store_true", help="skip the iSWAP-variant measurement")
    ap.add_argument("--bitstrings", type=int, default=0,
                    help="number of requested bitstrings instead of the workload's (amplitude-count scaling)")
    ap.add_argument("--chunk-paths", type=int, default=0,
                    help="split a step into run_paths calls of at most this many paths (accumulated; one progress "
                         "line each), for workloads whose step takes minutes")
    ap.add_argument("--max-paths", type=int, default=0,
                    help="time only the first N paths of the request (a bounded sample, for profiling)")
    ap.add_argument("--tuning", default="",
                    help="fixed tuning R,leaf_batch,waves_per_cu[,dense_qubits[,no_leaf_fold[,fold_levels]]] "
                         "(skips autotune)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (known HBM traffic for counter scaling)")
    return ap.parse_args()


def progress(msg):
    """One line on stderr per phase, so a long run shows it is moving."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


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
    from workload import CONFIGS, make_workload, path_block

    cfg = CONFIGS[args.workload]
    w = make_workload(args.workload, n_bits=args.bitstrings or None)
    gates, bits = w["gates"], w["bitstrings"]
    n = cfg.n_qubits
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    c = sf.Circuit(cfg.rows, cfg.cols, gates, cfg.cut_mask())
    if cfg.paths == "all":
        ids, begin, npaths = None, 0, 1 << c.k
    elif cfg.paths == "block":
        begin, npaths = path_block(c.k, cfg.block_bits, cfg.path_seed)
        ids = None
    else:
        ids = sf.sample_paths(c.k, cfg.f, cfg.path_seed)
        begin, npaths = 0, ids.size
    full_paths = npaths
    if 0 < args.max_paths < npaths:
        npaths = args.max_paths
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
    ws_bytes = min(ws_bytes, int(free_b * 0.85))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    flags = flags_base | sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE

    def step(extra=0):
        """One pass over the whole request; returns the summed run statistics of its calls."""
        chunk = args.chunk_paths if 0 < args.chunk_paths < npaths else npaths
        tot = None
        for off in range(0, max(npaths, 1), max(chunk, 1)):
            n = min(chunk, npaths - off)
            acc = sf.SF_ACCUMULATE if off else 0
            if ids is not None:
                sf.run_paths(c.handle, ids[off:off + n], 0, n, d_bits, bits.size, d_amps, flags | extra | acc, stream,
                             ws, ws_bytes)
            else:
                sf.run_paths(c.handle, None, begin + off, n, d_bits, bits.size, d_amps, flags | extra | acc, stream,
                             ws, ws_bytes)
            st = c.stats()
            tot = st if tot is None else {k: tot[k] + st[k] if k != "a_groups" else st[k] for k in st}
            if chunk < npaths:
                progress(f"  paths {off + n}/{npaths}")
        return tot

    progress(f"{args.workload}: k={c.k}, {npaths} paths, {bits.size} bitstrings, workspace {ws_bytes / 2**30:.1f} GiB")
    tuning = None
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")]
        r, lb, wpc = vals[:3]
        dense = vals[3] if len(vals) > 3 else 0
        nofold = vals[4] if len(vals) > 4 else 0
        flev = vals[5] if len(vals) > 5 else 0
        sf.set_tuning(c.handle, reg_qubits=r, leaf_batch=lb, waves_per_cu=wpc, dense_qubits=dense,
                      no_leaf_fold=nofold, fold_levels=flev)
        tuning = sf.get_tuning(c.handle)
    elif not args.no_autotune:
        progress("autotune")
        tuning = sf.autotune(c.handle, ids, begin, npaths, d_bits, bits.size, d_amps, flags, stream, ws, ws_bytes,
                             n_measure=6)

    for i in range(args.warmup):
        progress(f"warm-up step {i + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()
    sweep_ms = gather_ms = other_ms = host_ms = plan_ms = 0.0
    sweep_launches = gather_launches = 0
    sweep_bytes = gather_bytes = gather_row_bytes = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        progress(f"timed step {i + 1}/{args.steps}")
        st = step(sf.SF_TIMING)
        sweep_ms += st["ms_sweep"]
        gather_ms += st["ms_gather"]
        other_ms += st["ms_other"]
        host_ms += st["ms_total"]
        plan_ms += st["ms_plan"]
        sweep_launches += st["n_sweep_launches"]
        gather_launches += st["n_gather_launches"]
        sweep_bytes += st["sweep_bytes"]
        gather_bytes += st["gather_bytes"]
        gather_row_bytes += st["gather_row_bytes"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    paths_per_s = npaths * args.steps / elapsed
    amps_per_s = bits.size * args.steps / elapsed

    # dominant kernel category by measured time
    plan_text = sf.describe_plan(c.handle)
    folded = "folded" in plan_text
    if sweep_ms >= gather_ms:
        dom, dom_ms, dom_n, dom_bytes = "pass_kernel (gate sweep)", sweep_ms, sweep_launches, sweep_bytes
    elif folded and "iSWAP gates" in plan_text:
        dom, dom_ms, dom_n, dom_bytes = ("fold_iswap_kernel (last levels + path sum)", gather_ms, gather_launches,
                                         gather_bytes)
    elif folded:
        dom, dom_ms, dom_n, dom_bytes = "fold_kernel (last level + path sum)", gather_ms, gather_launches, gather_bytes
    else:
        dom, dom_ms, dom_n, dom_bytes = "gather_kernel (path sum)", gather_ms, gather_launches, gather_bytes
    avg_launch_ms = dom_ms / max(dom_n, 1)
    achieved = (dom_bytes / max(dom_n, 1)) / (avg_launch_ms * 1e-3) / 1e9 if dom_n else 0.0
    traffic = measured_traffic(args.workload, dom.split(" ")[0])

    # plain one-path-per-launch GPU form on a subset of the same paths
    plain = None
    plain_n = min(args.plain_paths, npaths)
    if plain_n > 0:
        plain_ids = ids[:plain_n] if ids is not None else None
        sf.run_paths(c.handle, plain_ids, begin, plain_n, d_bits, bits.size, d_amps, flags | sf.SF_PLAIN, stream, ws,
                     ws_bytes)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        sf.run_paths(c.handle, plain_ids, begin, plain_n, d_bits, bits.size, d_amps, flags | sf.SF_PLAIN, stream, ws,
                     ws_bytes)
        torch.cuda.synchronize()
        plain_paths_per_s = plain_n / (time.perf_counter() - tp)
        plain = {"paths_per_s": plain_paths_per_s, "paths": plain_n, "speedup_of_batched": paths_per_s / plain_paths_per_s}

    progress("timed steps done")
    serving = serving_bench(args.serve_jobs) if args.serve_jobs > 0 else None
    sampling = None if args.no_sampling else sampling_bench(c, ids, begin, npaths, bits.size, ws, ws_bytes, stream)
    validation = None
    if not args.no_sampling and cfg.paths == "all":
        step()                      # exact amplitudes again (the plain-form runs overwrote them)
        torch.cuda.synchronize()
        validation = validation_bench(c, bits, d_amps, cfg.bits_seed, ws, ws_bytes, stream)

    iswap = None
    if not args.no_iswap and args.workload != "grid5x6_d24_iswap":
        progress("iSWAP variant")
        iswap = iswap_bench(stream)

    cpu = None
    progress("CPU oracle sample")
    if not args.no_cpu:
        cpu = cpu_baseline(cfg, gates, bits, c.k, ids, begin, npaths, args.cpu_seconds)

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
                   "k": c.k, "paths": npaths, "f": cfg.f if cfg.paths == "sample" else npaths / 2.0 ** c.k,
                   "bitstrings": int(bits.size), "tuning": tuning or sf.get_tuning(c.handle),
                   **({"paths_sample": f"first {npaths} of {full_paths} paths"} if npaths < full_paths else {})},
        "amps_per_s": amps_per_s,
        "plain_form": plain,
        "kernel_ms_per_step": {"sweep": sweep_ms / args.steps, "gather": gather_ms / args.steps,
                               "other": other_ms / args.steps},
        "run_paths_wall_ms_per_step": host_ms / args.steps,
        "host_plan_ms_per_step": plan_ms / args.steps,
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": avg_launch_ms, "launches_per_step": dom_n / args.steps,
                     "bytes_per_launch": dom_bytes / max(dom_n, 1),
                     "row_bytes_per_launch": (gather_row_bytes / max(gather_launches, 1)
                                              if not dom.startswith("pass") else None),
                     "a_groups": st["a_groups"]},
        "sweep_roofline": {"kernels": "pass_kernel + dense_kernel (gate sweeps, all levels written)", "bound": "hbm",
                           "achieved": (sweep_bytes / max(sweep_ms, 1e-9)) / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": (sweep_bytes / max(sweep_ms, 1e-9)) / 1e6 / HBM_PEAK_GBS,
                           "bytes_per_step": sweep_bytes / args.steps, "launches_per_step": sweep_launches / args.steps,
                           "note": "time of one event pair around each run of sweep launches, gaps included"},
        "cpu_baseline": cpu,
        "serving": serving,
        "sampling": sampling,
        "validation": validation,
        "iswap": iswap,
    }
    print(json.dumps(out), flush=True)
    c.close()


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of
    this workload, or None if there is none or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1807_10749_amd", "csrc", "kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernel_source_sha256"):
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


def iswap_bench(stream, steps=3, warmup=1):
    """The harder variant (every CZ of the default circuit an iSWAP, Eq. (4way): four terms and
    two path bits per crossing gate, k = 30): one seeded aligned block of 2^18 paths, 1e5
    bitstrings, autotuned, timed like the headline step."""
    import torch
    from paper_1807_10749_amd import binding as sf
    from workload import make_workload, path_block
    w = make_workload("grid5x6_d24_iswap")
    cfg, bits = w["cfg"], w["bitstrings"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    begin, npaths = path_block(c.k, cfg.block_bits, cfg.path_seed)
    d_bits = torch.from_numpy(bits.view(np.int64)).cuda()
    d_amps = torch.zeros(2 * bits.size, dtype=torch.float64, device="cuda")
    # the bound assumes every leaf resident at once; the library batches leaves within what it gets
    free_b, _ = torch.cuda.mem_get_info()
    ws_bytes = min(sf.workspace_size(c.handle, npaths, bits.size, 0), 64 << 30, int(free_b * 0.5))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    flags = sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    tuning = sf.autotune(c.handle, None, begin, npaths, d_bits, bits.size, d_amps, flags, stream, ws, ws_bytes,
                         n_measure=4)
    for _ in range(warmup):
        sf.run_paths(c.handle, None, begin, npaths, d_bits, bits.size, d_amps, flags, stream, ws, ws_bytes)
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
           "tuning": tuning}
    c.close()
    return out


def serving_bench(n_jobs, workers=4, chunk_paths=16384, seed=5005):
    """Serving mix: Poisson arrivals at 0.7 of the sequential service rate.

    Jobs (grid 4x5..6x6, depth 1+16+1..1+32+1, 1e3..1e5 bitstrings, f in
    {0.01, 0.1, 1}) are served by the library's server (continuous batching over
    `workers` streams).  References on the same jobs: the batched form run one
    job at a time (its throughput, and the latencies a FIFO queue of those
    measured run times gives under the same arrivals), and the plain
    one-path-per-launch form run one job at a time (timed on up to 8 paths per
    job and scaled to the job's path count).  A second served run submits every
    job at once, for the throughput of a saturated server.
    """
    import math
    from paper_1807_10749_amd import binding as sf
    from workload import SplitMix64, grid_circuit, random_bitstrings, serving_mix

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

    # one job at a time (batched form)
    srv = sf.server_create(arena, None, 1, chunk_paths)
    seq_res, seq_t, n_paths = [], [], []
    for i in range(n_jobs):
        jid = submit(srv, i)
        sf.server_drain(srv)
        done, a, info = sf.server_poll(srv, jid, specs[i]["n_bits"])
        seq_res.append(a.copy())
        seq_t.append(info["t_done"] - info["t_admit"])
        n_paths.append(info["n_paths"])
        sf.server_release(srv, jid)
    sf.server_destroy(srv)
    total_paths = sum(n_paths)
    mean_s = sum(seq_t) / n_jobs

    # plain form, one job at a time, timed on a few paths per job
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
    def served(arr):
        """Submit job i at arr[i] seconds (all at once when arr is all zeros), drain, and return
        the latencies, the first submit and last completion times, the largest relative
        difference from the one-at-a-time results, and the server's counters."""
        srv = sf.server_create(arena, None, workers, chunk_paths)
        t0 = time.perf_counter()
        jids = []
        for i in range(n_jobs):
            dt = arr[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            jids.append(submit(srv, i))
        sf.server_drain(srv)
        lat, first, last, dev = [], 1e300, 0.0, 0.0
        for i, jid in enumerate(jids):
            done, a, info = sf.server_poll(srv, jid, specs[i]["n_bits"])
            lat.append(info["t_done"] - info["t_submit"])
            first, last = min(first, info["t_submit"]), max(last, info["t_done"])
            ref = seq_res[i]
            dev = max(dev, float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300)))
        st = sf.server_stats(srv)
        sf.server_destroy(srv)
        return sorted(lat), first, last, dev, st

    def pct(lat, q):
        return lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)]

    lat, first, last, dev, st = served(arrivals)
    # the one-at-a-time form under the same arrivals: a FIFO queue whose service times are the
    # measured one-at-a-time run times of the same jobs
    fifo, free = [], 0.0
    for i in range(n_jobs):
        start = max(arrivals[i], free)
        free = start + seq_t[i]
        fifo.append(free - arrivals[i])
    fifo.sort()
    # saturated: every job submitted at once, so the device always has admitted work queued
    sat_lat, sat_first, sat_last, sat_dev, sat_st = served([0.0] * n_jobs)
    return {"jobs": n_jobs, "workers": workers, "arrival_rate_jobs_per_s": rate, "total_paths": total_paths,
            "p50_latency_ms": 1e3 * pct(lat, 0.50), "p99_latency_ms": 1e3 * pct(lat, 0.99),
            "served_paths_per_s": total_paths / (last - first), "makespan_s": last - first,
            "sequential_paths_per_s": total_paths / sum(seq_t),
            "sequential_fifo_p50_latency_ms": 1e3 * pct(fifo, 0.50),
            "sequential_fifo_p99_latency_ms": 1e3 * pct(fifo, 0.99),
            "saturated": {"paths_per_s": total_paths / (sat_last - sat_first), "makespan_s": sat_last - sat_first,
                          "p50_latency_ms": 1e3 * pct(sat_lat, 0.50), "p99_latency_ms": 1e3 * pct(sat_lat, 0.99),
                          "max_concurrent_chunks": sat_st["max_concurrent_chunks"],
                          "alone_vs_mix_max_rel_diff": sat_dev},
            "plain_sequential_paths_per_s": total_paths / plain_total, "plain_extrapolated": True,
            "max_concurrent_chunks": st["max_concurrent_chunks"], "peak_arena_bytes": st["peak_bytes"],
            "alone_vs_mix_max_rel_diff": dev}


def cpu_baseline(cfg, gates, bits, k, ids, begin, npaths, budget_s):
    """The FP64 oracle's path sum on a bounded, time-boxed sample of the same workload."""
    import oracle
    from oracle.build import build
    if not os.path.exists(oracle.lib_path()):
        build()
    all_ids = ids if ids is not None else None
    chunk = 16
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < npaths:
        m = min(chunk, npaths - done)
        sel = all_ids[done:done + m] if all_ids is not None else np.arange(begin + done, begin + done + m, dtype=np.uint64)
        oracle.path_sum(cfg.n_qubits, gates, cfg.cut_mask(), sel, bits)
        done += m
        chunk = min(chunk * 2, 4096)
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "paths/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {done} of {npaths} paths x all {bits.size} bitstrings, {el:.1f} s"}


if __name__ == "__main__":
    main()
