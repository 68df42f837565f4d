"""Benchmark of the FACO hot path on one MI355X.

A step is one iteration of the FACO main loop over the whole colony: every ant
builds its focused tour and improves it with 2-opt/Or-opt, then the colony
update and the pheromone update run.  The workload is the 100 000-city
stipple-like instance (64 ants, 32 new edges, retention 0.5, k = 16, backup
lists of 64).  Prints one JSON line on stdout (progress goes to stderr).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

The line's `value` is the rate of the K timed iterations that follow W
untimed ones.  Beside it the line carries:
  full_run        the configured run (1000 iterations from the build) timed
                  on a fresh instance, every tour length recomputed and
                  checked on the device in every iteration;
  lengths_verified  the timed instance's tours recomputed after the region;
  roofline        the ant kernel against HBM bandwidth, algorithmic bytes from
                  the per-ant counters (the byte model below) over the mean
                  ant-kernel launch time taken with HIP events in the timed
                  region; traffic from the committed counter profile when it
                  was taken on this kernel source and window;
  cpu_baseline    the oracle on the host over the same iterations, with
                  threads = min(nproc, ants), plus one-thread and smaller-
                  workload figures;
  batched, served short runs of the 256-instance batch and of the 256-request
                  Poisson stream (--no-batch / --no-served to skip).

    python bench.py --workload batch256 | served   runs only that mode.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


HW_QUEUES = 16


def _needs_hw_queues():
    """True when this process should run the benchmark as a child with
    HW_QUEUES hardware queues: the setting is missing or lower (a child never
    relaunches)."""
    if os.environ.get("FACO_BENCH_CHILD") == "1":
        return False
    try:
        have = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    except ValueError:
        have = 4
    return have < HW_QUEUES


def _run_with_hw_queues(count=HW_QUEUES):
    """The served stream runs three builder streams and four size-class
    streams beside the library's own.  HIP maps a process's streams onto
    GPU_MAX_HW_QUEUES hardware queues (4 unless set) and work on streams that
    share a queue runs in submission order: a class's batches then wait behind
    another stream's build kernels (up to seconds for a 200k-city initial
    solution).  HIP takes the setting from the environment the process starts
    with, so with fewer the benchmark runs itself as a child process that has
    it (before anything here touches the GPU) and exits with its status; the
    child gets SIGTERM if this process ends first."""
    import signal
    import subprocess

    def die_with_parent():
        import ctypes
        ctypes.CDLL("libc.so.6", use_errno=True).prctl(1, signal.SIGTERM)  # PR_SET_PDEATHSIG

    env = dict(os.environ, GPU_MAX_HW_QUEUES=str(count), FACO_BENCH_CHILD="1")
    return subprocess.run([sys.executable] + sys.argv, env=env,
                          preexec_fn=die_with_parent).returncode

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the ant kernel's device code: the headers and the ant-kernel
    translation units (the host side of the library, faco_api.hip, is left
    out)."""
    import hashlib
    import glob
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2203_02228_amd", "csrc", "*"))):
        if os.path.basename(f) == "faco_api.hip":
            continue
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload, warmup, steps):
    """HBM bytes per ant-kernel launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on this kernel source over this window."""
    path = os.path.join(ROOT, "profiles", f"ant_kernel_{workload}_w{warmup}_s{steps}_traffic.md")
    if not os.path.exists(path):
        return None, "no committed counter profile for this window"
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("#", "|", "`", "cd ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None, "counter profile taken on another kernel source"
    if kv.get("window") != f"{warmup + 1}..{warmup + steps}":
        return None, "counter profile taken over another window"
    return float(kv["traffic_bytes_per_launch"]), path


def survey_bytes_per_ant(cnt, n, k):
    """The byte model of the measurement plan, per ant-tour, from the per-ant
    counters (identical on the oracle and the GPU):
      8n                route + pos written once
      4 C               the source read along the copy (C copied cities)
      S (12k + 8)       per ACO step the candidate, pheromone and heuristic
                        rows and the source successor/predecessor
      F 8n              per nearest-unvisited scan every coordinate
      P (4k + 16k)      per LS pop the candidate row, and per candidate its
                        position, tour neighbour and two coordinates
      12 R              per moved element a route read + write and a pos write
    """
    S, C, Fb = cnt[:, 0], cnt[:, 1], cnt[:, 3]
    P, R = cnt[:, 5], cnt[:, 8]
    return (8 * n + 4 * C + S * (12 * k + 8) + Fb * 8 * n + P * 20 * k + 12 * R).astype(np.float64)


def lower_bound_bytes_per_ant(cnt, n, k, bl):
    """A tighter lower-bound model of what this kernel must move: ACO step
    12k + 28 (rows, source neighbours, coordinates, route/pos writes); copied
    city 20; backup pick 4 bl; nearest-unvisited scan n/2 (the bounding boxes
    of the 32-city words it tests; pruned words' coordinates not counted);
    LS pop 52k + 64 (row, per candidate position, neighbour and coordinates
    for both 2-opt loops, own neighbourhood); moved element 12."""
    S, C, B, Fb = cnt[:, 0], cnt[:, 1], cnt[:, 2], cnt[:, 3]
    P, R = cnt[:, 5], cnt[:, 8]
    return (S * (12 * k + 28) + 20 * C + B * 4 * bl + Fb * (n // 2) +
            P * (52 * k + 64) + 12 * R).astype(np.float64)


# ------------------------------------------------------------- CPU legs ---

def _oracle_rate(xy, params, warmup, steps, threads, budget_s):
    from oracle import oracle as O
    t0 = time.time()
    o = O.Oracle(xy, threads=threads, **params)
    build_s = time.time() - t0
    o.run(warmup)
    iters, t_run = 0, 0.0
    while t_run < budget_s and iters < steps:
        t1 = time.time()
        o.run(1)
        t_run += time.time() - t1
        iters += 1
    o.close()
    return params["n_ants"] * iters / t_run, iters, t_run, build_s


def cpu_baseline(xy, params, warmup, steps, budget_s):
    """The oracle on the host over the timed iterations (fewer if the budget
    runs out first), threads = min(nproc, ants); the oracle's parallelism is
    over ants.  Also its one-thread rate and its rate on the 1000- and
    20 000-city workloads."""
    from paper_2203_02228_amd import instances as I
    nproc = os.cpu_count() or 1
    A = params["n_ants"]
    threads = max(1, min(nproc, A))
    log(f"cpu baseline: oracle, {threads} threads ...")
    v, iters, t_run, build_s = _oracle_rate(xy, params, warmup, steps, threads, budget_s)
    out = {"value": round(v, 2), "unit": "ant-tours/s", "cores": threads, "kind": "oracle",
           "sample": f"iterations {warmup + 1}..{warmup + iters} of the same instance "
                     f"({iters} iterations, {t_run:.1f} s; build {build_s:.1f} s untimed); "
                     f"host nproc {nproc}"}
    log("cpu baseline: oracle, 1 thread ...")
    v1, it1, t1, _ = _oracle_rate(xy, params, warmup, steps, 1, budget_s / 2)
    out["one_thread"] = {"value": round(v1, 2), "iterations": it1, "seconds": round(t1, 1)}
    out["other_workloads"] = {}
    for name in ("uniform1k", "gmm20k"):
        w = I.WORKLOADS[name]
        wt = max(1, min(nproc, w.n_ants))
        log(f"cpu baseline: oracle on {name}, {wt} threads ...")
        vr, itr, tr, _ = _oracle_rate(w.points(), w.params(), 0, w.iterations, wt, budget_s / 4)
        out["other_workloads"][name] = {"value": round(vr, 2), "cores": wt,
                                        "iterations": f"1..{itr}", "seconds": round(tr, 1)}
    return out


def _gen_points(args):
    from paper_2203_02228_amd import instances as I
    kind, n, seed = args
    return I.make_points(kind, n, seed)


def gen_points_parallel(specs, procs=None):
    """Generate [(kind, n, seed)] point sets in a process pool (deterministic)."""
    import multiprocessing as mp
    procs = procs or min(16, os.cpu_count() or 1, len(specs))
    if procs <= 1:
        return [_gen_points(s) for s in specs]
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_gen_points, specs)


# ------------------------------------------------------------- batched ---

def run_batch_mode(args):
    """Uneven batch (256 instances, n log-uniform in [200, 5000], k 12, 16
    ants, m 8, 300 iterations): shared graph-replayed launches vs one
    instance at a time, at equal iteration budgets; results must agree."""
    import torch
    from paper_2203_02228_amd import faco as F
    from paper_2203_02228_amd import instances as I
    ws = I.batch_instances(count=args.batch_count)
    iters = args.batch_iterations or ws[0].iterations
    pts = gen_points_parallel([(w.kind, w.n, w.instance_seed) for w in ws])
    torch.cuda.set_device(0)
    # a stream of its own (not the legacy default stream, which orders itself
    # against the library's streams)
    stream = torch.cuda.Stream()
    hs = [F.faco_build_instance(p, stream=stream, **w.params()) for p, w in zip(pts, ws)]
    torch.cuda.synchronize()
    # the library's autotuner times every configuration on twins of the batch
    # and stores the fastest for this size class
    t0 = time.perf_counter()
    if args.batch_config:
        # a given configuration instead of the autotuner's
        keys = ["persistent", "team_waves", "ants_per_block", "queue_lds_capacity",
                "big_percent", "big_team_waves"]
        tuned = dict(zip(keys, [int(x) for x in args.batch_config.split(",")]))
        F.faco_set_batch_config(**tuned)
    else:
        tuned = F.faco_autotune_batch(hs, trial_iterations=args.tune_iterations, stream=stream)
    tune_s = time.perf_counter() - t0
    log(f"batch configuration ({tune_s:.1f} s) -> {tuned}")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    F.faco_run_batch(hs, iters, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_batch = ev0.elapsed_time(ev1) * 1e-3
    res_batch = [F.faco_get_best_tour(h)[1] for h in hs]
    for h in hs:
        h.close()
    # one instance per launch sequence, on a subset
    sub = min(args.batch_seq_count, len(ws))
    hs = [F.faco_build_instance(p, stream=stream, **w.params())
          for p, w in zip(pts[:sub], ws[:sub])]
    torch.cuda.synchronize()
    ev0.record(stream)
    for h in hs:
        F.faco_run_iterations(h, iters)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_seq = ev0.elapsed_time(ev1) * 1e-3
    res_seq = [F.faco_get_best_tour(h)[1] for h in hs]
    for h in hs:
        h.close()
    F.faco_set_batch_config()   # forget the tuned choice
    same = res_seq == res_batch[:sub]
    return {
        "metric": "batched solves/s (256 uneven instances, 300 iterations each)",
        "value": round(len(ws) / t_batch, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": iters, "warmup": 0, "ms_per_step": round(t_batch / iters * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32+f32", "data": "synthetic",
        "config": {"workload": "batch256", "instances": len(ws),
                   "n_range": [min(w.n for w in ws), max(w.n for w in ws)],
                   "ants": 16, "cl_size": 12, "min_new_edges": 8, "rho": 0.5,
                   "tuned": tuned, "autotune_s": round(tune_s, 2)},
        "one_launch_per_instance": {"solves_per_s": round(sub / t_seq, 3), "instances": sub,
                                    "speedup": round((len(ws) / t_batch) / (sub / t_seq), 2),
                                    "identical_lengths": bool(same)},
    }


# -------------------------------------------------------------- served ---

def run_served_mode(args):
    """Poisson stream of stipple solves (n log-uniform in [1000, 200000], 32
    ants, m 16, 200 iterations) through the continuous-batching server, vs
    the same requests solved one after another."""
    import torch
    from paper_2203_02228_amd import faco as F
    from paper_2203_02228_amd import instances as I
    from paper_2203_02228_amd import serve as S
    count = args.requests
    reqs = I.served_requests(count=count, rate=args.rate)
    t0 = time.time()
    pts = gen_points_parallel([(w.kind, w.n, w.instance_seed) for _, w in reqs])
    log(f"served: {count} request point sets in {time.time() - t0:.0f} s")
    torch.cuda.set_device(0)
    classes = tuple(int(x) for x in args.served_classes.split(",")) + (1 << 30,)
    srv = S.Server(hbm_budget_bytes=args.hbm_budget << 30, chunk=args.chunk, classes=classes,
                   builders=args.served_builders)
    tuned, tune_s = {}, 0.0
    if args.serve_tune:
        # before the stream: a few requests of each size class, built aside
        t0 = time.perf_counter()
        per_class = {}
        for (_, w), p in zip(reqs, pts):
            c = srv._class_of(w.n)
            if len(per_class.setdefault(c, [])) < args.serve_tune_samples:
                per_class[c].append((p, w.params()))
        tuned = srv.tune([x for v in per_class.values() for x in v],
                         trial_iterations=args.serve_tune_iterations)
        tune_s = time.perf_counter() - t0
        log(f"served: per-class autotune ({tune_s:.1f} s) -> {tuned}")
    t0 = time.perf_counter()
    futs = []
    for (arr, w), p in zip(reqs, pts):
        now = time.perf_counter() - t0
        if arr > now:
            time.sleep(arr - now)
        futs.append(srv.submit(len(futs), p, w.params(), w.iterations))
    for i, f in enumerate(futs):
        f.result(timeout=args.result_timeout)
        if (i + 1) % 64 == 0:
            log(f"served: {i + 1}/{count} results ({time.perf_counter() - t0:.0f} s)")
    makespan = time.perf_counter() - t0
    srv.close()
    F.faco_set_batch_config()   # forget the tuned choices
    done = sorted(srv.completed, key=lambda r: r.rid)
    lat = S.latency_stats(done)
    lengths = {r.rid: r.result[1] for r in done}
    # sequential plain solves of a sample of the same requests
    sample = list(range(0, count, max(1, count // args.seq_sample)))[:args.seq_sample]
    stream = torch.cuda.current_stream()
    svc, same = [], True
    for i in sample:
        (_, w), p = reqs[i], pts[i]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h = F.faco_build_instance(p, stream=stream, **w.params())
        F.faco_run_iterations(h, w.iterations)
        _, L = F.faco_get_best_tour(h)
        svc.append(time.perf_counter() - t1)
        h.close()
        same = same and (L == lengths[i])
    seq_rate = len(sample) / sum(svc)
    # where each request's latency went: admission wait, build, resident run
    stages = {}
    for name, lo, hi in (("all", 0, 1 << 30), ("n<8000", 0, 8000), ("8000<=n<40000", 8000, 40000),
                         ("n>=40000", 40000, 1 << 30)):
        rs = [r for r in done if lo <= len(r.xy) < hi]
        if not rs:
            continue
        part = {}
        for key, f in (("wait", lambda r: r.admitted - r.arrival),
                       ("build", lambda r: r.built - r.admitted),
                       ("run", lambda r: r.finished - r.built),
                       ("total", lambda r: r.finished - r.arrival)):
            v = np.array([f(r) for r in rs])
            part[key] = {"mean": round(float(v.mean()), 2), "p50": round(float(np.percentile(v, 50)), 2),
                         "p99": round(float(np.percentile(v, 99)), 2)}
        part["requests"] = len(rs)
        stages[name] = part
    return {
        "solves_per_s": round(count / makespan, 3),
        "p50_latency_s": round(lat["p50_s"], 3), "p99_latency_s": round(lat["p99_s"], 3),
        "requests": count, "arrival_rate_per_s": args.rate, "makespan_s": round(makespan, 2),
        "sequential_solves_per_s": round(seq_rate, 3),
        "sequential_sample": len(sample),
        "identical_lengths": bool(same),
        "n_range": [min(w.n for _, w in reqs), max(w.n for _, w in reqs)],
        "errors": len(srv.errors),
        "latency_stages_s": stages,
        # per size class: resident solves per batch call and time per iteration
        "classes": [{"n_below": hi, "calls": st["calls"],
                     "mean_resident": round(st["active_sum"] / max(1, st["calls"]), 2),
                     "max_resident": st["max_active"],
                     "ms_per_iteration": round(1e3 * st["busy_s"] / max(1, st["iterations"]), 2),
                     "busy_frac": round(st["busy_s"] / makespan, 3)}
                    for hi, st in zip(srv.classes, srv.class_stats)],
        "tuned_by_class": {str(k): v for k, v in tuned.items()}, "autotune_s": round(tune_s, 1),
    }


# ------------------------------------------------------------ headline ---

def run_iterations_timed(F, g, stream, steps, torch, label):
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    done, chunk = 0, max(1, steps // 10)
    while done < steps:
        step = min(chunk, steps - done)
        F.faco_run_iterations(g, step)
        done += step
        log(f"{label}: {done}/{steps} iterations enqueued")
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def window_without_events(F, stream, w, warmup, steps, torch):
    """The timed window again on a fresh build with the per-launch HIP events
    off (the headline keeps them on: the roofline takes the ant kernel's mean
    launch time from them), to show what they cost."""
    g = F.faco_build_instance(w.points(), stream=stream, **w.params())
    F.faco_run_iterations(g, warmup)
    torch.cuda.synchronize()
    ms = run_iterations_timed(F, g, stream, steps, torch, "window without launch events")
    g.close()
    return {"value": round(w.n_ants * steps / (ms * 1e-3), 2),
            "ms_per_step": round(ms / steps, 4)}


def slowest_ants(F, stream, w, warmup, steps, torch):
    """The same window on a fresh build, one iteration at a time: the phase
    times of each iteration's slowest ant (it sets the launch time), averaged
    over the window, beside the median ant's.  Outside the timed region."""
    g = F.faco_build_instance(w.points(), stream=stream, **w.params())
    F.faco_run_iterations(g, warmup)
    torch.cuda.synchronize()
    names = {0: "construct", 1: "ls_eval", 2: "ls_apply", 15: "ls_rewrite", 3: "sweep",
             24: "sweep_tests", 25: "sweep_listing", 4: "ant_total"}
    prev = F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS).astype(np.int64)
    cprev = F.faco_debug_get(g, F.FACO_DBG_COUNTER_TOTALS).astype(np.int64)
    slow, med = [], []
    for _ in range(steps):
        F.faco_run_iterations(g, 1)
        tk = F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS).astype(np.int64)
        c = F.faco_debug_get(g, F.FACO_DBG_COUNTER_TOTALS).astype(np.int64)
        d, dc = tk - prev, c - cprev
        prev, cprev = tk, c
        order = np.argsort(d[:, 4])
        for a, out in ((order[-1], slow), (order[len(order) // 2], med)):
            row = {v: d[a, k] / 100.0 for k, v in names.items()}
            row["moves"] = dc[a, 6] + dc[a, 7]
            row["sweep_cities"] = d[a, 26]
            row["moved_elems"] = dc[a, 8]
            out.append(row)
    g.close()
    avg = lambda rows: {k: round(float(np.mean([r[k] for r in rows])), 1) for k in rows[0]}
    return {"slowest": avg(slow), "median": avg(med)}


def full_run(F, I, torch, stream, w):
    """The configured run: all of the workload's iterations from a fresh build,
    with every tour length recomputed and checked on the device in every
    iteration (the checks' own time is measured and reported apart)."""
    xy = w.points()
    g = F.faco_build_instance(xy, stream=stream, **w.params())
    F.faco_set_verify(g, True)
    F.faco_set_timing(g, True, reserve_iterations=w.iterations)
    tk0 = F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS)
    total_ms = run_iterations_timed(F, g, stream, w.iterations, torch, "full run")
    phase_ms, launches = F.faco_phase_times(g)
    per = (F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS) - tk0).astype(np.float64).mean(0) / w.iterations
    per_ant_us = {name: round(float(per[i]) / 100.0, 1) for i, name in
                  [(0, "construct"), (1, "ls_eval"), (2, "ls_apply"), (3, "sweep"),
                   (4, "ant_total"), (15, "ls_rewrite")]}
    fault = F.faco_debug_get(g, F.FACO_DBG_FAULT)
    _, best_len = F.faco_get_best_tour(g) if fault[0] == 0 else (None, -1)
    info = F.faco_debug_get(g, F.FACO_DBG_INFO)
    g.close()
    A = w.n_ants
    return {
        "iterations": int(info[0]), "ms_per_iteration": round(total_ms / w.iterations, 4),
        "ant_tours_per_s": round(A * w.iterations / (total_ms * 1e-3), 2),
        "ant_kernel_mean_ms": round(phase_ms[0] / max(1, launches[0]), 4),
        "best_length": int(best_len),
        "lengths_verified": bool(fault[0] == 0 and fault[3] == w.iterations * (A + 1)),
        "tours_verified": int(fault[3]), "device_faults": int(fault[0]),
        "per_ant_us": per_ant_us,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="stipple100k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-run", action="store_true")
    ap.add_argument("--no-slowest", action="store_true",
                    help="skip the per-iteration slowest-ant breakdown")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-iterations", type=int, default=0)
    ap.add_argument("--batch-seq-count", type=int, default=32)
    ap.add_argument("--tune-iterations", type=int, default=30)
    ap.add_argument("--batch-config", default="",
                    help="persistent,team_waves,ants_per_block,queue_lds_capacity,big_percent,"
                         "big_team_waves: run the batch with this configuration, untuned")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--chunk", type=int, default=10)
    ap.add_argument("--hbm-budget", type=int, default=64, help="GiB for resident solves")
    ap.add_argument("--seq-sample", type=int, default=16)
    ap.add_argument("--served-classes", default="4000,16000,64000",
                    help="upper size bounds of the served size classes but the last")
    ap.add_argument("--served-builders", type=int, default=3)
    ap.add_argument("--serve-tune", type=int, default=1)
    ap.add_argument("--serve-tune-samples", type=int, default=8,
                    help="requests per size class the served autotune times")
    ap.add_argument("--serve-tune-iterations", type=int, default=6)
    ap.add_argument("--result-timeout", type=float, default=900.0)
    ap.add_argument("--team-waves", type=int, default=0,
                    help="waves per ant (0 = the library's choice by size; 1, 4, 8)")
    ap.add_argument("--tour-segments", type=int, default=0,
                    help="local-search tour: 0 or 1 flat arrays, 2 segment lists")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB copied once by a plain device-to-device copy kernel before "
                         "the workload (scales hardware byte counters)")
    args = ap.parse_args()
    log(f"GPU_MAX_HW_QUEUES={os.environ.get('GPU_MAX_HW_QUEUES', '(unset)')}")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the ants of an iteration would shard across GPUs; this benchmark "
              "runs and measures one)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch256":
        print(json.dumps(run_batch_mode(args)), flush=True)
        return
    if args.workload == "served":
        out = run_served_mode(args)
        out.update({"metric": "served solves/s (Poisson stipple requests, 200 iterations)",
                    "value": out["solves_per_s"], "unit": "solves/s", "n_gpus": 1})
        print(json.dumps(out), flush=True)
        return

    import torch
    from paper_2203_02228_amd import faco as F
    from paper_2203_02228_amd import instances as I

    w = I.WORKLOADS[args.workload]
    params = w.params()
    xy = w.points()
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read, {nbytes} written")
        del src, dst
    stream = torch.cuda.current_stream()
    F.faco_set_team_waves(args.team_waves)
    F.faco_set_tour_segments(args.tour_segments)
    t0 = time.time()
    g = F.faco_build_instance(xy, stream=stream, **params)
    build_s = time.time() - t0
    team_waves = int(F.faco_debug_get(g, F.FACO_DBG_TEAM_WAVES)[0])
    log(f"built {w.name} n={w.n} in {build_s:.2f} s")
    F.faco_run_iterations(g, args.warmup)
    torch.cuda.synchronize()
    F.faco_phase_times(g)  # clear
    F.faco_set_timing(g, True, reserve_iterations=args.steps)

    n, k, bl, A = w.n, g.k, g.bl, w.n_ants
    tot0 = F.faco_debug_get(g, F.FACO_DBG_COUNTER_TOTALS)
    tk0 = F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS)
    total_ms = run_iterations_timed(F, g, stream, args.steps, torch, "timed")
    phase_ms, launches = F.faco_phase_times(g)
    F.faco_set_timing(g, False)
    tot1 = F.faco_debug_get(g, F.FACO_DBG_COUNTER_TOTALS)
    tk = (F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS) - tk0).astype(np.float64)
    # per ant and iteration: microseconds (100 MHz wall clock) and call counts
    per = tk.mean(0) / args.steps
    tk_us = {name: round(float(per[i]) / 100.0, 1) for i, name in
             [(0, "construct"), (1, "ls_eval"), (2, "ls_apply"), (3, "sweep"), (4, "ant_total"),
              (8, "spec_windows"), (9, "one_steps"), (10, "copies"), (11, "fallbacks"),
              (13, "ls_eval_oropt"), (15, "ls_rewrite"), (24, "sweep_tests"),
              (25, "sweep_listing")]}
    tk_calls = {name: round(float(per[i]), 1) for i, name in
                [(5, "spec_windows"), (6, "one_steps"), (7, "copies"), (12, "eval_rounds"),
                 (14, "oropt_rounds"), (26, "sweep_cities")]}
    slowest_us = round(float(tk[:, 4].max()) / args.steps / 100.0, 1)
    dcnt = tot1 - tot0
    bytes_survey = float(survey_bytes_per_ant(dcnt, n, k).sum())
    bytes_lb = float(lower_bound_bytes_per_ant(dcnt, n, k, bl).sum())
    cnt_mean = (dcnt.sum(0) / (A * args.steps)).tolist()
    # the timed instance's tours, recomputed on the device after the region
    rec = F.faco_debug_get(g, F.FACO_DBG_RECOMPUTED_LENGTHS)
    lens = F.faco_debug_get(g, F.FACO_DBG_ANT_LENGTHS)
    fault = F.faco_debug_get(g, F.FACO_DBG_FAULT)
    best_tour, best_len = F.faco_get_best_tour(g)
    lengths_ok = bool(np.array_equal(rec[:-1], lens) and rec[-1] == best_len and fault[0] == 0)
    info = F.faco_debug_get(g, F.FACO_DBG_INFO)
    tour = F.faco_debug_get(g, F.FACO_DBG_TOUR)
    g.close()
    tour_cfg = ("flat arrays" if not tour[0] else
                f"segment lists (length {int(tour[1])}, {int(tour[2])} records)")
    seg_stats = None
    if tour[0]:
        # per ant and iteration: materialisations, their time, splits,
        # relabelled cities, leader / team time of moves
        seg_stats = {"materialisations": round(float(per[16]), 2),
                     "materialise_us": round(float(per[17]) / 100.0, 1),
                     "splits": round(float(per[19]), 1),
                     "relabelled": round(float(per[18]), 1),
                     "move_leader_us": round(float(per[21]) / 100.0, 1),
                     "move_team_us": round(float(per[22]) / 100.0, 1)}

    ms_per_step = total_ms / args.steps
    ant_ms = phase_ms[0] / max(1, launches[0])
    launches_ant = max(1, launches[0])
    achieved = (bytes_survey / launches_ant) / (ant_ms * 1e-3) / 1e9
    achieved_lb = (bytes_lb / launches_ant) / (ant_ms * 1e-3) / 1e9
    traffic, traffic_src = profiled_traffic(w.name, args.warmup, args.steps)
    if tour[0]:
        traffic, traffic_src = None, "counter profile taken with flat-array tours"

    value = A * args.steps / (total_ms * 1e-3)
    out = {
        "metric": "ant-tours/s (construct+2-opt/Or-opt) at 100k cities",
        "value": round(value, 2),
        "unit": "ant-tours/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "ants": A, "min_new_edges": w.min_new_edges,
                   "cl_size": k, "bl_size": bl, "rho": w.rho, "p_best": 0.05,
                   "local_search": "2-opt+Or-opt+sweep", "iterations_timed":
                   f"{args.warmup + 1}..{args.warmup + args.steps}",
                   "best_length": int(best_len), "iterations_done": int(info[0]),
                   "waves_per_ant": team_waves, "tour": tour_cfg,
                   "build_s": round(build_s, 2)},
        "lengths_verified": lengths_ok,
        "device_faults": int(fault[0]),
        "per_ant_us": tk_us,
        "per_ant_calls": tk_calls,
        "slowest_ant_us": slowest_us,
        "segment_lists": seg_stats,
        "per_ant_counters": {name: round(v, 1) for name, v in zip(F.CNT_NAMES, cnt_mean)},
        "phase_ms_per_iteration": {name: round(phase_ms[i] / max(1, launches[i]), 4)
                                   for i, name in enumerate(["ants", "colony", "source",
                                                             "pheromone"])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic, "kernel": "ant_kernel",
                     "avg_launch_ms": round(ant_ms, 4), "launches": int(launches[0]),
                     "algorithmic_bytes_per_launch": round(bytes_survey / launches_ant),
                     "byte_model": "per ant-tour 8n + 4C + S(12k+8) + F 8n + P 20k + 12R",
                     "traffic_source": traffic_src,
                     "lower_bound_model": {
                         "achieved": round(achieved_lb, 2),
                         "frac": round(achieved_lb / HBM_PEAK_GBS, 5),
                         "bytes_per_launch": round(bytes_lb / launches_ant)}},
    }
    if not args.no_full_run:
        log(f"full run: {w.iterations} iterations from a fresh build, verification on ...")
        out["full_run"] = full_run(F, I, torch, stream, w)
        log(f"full run: {out['full_run']}")
    if not args.no_slowest:
        out["window_without_launch_events"] = window_without_events(F, stream, w, args.warmup,
                                                                    args.steps, torch)
        log("slowest ant of each iteration over the same window (fresh build) ...")
        out["ants_by_iteration_us"] = slowest_ants(F, stream, w, args.warmup, args.steps, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(xy, params, args.warmup, args.steps, args.cpu_budget)
    if not args.no_batch:
        log("batch256 ...")
        b = run_batch_mode(args)
        out["batched"] = {"solves_per_s": b["value"], "ms_per_iteration": b["ms_per_step"],
                          "tuned": b["config"]["tuned"],
                          "one_launch_per_instance": b["one_launch_per_instance"]}
    if not args.no_served:
        log(f"served: {args.requests} requests at {args.rate}/s ...")
        out["served"] = run_served_mode(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    if _needs_hw_queues():
        sys.exit(_run_with_hw_queues())
    main()
