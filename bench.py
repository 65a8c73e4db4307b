"""Benchmark of the REPT counting path on one MI355X.

One step = the whole hot path over one synthetic stream already resident in HBM:
validate + orient + build (rept_build), the counting pass for all c processors (rept_count),
the reduction of the local rows to node sums on the device (rept_reduce_local), the
device-to-host copy of the c global counters and the n sums, and the FP64 estimators on the
host (rept_estimate_sums).

Default workload (the largest single-GPU one): R-MAT scale 24, edge factor 16,
(a, b, c) = (0.57, 0.19, 0.19), deduplicated, generation order (260,384,039 edges), m = c = 100.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-batched] [--no-served]
                  [--no-alg2] [--no-mascot] [--no-incremental] [--no-side] [--workload NAME]

The line also carries "config2" (the Chung-Lu 1M/20M stream, m = 10, c = 40: its steps and
roofline), "batched" (512 jobs: plain one-by-one vs one graph-captured batched launch) and
"served" (Poisson requests: continuous batching vs a FIFO plain loop) comparisons, and, on the
1M/20M stream, "alg2" (Algorithm 2's pass, c mod m != 0, against the plain count), "mascot"
(parallel MASCOT against REPT with the same m and c) and "incremental" (the stream appended in
ten chunks).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    # name: (description, generator, n, m, c)
    "config2": ("Chung-Lu 1M nodes / 20M edges, gamma 2.1, shuffled; m=10 c=40", "config2", 1_000_000, 10, 40),
    "config1": ("Erdos-Renyi 2k nodes / 20k edges, shuffled; m=10 c=10", "config1", 2000, 10, 10),
    "config3": ("R-MAT scale 24 edge factor 16 (0.57,0.19,0.19), dedup, generation order; m=100 c=100",
                "config3", 1 << 24, 100, 100),
}
HASH_SEED = 20181122
SIDE_WORKLOAD = "config2"  # measured beside the headline; the next rows run on it


def say(*a):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="config3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-side", action="store_true",
                    help=f"skip the {SIDE_WORKLOAD} workload's steps (the next rows then run only if it is the headline)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--no-served", action="store_true", help="skip the served-vs-plain comparison")
    ap.add_argument("--no-alg2", action="store_true", help="skip the Algorithm 2 (c mod m != 0) pass")
    ap.add_argument("--no-mascot", action="store_true", help="skip the parallel MASCOT pass")
    ap.add_argument("--no-incremental", action="store_true", help="skip the incremental-stream pass")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of 1 GiB (reference for FETCH_SIZE/WRITE_SIZE scaling)")
    return ap.parse_args()


def stream_for(name):
    import synth
    gen = WORKLOADS[name][1]
    return {"config1": synth.config1_stream, "config2": synth.config2_stream, "config3": synth.config3_stream}[gen]()


def count_kernel_source_digest() -> str:
    """Digest of the counting kernel's sources and of the file that picks its launch shape."""
    h = hashlib.sha256()
    for f in ("count.hip", "common.h", "api.hip"):
        with open(os.path.join(ROOT, "paper_1811_09136_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload: str):
    """HBM bytes per count launch from the committed PMC summary, if it was taken on the
    current counting kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_count_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != count_kernel_source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(info, tau: int, c: int, rows: int, n: int) -> float:
    """Bytes the counting pass must move per launch (per-unit model of the recast): per oriented
    edge 8 B staged in its unit's hash table (neighbour id, arrival time) and 16 B staged as a list
    to walk (node id, arrival time, that node's two offsets), 4 B more when it comes from a reverse
    list (its position); 20 B per unit (id, two offsets, two reverse-list offsets); 4 B per list
    entry probed (neighbour id); 4 B per triangle found (arrival time of the walked edge); 8 B per
    output counter."""
    E = info.num_edges
    return (24.0 * E + 4.0 * info.num_reverse + 20.0 * info.num_apex + 4.0 * info.oriented_work + 4.0 * tau
            + 8.0 * (c + rows * n))


def streaming_model_bytes(deg_sq_half_sum: int, E: int, groups: int, semi: int, c: int, n: int) -> float:
    """Bytes of the per-processor streaming formulation (each time-filtered per-processor set
    read at every edge): 8 E + 8 W G + 24 sum tau^(i) + 8 (c + G n), W = sum_x C(d_x, 2)."""
    return 8.0 * E + 8.0 * deg_sq_half_sum * groups + 24.0 * semi + 8.0 * (c + groups * n)


def cpu_baseline(edges, n, m, c):
    """The oracle (Algorithm 1 replay) timed on the host cores this process may use, capped at the
    16 that the GPU machine allots to one GPU: a sample of the job's processors, 0..W-1 of the c, one
    per thread, each replaying the whole stream with its own sample of about E/m edges.  Every
    processor does the same kind of work, so the whole job on W cores takes c/W times the
    sample's wall time."""
    import oracle
    usable = len(os.sched_getaffinity(0))
    W = max(1, min(16, usable, c))
    t0 = time.perf_counter()
    oracle.rept_threads(edges, n, m, c, HASH_SEED, workers=W, procs=(0, W))
    dt = time.perf_counter() - t0
    job_s = dt * c / W
    return {"value": len(edges) / job_s, "unit": "stream edges/s", "cores": W, "kind": "oracle",
            "host_cpu_count": os.cpu_count(), "host_cores_usable": usable,
            "sample": f"Algorithm 1 replay of processors 0..{W - 1} of {c} over all {len(edges)} stream edges, "
                      f"one thread each, took {dt:.2f} s on {W} cores (os.cpu_count() = {os.cpu_count()}, "
                      f"{usable} usable by this process); whole job = {c}/{W} x that"}


def bench_alg2(dev, edges, n: int, m: int, c: int, reps: int = 3):
    """Algorithm 2 on the same stream (c > m, c mod m != 0): rept_count_eta (slot table, counts
    with the per-edge pair counters, k_eta) against rept_count under the same parameters, then the
    combined estimators on the host.  The counts of both calls must agree."""
    import numpy as np
    import torch
    from paper_1811_09136_amd import rept
    params = rept.Params(m, c, HASH_SEED)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    g = rept.Graph(rept.to_device_edges(edges, dev), n)
    glob, loc = g.outputs(params)
    eta = torch.empty((2, c), dtype=torch.int64, device=dev)
    eta_v = torch.empty((2, n), dtype=torch.int64, device=dev)
    wsb = rept.rept_count_eta_workspace_size(g.handle, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    plain_ms, eta_ms = [], []
    for r in range(reps + 1):
        for kind in ("plain", "eta"):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            if kind == "plain":
                rept.rept_count(g.handle, params, glob.data_ptr(), loc.data_ptr(), ws.data_ptr(), wsb, sp)
            else:
                rept.rept_count_eta(g.handle, params, glob.data_ptr(), loc.data_ptr(), eta.data_ptr(),
                                    eta_v.data_ptr(), ws.data_ptr(), wsb, None, sp)
            ev1.record(stream)
            stream.synchronize()
            if kind == "plain":
                ref = glob.cpu().numpy()
            elif not np.array_equal(glob.cpu().numpy(), ref):
                raise RuntimeError("rept_count_eta and rept_count disagree")
            if r:
                (plain_ms if kind == "plain" else eta_ms).append(ev0.elapsed_time(ev1))
    h_glob, h_loc = glob.cpu().numpy(), loc.cpu().numpy()
    h_eta, h_eta_v = eta.cpu().numpy(), eta_v.cpu().numpy()
    t0 = time.perf_counter()
    tau_hat, _ = rept.rept_estimate_combined(n, params, h_glob, h_loc, int(h_eta[0].sum()), h_eta_v[0])
    est_ms = 1e3 * (time.perf_counter() - t0)
    g.close()
    cm, em = float(np.median(plain_ms)), float(np.median(eta_ms))
    return {"m": m, "c": c, "count_ms": cm, "count_eta_ms": em, "eta_overhead": em / cm,
            "count_eta_edges_per_s": len(edges) / (em * 1e-3), "combined_estimate_ms": est_ms,
            "tau_hat": tau_hat, "eta_def_sum": int(h_eta[0].sum()), "eta_printed_sum": int(h_eta[1].sum()),
            "semi_triangles": int(h_glob.sum())}


def bench_mascot(dev, edges, n: int, m: int, c: int = 8, reps: int = 3):
    """Parallel MASCOT (Section III-C) on the same stream with c independent samplers, against
    REPT with the same m and c (the paper expects the same computational cost)."""
    import numpy as np
    import torch
    from paper_1811_09136_amd import rept
    stream = torch.cuda.current_stream()
    g = rept.Graph(rept.to_device_edges(edges, dev), n)
    res = {"m": m, "c": c}
    for name, p in (("rept", rept.Params(m, c, HASH_SEED)), ("mascot", rept.Params(m, c, HASH_SEED, mascot=True))):
        out = g.outputs(p)
        ws = g.new_workspace(p)
        ms = []
        for r in range(reps + 1):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            g.count(p, out=out, workspace=ws)
            ev1.record(stream)
            stream.synchronize()
            if r:
                ms.append(ev0.elapsed_time(ev1))
        glob, loc = out[0].cpu().numpy(), out[1].cpu().numpy()
        tau_hat, _ = rept.rept_estimate(n, p, glob, None)
        res[name] = {"count_ms": float(np.median(ms)), "edges_per_s": len(edges) / (float(np.median(ms)) * 1e-3),
                     "semi_triangles": int(glob.sum()), "tau_hat": tau_hat}
    g.close()
    res["mascot_over_rept_time"] = res["mascot"]["count_ms"] / res["rept"]["count_ms"]
    return res


def bench_incremental(dev, edges, n: int, m: int, c: int, ref_glob, chunks: int = 10):
    """The same stream appended in `chunks` equal chunks (rept_stream_append: validate, merge,
    count the chunk's edges by the default policy, which picks per append between counting edge
    by edge against the earlier edges and a windowed recount of the prefix); per-append latency
    and whole-stream throughput, and the same with every append counted edge by edge.  The final
    counters must equal the one-shot count's."""
    import numpy as np
    import torch
    from paper_1811_09136_amd import rept
    E = len(edges)
    step = -(-E // chunks)
    d_edges = rept.to_device_edges(edges, dev)
    params = rept.Params(m, c, HASH_SEED)
    res = {"chunks": chunks, "chunk_edges": step}

    def run(policy):
        for rep in range(2):  # the first pass warms the code objects
            inc = rept.IncrementalStream(n, E, step, params, dev, policy=policy)
            torch.cuda.synchronize()
            lat = []
            t0 = time.perf_counter()
            for a in range(0, E, step):
                ta = time.perf_counter()
                inc.append(d_edges[a:a + step])
                torch.cuda.synchronize()
                lat.append(1e3 * (time.perf_counter() - ta))
            total = time.perf_counter() - t0
            same = bool(np.array_equal(inc.counts[0].cpu().numpy(), ref_glob))
            paths = inc.paths()
            inc.close()
            del inc
        if not same:
            raise RuntimeError(f"incremental counters ({policy}) disagree with the one-shot count")
        return total, lat, same, paths

    total, lat, same, paths = run("auto")
    res.update({"total_ms": 1e3 * total, "edges_per_s": E / total, "append_ms_first": lat[0],
                "append_ms_last": lat[-1], "append_ms_median": float(np.median(lat)), "equal_to_one_shot": same,
                "appends_per_edge": paths[0], "appends_recount": paths[1]})
    total_pe, lat_pe, _, _ = run("per_edge")
    res.update({"per_edge_total_ms": 1e3 * total_pe, "per_edge_append_ms_first": lat_pe[0],
                "per_edge_append_ms_last": lat_pe[-1]})
    return res


def bench_batched(dev, reps: int = 3):
    """512 jobs (256 independent Chung-Lu streams, 10k-2M edges log-uniform, plus 256 hash-seed
    replicas of one 5M-edge stream), m = c = 20: one rept_count per job (plain) against one
    autotuned, graph-captured launch of all jobs (batched).  Outputs must be identical."""
    import numpy as np
    import torch
    import synth
    from paper_1811_09136_amd import rept
    from paper_1811_09136_amd.batch import Autotuner, Batch, Job, run_plain, time_call

    t_gen = time.perf_counter()
    streams, (rep, rep_n), rep_seeds = synth.batch_jobs(seed=4)
    t_gen = time.perf_counter() - t_gen
    graphs = [rept.Graph(rept.to_device_edges(e, dev), n) for e, n in streams]
    rg = rept.Graph(rept.to_device_edges(rep, dev), rep_n)
    P = lambda s: rept.Params(20, 20, int(s))
    jobs = [Job(g, P(i + 1)) for i, g in enumerate(graphs)] + [Job(rg, P(s)) for s in rep_seeds]
    for j in jobs:
        j.ensure_outputs()
    total = sum(len(e) for e, _ in streams) + len(rep) * len(rep_seeds)
    run_plain(jobs)
    plain_s = min(time_call(run_plain, jobs) for _ in range(reps))
    ref = [(j.out[0].clone(), j.out[1].clone()) for j in jobs]
    tuner = Autotuner(reps=2)
    shape = tuner.best(jobs)
    b = Batch(jobs, rept.tuning(**shape) if shape else None)
    b.capture()
    batched_s = min(time_call(b.replay) for _ in range(reps))
    same = all(torch.equal(j.out[0], g) and torch.equal(j.out[1], l) for j, (g, l) in zip(jobs, ref))
    # replica statistics (Theorem 3 with c = m: Var = tau (m - 1))
    tau = int(rg.count(rept.Params(1, 1, 0))[0].item())
    ests = np.array([rept.rept_estimate(rep_n, j.params, j.out[0].cpu().numpy(), None)[0]
                     for j in jobs[len(streams):]])
    nrmse = float(np.sqrt(np.mean((ests - tau) ** 2)) / tau)
    for g in graphs:
        g.close()
    rg.close()
    return {"workload": "256 Chung-Lu streams (1e4-2e6 edges, log-uniform) + 256 hash-seed replicas of a 5e6-edge "
                        "stream, m=c=20",
            "jobs": len(jobs), "stream_edges": int(total),
            "plain_edges_per_s": total / plain_s, "batched_edges_per_s": total / batched_s,
            "speedup": plain_s / batched_s, "plain_ms": 1e3 * plain_s, "batched_ms": 1e3 * batched_s,
            "identical_outputs": bool(same), "tuned_shape": shape, "generation_s": t_gen,
            "replicas": {"R": len(ests), "tau": tau, "mean_tau_hat": float(ests.mean()),
                         "nrmse": nrmse, "nrmse_theory": float(np.sqrt(19.0 / tau))}}


def bench_served(dev, n_requests: int = 256, mults=(0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0)):
    """Poisson arrivals of count requests (lognormal sizes, median 2e5 edges, clipped to [1e3,
    2e7]; m in {10, 50, 100}, c in {m, 4m}), plus one request at the size limit of 2e7 edges in the
    middle of the trace (a lognormal draw reaches it with probability ~1e-6, so 256 draws would not
    show the tail); continuous batching against a FIFO plain loop at arrival rates swept around the
    plain loop's saturation rate."""
    import numpy as np
    import synth
    from paper_1811_09136_amd.serve import DeviceExecutor, Request, Server, run_fifo_plain, summarize

    tr = synth.serving_trace(seed=5, n_requests=n_requests, rate_per_s=1.0)
    tail = dict(tr[n_requests // 2])
    tail["E"], tail["n"] = 20_000_000, 1_000_000
    tr = tr[:n_requests // 2] + [tail] + tr[n_requests // 2:]
    gaps = np.diff([0.0] + [r["arrival_s"] for r in tr])
    graphs = [synth.scaled_chung_lu(r["E"], r["graph_seed"] % (2**31)) for r in tr]
    import torch
    free = torch.cuda.mem_get_info(dev)[0]
    budget = int(0.5 * free)
    # both loops take their buffers from one arena of the budget's size, reserved up front
    ex = DeviceExecutor(dev, arena_bytes=budget)

    def requests(rate):
        arr = np.cumsum(gaps) / rate
        return [Request(i, float(arr[i]), e, n, r["m"], r["c"], r["hash_seed"])
                for i, ((e, n), r) in enumerate(zip(graphs, tr))]

    run_fifo_plain(ex, requests(1e9)[:4])  # warm-up
    sat = run_fifo_plain(ex, requests(1e9))  # everything at t = 0: service rate of the plain loop
    mu = len(tr) / (max(r.done_s for r in sat) - min(r.arrival_s for r in sat))
    sweep = []
    for mult in mults:
        reqs = requests(mult * mu)
        fifo = summarize(run_fifo_plain(ex, reqs), reqs)
        srv = Server(ex, budget_bytes=budget, max_active=64, chunk_units=1 << 16, build_workers=4,
                     finish_workers=2, max_inflight=2)
        served = summarize(srv.run(reqs), reqs)
        sweep.append({"rate_per_s": mult * mu, "rate_x_plain_saturation": mult, "fifo_plain": fifo,
                      "served": served, "served_over_fifo_edges_per_s": served["edges_per_s"] / fifo["edges_per_s"]})
    return {"workload": f"{n_requests} Poisson requests, lognormal edges (median 2e5, clipped to [1e3, 2e7]), plus "
                        "one 2e7-edge request mid-trace; m in {10,50,100}, c in {m,4m}",
            "requests": len(tr), "plain_saturation_req_per_s": mu, "hbm_budget_bytes": budget,
            "total_edges": int(sum(len(e) for e, _ in graphs)), "sweep": sweep}


def measure_plain(dev, workload: str, steps: int, warmup: int, host_input: bool = True) -> dict:
    """Time `steps` whole-path steps (after `warmup`) of one workload resident in HBM, then the
    counting kernel alone for the roofline; returns the figures of the JSON line."""
    import numpy as np
    import torch
    from paper_1811_09136_amd import rept

    desc, _, n, m, c = WORKLOADS[workload]
    edges = stream_for(workload)
    E = len(edges)
    say(f"workload {workload}: n={n} E={E} m={m} c={c}")
    params = rept.Params(m, c, HASH_SEED)
    rows = params.rows
    d_edges = rept.to_device_edges(edges, dev)
    pbytes, sbytes = rept.rept_query_sizes(n, E)
    persistent = torch.empty(pbytes, dtype=torch.uint8, device=dev)
    scratch = torch.empty(sbytes, dtype=torch.uint8, device=dev)
    glob = torch.empty(c, dtype=torch.int64, device=dev)
    loc = torch.empty((rows, n), dtype=torch.int64, device=dev)
    sums = torch.empty(n, dtype=torch.int64, device=dev)
    h_glob = torch.empty(c, dtype=torch.int64, pin_memory=True)
    h_sums = torch.empty(n, dtype=torch.int64, pin_memory=True)
    h_tau_v = np.zeros(n, dtype=np.float64)  # local estimators, written by rept_estimate
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    # the count workspace (slot table) depends on the built graph's size: size it once
    h = rept.rept_build(n, d_edges.data_ptr(), E, persistent.data_ptr(), pbytes, scratch.data_ptr(), sbytes, sp)
    wbytes = max(rept.rept_count_workspace_size(h, params), rept.rept_count_workspace_size(h, rept.Params(1, 1, 0)))
    rept.rept_destroy(h)
    ws = torch.empty(wbytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    count_ms = []
    build_ms = []
    reduce_d2h_ms = []
    estimate_ms = []

    def step(record):
        t0 = time.perf_counter()
        h = rept.rept_build(n, d_edges.data_ptr(), E, persistent.data_ptr(), pbytes, scratch.data_ptr(), sbytes, sp)
        t1 = time.perf_counter()  # rept_build synchronises its stream once (validation result)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        rept.rept_count(h, params, glob.data_ptr(), loc.data_ptr(), ws.data_ptr(), wbytes, sp)
        ev1.record(stream)
        rept.rept_reduce_local(loc.data_ptr(), rows, n, sums.data_ptr(), sp)
        h_glob.copy_(glob, non_blocking=True)
        h_sums.copy_(sums, non_blocking=True)
        ev2 = torch.cuda.Event(enable_timing=True)
        ev2.record(stream)
        stream.synchronize()
        t2 = time.perf_counter()
        tau_hat, tau_v = rept.rept_estimate_sums(n, params, h_glob.numpy(), h_sums.numpy(), h_tau_v)
        t3 = time.perf_counter()
        info = rept.rept_graph_get_info(h)
        rept.rept_destroy(h)
        if record:
            count_ms.append(ev0.elapsed_time(ev1))
            build_ms.append(1e3 * (t1 - t0))
            reduce_d2h_ms.append(ev1.elapsed_time(ev2))
            estimate_ms.append(1e3 * (t3 - t2))
        return tau_hat, info

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tau_hat, info = step(True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / steps
    value = E * steps / dt
    say(f"{workload}: timed {steps} steps: {ms_per_step:.2f} ms/step, count {sum(count_ms) / len(count_ms):.3f} ms")

    # the counting kernel alone, for the roofline: one job whose slot table an earlier launch
    # wrote (REPT_JOB_TABLE_READY), so a launch runs setup, the output clear and k_count only;
    # HIP events on the stream the kernels are launched on
    h = rept.rept_build(n, d_edges.data_ptr(), E, persistent.data_ptr(), pbytes, scratch.data_ptr(), sbytes, sp)
    bw = rept.rept_batch_workspace_size(1)
    ws_fill = torch.empty(bw, dtype=torch.uint8, device=dev)
    ws_ready = torch.empty(bw, dtype=torch.uint8, device=dev)
    job = rept.rept_job(h, params.c_struct(), glob.data_ptr(), loc.data_ptr(), 0, rept.UINT64_MAX, 0,
                        rept.UINT32_MAX, 0, 0, ws.data_ptr(), wbytes)
    rept.rept_batch_prepare([job], None, ws_fill.data_ptr(), bw, sp)
    job.flags = rept.REPT_JOB_TABLE_READY
    rept.rept_batch_prepare([job], None, ws_ready.data_ptr(), bw, sp)
    rept.rept_batch_launch(ws_fill.data_ptr(), sp)
    rept.rept_batch_launch(ws_ready.data_ptr(), sp)  # warm
    kernel_ms = []
    for _ in range(max(3, steps)):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        rept.rept_batch_launch(ws_ready.data_ptr(), sp)
        ev1.record(stream)
        stream.synchronize()
        kernel_ms.append(ev0.elapsed_time(ev1))
    if not np.array_equal(glob.cpu().numpy(), h_glob.numpy()):
        raise RuntimeError("kernel-only launches disagree with the timed steps")

    # PCIe-inclusive steps (not `value`): the stream starts in pinned host memory and
    # rept_build_host copies it in; the rest of the step as above
    host_step_ms = None
    ref_glob = h_glob.numpy().copy()  # the timed steps' global counters
    if host_input:
        say(f"{workload}: host-input steps")
        h_edges = torch.from_numpy(np.ascontiguousarray(edges, dtype=np.uint32)).pin_memory().numpy()
        host_ms = []
        for r in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hh = rept.rept_build_host(n, h_edges, persistent.data_ptr(), pbytes, scratch.data_ptr(), sbytes, sp)
            rept.rept_count(hh, params, glob.data_ptr(), loc.data_ptr(), ws.data_ptr(), wbytes, sp)
            rept.rept_reduce_local(loc.data_ptr(), rows, n, sums.data_ptr(), sp)
            h_glob.copy_(glob, non_blocking=True)
            h_sums.copy_(sums, non_blocking=True)
            stream.synchronize()
            rept.rept_estimate_sums(n, params, h_glob.numpy(), h_sums.numpy(), h_tau_v)
            rept.rept_destroy(hh)
            if r:
                host_ms.append(1e3 * (time.perf_counter() - t0))
        del h_edges
        if not np.array_equal(h_glob.numpy(), ref_glob):
            raise RuntimeError("host-input step disagrees with the device-input steps")
        host_step_ms = float(np.median(host_ms))

    # exact triangle count (m = 1, untimed) for the per-launch byte model
    p1 = rept.Params(1, 1, 0)
    g1 = torch.empty(1, dtype=torch.int64, device=dev)
    l1 = torch.empty((1, n), dtype=torch.int64, device=dev)
    rept.rept_count(h, p1, g1.data_ptr(), l1.data_ptr(), ws.data_ptr(), wbytes, sp)
    torch.cuda.synchronize()
    tau = int(g1.item())
    rept.rept_destroy(h)

    avg_count_ms = float(np.median(count_ms))
    avg_kernel_ms = float(np.median(kernel_ms))
    alg = algorithmic_bytes(info, tau, c, rows, n)
    achieved = alg / (avg_kernel_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(workload)
    deg = np.bincount(edges.ravel(), minlength=n).astype(np.int64)
    W = int((deg * (deg - 1) // 2).sum())
    semi = int(ref_glob.sum())
    sm_bytes = streaming_model_bytes(W, E, params.groups, semi, c, n)
    # context: the bytes an id-sorted merge of the per-group CSR segments would read,
    # 8 sum_k sum_x d_x d_x^act, with d_x^act = d_x for a full group and its expectation
    # d_x c2 / m for a partial last group
    csr_bytes = 8.0 * float((deg * deg).sum()) * (c // m + (c % m) / m)
    return {
        "edges": edges, "n": n, "m": m, "c": c, "ref_glob": ref_glob,
        "value": value, "ms_per_step": ms_per_step,
        "config": {"workload": desc, "n": n, "edges": E, "m": m, "c": c, "hash_seed": HASH_SEED},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic},
        "kernel": {"count_ms": avg_count_ms, "count_kernel_ms": avg_kernel_ms, "build_ms": float(np.median(build_ms)),
                   "count_edges_per_s": E / (avg_count_ms * 1e-3), "algorithmic_bytes": alg,
                   "oriented_work": int(info.oriented_work), "num_reverse": int(info.num_reverse), "triangles": tau,
                   "semi_triangles": semi,
                   "streaming_model_bytes": sm_bytes,
                   "streaming_model_equiv_gbps": sm_bytes / (avg_kernel_ms * 1e-3) / 1e9,
                   "reduce_d2h_ms": float(np.median(reduce_d2h_ms)), "estimate_ms": float(np.median(estimate_ms)),
                   "stream_edge_processors_per_s": value * c,
                   "traffic_frac": None if traffic is None else traffic / (avg_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                   "traffic_over_algorithmic": None if traffic is None else traffic / alg,
                   "csr_merge_bytes": csr_bytes,
                   "host_input_step_ms": host_step_ms,
                   "host_input_edges_per_s": None if host_step_ms is None else E / (host_step_ms * 1e-3),
                   "traffic_over_csr_merge": None if traffic is None else traffic / csr_bytes,
                   "source_digest": count_kernel_source_digest()},
        "tau_hat": tau_hat,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design note, "
                                   "run with --gpus 1"}))
        sys.exit(2)
    import torch

    dev = torch.device("cuda:0")
    head = measure_plain(dev, args.workload, args.steps, args.warmup)
    if args.copy_calibration:  # a plain device copy of 1 GiB, for counter scaling
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    out = {
        "metric": "stream edges/sec on 1 GPU, % HBM roofline; batched/served vs plain",
        "value": head["value"],
        "unit": "stream edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "kernel": head["kernel"],
        "tau_hat": head["tau_hat"],
    }
    # the other single-stream workload and the "next" rows on the 1M/20M power-law stream
    side = head if args.workload == SIDE_WORKLOAD else None
    if not args.no_side and side is None:
        say(f"side workload {SIDE_WORKLOAD}")
        side = measure_plain(dev, SIDE_WORKLOAD, args.steps, min(args.warmup, 3), host_input=False)
        out[SIDE_WORKLOAD] = {k: side[k] for k in ("value", "ms_per_step", "config", "roofline", "kernel", "tau_hat")}
    if side is not None:
        edges, n, m, c = side["edges"], side["n"], side["m"], side["c"]
        if not args.no_alg2 and c > m:
            say("algorithm 2 pass")
            out["alg2"] = bench_alg2(dev, edges, n, m, c - m // 2)
        if not args.no_mascot and m > 1:
            say("parallel MASCOT pass")
            out["mascot"] = bench_mascot(dev, edges, n, m, min(c, 8))
        if not args.no_incremental:
            say("incremental stream")
            out["incremental"] = bench_incremental(dev, edges, n, m, c, side["ref_glob"])
    if not args.no_batched:
        say("batched workload")
        out["batched"] = bench_batched(dev)
    if not args.no_served:
        say("served workload")
        out["served"] = bench_served(dev)
    if not args.no_cpu:
        say("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(head["edges"], head["n"], head["m"], head["c"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
