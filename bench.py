#!/usr/bin/env python3
"""Benchmark: task-DAG dependencies (edges) partitioned per second on one MI355X.

Workload (one step): the two-way CPU:GPU partition (ratio 1:3, eps 5 %) of a
random layered task DAG with 4,000,000 vertices in 64 layers (Poisson(4)
out-edges to the next 1-3 layers, lognormal(8, 1) costs, GPU cost = CPU
cost / 3, lognormal(16, 1.5) bytes per dependency; 15,748,986 dependencies
after merging).  Each step is one gp_partition call on the device-resident
graph (handed to gp_create beforehand; its time is reported as create_ms).

Secondary numbers in the same line: the tiled Cholesky T=64 + LU T=48 step
(1:4, 3 %), the 4,096-graph batch, the learned proposal against the plain
bisection, and the host-memory end-to-end time (PCIe included).

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import ctypes
import glob
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DAG edges/sec partitioned on 1 MI355X vs CPU oracle; cut bytes; % HBM peak"
HBM_PEAK_GBS = 8000.0
L4M_OPTS = dict(ratio=(1, 3), eps_ppm=50000)
STEP2_OPTS = dict(ratio=(1, 4), eps_ppm=30000)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ensure_built():
    if not all(os.path.exists(os.path.join(ROOT, p)) for p in (
            "paper_1502_07451_amd/libgp.so", "dagen/libdagen.so")):
        import __graft_entry__
        __graft_entry__.build()


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_1502_07451_amd", "csrc", "*"))):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or the kernel sources have changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        kv = dict(l.split(" = ", 1) for l in f.read().splitlines() if " = " in l)
    if kv.get("kernel") != kernel or kv.get("source_sha256") != kernel_sources_sha256():
        return None
    return int(kv["traffic_bytes_per_launch"])


def aggregate(rows_lists):
    agg = {}
    for rows in rows_lists:
        for r in rows:
            a = agg.setdefault(r["name"], dict(launches=0, executed=0, ms=0.0, bytes=0.0))
            for k in ("launches", "executed", "ms", "bytes"):
                a[k] += r[k]
    return agg


def profile_table(agg, reps):
    total_ms = sum(a["ms"] for a in agg.values())
    log(f"{'kernel':28s} {'launch':>7s} {'exec':>6s} {'ms/step':>9s} {'share':>6s} {'GB/s':>8s}")
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["ms"]):
        gbs = a["bytes"] / (a["ms"] * 1e-3) / 1e9 if a["ms"] > 0 and a["bytes"] > 0 else 0.0
        log(f"{name:28s} {a['launches'] // reps:7d} {a['executed'] // reps:6d} "
            f"{a['ms'] / reps:9.4f} {a['ms'] / total_ms:6.1%} {gbs:8.1f}")
    return total_ms


def roofline_of(agg, workload):
    """The kernel with the largest summed time among those whose algorithmic
    bytes are defined: achieved = bytes per launch / average launch time."""
    total_ms = sum(a["ms"] for a in agg.values())
    cand = {k: v for k, v in agg.items() if v["bytes"] > 0 and v["executed"] > 0}
    name, dom = max(cand.items(), key=lambda kv: kv[1]["ms"])
    # bytes are counted for launches that did their work; time over all of them
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    base = name.split("<")[0]
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": measured_traffic(base, workload), "kernel": name,
            "launches_per_step": None, "avg_launch_us": round(avg_ms * 1e3, 3),
            "alg_bytes_per_launch": round(bytes_per_launch),
            "kernel_share_of_step": round(dom["ms"] / total_ms, 4)}
    if base == "k_init_trials":
        roof["limiter"] = ("serial greedy picks: dependent LDS round trips and two block "
                           "barriers per pick, not HBM bandwidth")
    return roof


def batch_timeline(bt, bb, chosen):
    """What sets the batched kernel's time, from the per-graph start and end
    ticks of the last call: the span, how long every workgroup stayed busy,
    the tail after the first one ran dry, and the graphs that finished last."""
    import numpy as np
    G = len(bb.voff) - 1
    t, hz = bt.timeline(G)
    t = (t - t[:, 0].min()).astype(np.float64) * 1e3 / hz  # ms from the first start
    span = float(t[:, 1].max())
    # workgroups busy at once: +1 at each start, -1 at each end
    ev = sorted([(a, 1) for a in t[:, 0]] + [(b, -1) for b in t[:, 1]])
    busy, peak = 0, 0
    for x, d in ev:
        busy += d
        peak = max(peak, busy)
    queue_empty = float(t[:, 0].max())  # the last graph is taken
    dur = t[:, 1] - t[:, 0]
    n = np.diff(bb.voff)
    last = np.argsort(t[:, 1])[-5:][::-1]
    big = n >= np.percentile(n, 90)
    return {"span_ms": round(span, 3), "workgroups_busy": int(peak),
            "queue_empty_ms": round(queue_empty, 3),
            "tail_ms": round(span - queue_empty, 3),
            "graph_ms_p50": round(float(np.median(dur)), 3),
            "graph_ms_max": round(float(dur.max()), 3),
            "largest_decile_graph_ms_mean": round(float(dur[big].mean()), 3),
            "last_finished": [{"graph": int(g), "vertices": int(n[g]),
                               "ms": round(float(dur[g]), 3),
                               "end_ms": round(float(t[g, 1]), 3)} for g in last],
            "sum_graph_ms_over_workgroups": round(float(dur.sum()) / max(peak, 1), 3)}


def cpu_model_name() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def copy_probe(torch, dev, mib):
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: 3 copies of {mib} MiB")


def step2_secondary(gp, dagen, torch, dev, args):
    """The tiled Cholesky T=64 + LU T=48 DAGs (1:4, 3 %), both partitioned
    concurrently, each on its own stream and host thread."""
    graphs = dagen.config_cholesky64_lu48()
    edges = sum(g.m for g in graphs)
    arrays = [gp.to_device(g, dev) for g in graphs]
    streams = [torch.cuda.Stream(device=dev) for _ in graphs]
    torch.cuda.synchronize()
    handles = [gp.Graph(*a, stream=ctypes.c_void_p(s.cuda_stream))
               for a, s in zip(arrays, streams)]
    opts = gp.options(**STEP2_OPTS)
    parts = [torch.empty(g.n, dtype=torch.int8, device=dev) for g in graphs]
    torch.cuda.synchronize()
    results = [None] * len(graphs)
    pool = concurrent.futures.ThreadPoolExecutor(max_workers=len(graphs))

    def run_one(i):
        _, results[i] = handles[i].partition(opts, part=parts[i])

    def step():
        for f in [pool.submit(run_one, i) for i in range(len(graphs))]:
            f.result()

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    for h in handles:
        h.profile(True)
    for _ in range(5):
        for i in range(len(graphs)):
            run_one(i)
    torch.cuda.synchronize()
    agg = aggregate([h.profile_read(reset=True) for h in handles])
    for h in handles:
        h.profile(False)
        h.close()
    pool.shutdown()
    out = {"workload": "tiled Cholesky T=64 (45,760 tasks, 131,040 deps) + tiled LU T=48 "
                       "(38,024 tasks, 109,416 deps), 1024x1024 tiles, +-10% jitter, 8 MiB/dep, "
                       "1:4, eps 3%, concurrent streams",
           "edges": edges, "ms": round(ms, 4), "edges_per_s": round(edges / (ms / 1e3), 1),
           "cut": [r.cut for r in results], "feasible": [r.feasible for r in results],
           "levels": [r.levels for r in results],
           "roofline": roofline_of(agg, "cholesky64_lu48")}
    parity = None
    if not args.no_cpu:
        import numpy as np
        import oracle
        oo = oracle.Options(**STEP2_OPTS)
        t0 = time.perf_counter()
        refs = [oracle.partition(g, oo) for g in graphs]
        tc = time.perf_counter() - t0
        parity = all(bool(np.array_equal(p.cpu().numpy(), r.part)) and res.cut == r.cut
                     for p, r, res in zip(parts, refs, results))
        out["cpu_oracle_1thread_ms"] = round(tc * 1e3, 1)
    out["parity_with_oracle"] = parity
    return out, graphs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle runs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary workloads (Cholesky/LU step, batch, learned)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only warmup + timed steps of the headline workload (profiler runs)")
    ap.add_argument("--layered4m-kernels", action="store_true",
                    help="only two partitions of the 4M-vertex layered DAG (counter runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run 3 device copies of MIB MiB (the reference kernel that "
                         "scales rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build partitions on one GPU only; --gpus {args.gpus} "
              f"(WORLD_SIZE {world}) is not supported", file=sys.stderr)
        sys.exit(2)

    ensure_built()
    import numpy as np
    import torch

    import dagen
    import paper_1502_07451_amd as gp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g4 = dagen.config_layered4m()
    log(f"layered4m: n={g4.n} edges={g4.m}")
    arrays = gp.to_device(g4, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h4 = gp.Graph(*arrays)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    del arrays
    p4 = torch.empty(g4.n, dtype=torch.int8, device=dev)
    o4 = gp.options(**L4M_OPTS)
    if args.layered4m_kernels:
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r4 = h4.partition(o4, part=p4)
            torch.cuda.synchronize()
            log(f"layered4m partition: {(time.perf_counter() - t0) * 1e3:.3f} ms, cut {r4.cut}")
        if args.copy_probe > 0:
            copy_probe(torch, dev, args.copy_probe)
        h4.close()
        return

    for _ in range(args.warmup):
        _, r4 = h4.partition(o4, part=p4)
    torch.cuda.synchronize()
    step_ms = []
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        _, r4 = h4.partition(o4, part=p4)
        step_ms.append((time.perf_counter() - t0) * 1e3)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t_all) * 1e3 / max(args.steps, 1)
    value = g4.m / (ms_per_step / 1e3)
    log(f"{args.steps} steps, {ms_per_step:.3f} ms/step (median {statistics.median(step_ms):.3f}),"
        f" {value:.4g} edges/s")
    if args.copy_probe > 0:
        copy_probe(torch, dev, args.copy_probe)
    if args.kernels_only:
        h4.close()
        return

    # roofline: the same step again with HIP events around every launch on
    # the handle's stream
    h4.profile(True)
    prof_steps = 3
    for _ in range(prof_steps):
        h4.partition(o4, part=p4)
    torch.cuda.synchronize()
    agg = aggregate([h4.profile_read(reset=True)])
    h4.profile(False)
    profile_table(agg, prof_steps)
    roofline = roofline_of(agg, "layered4m")
    roofline["launches_per_step"] = agg[roofline["kernel"]]["launches"] // prof_steps

    # algorithmic bytes of the whole step at one matching round and one
    # refinement pass per level: per level S = 4(n+1) + 12*2m + 16n read by
    # matching, contraction and refinement, the next level written once, plus
    # match, cmap and part (10 B per vertex)
    _, _, tr4 = h4.partition(o4, part=p4, trace_cap=64)
    S = [4 * (int(r[0]) + 1) + 12 * int(r[1]) + 16 * int(r[0]) for r in tr4]
    b_alg = sum(3 * S[l] + (S[l + 1] if l + 1 < len(S) else 0) + 10 * int(tr4[l][0])
                for l in range(len(S) - 1))
    with open(os.path.join(ROOT, "tests", "golden", "layered4m_1to3_eps5.txt")) as f:
        exp = dict(l.split("=", 1) for l in f.read().split("\n") if "=" in l)
    got4 = p4.cpu().numpy()
    digest = hashlib.sha256(got4.tobytes()).hexdigest()

    out = {"metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic",
           "config": {"workload": "layered4m: random layered task DAG, 4,000,000 vertices in 64 "
                                  "layers, Poisson(4) out-edges to the next 1-3 layers, "
                                  "lognormal(8,1) costs (GPU = CPU/3), lognormal(16,1.5) "
                                  "bytes/dep, seed 0",
                      "vertices": g4.n, "edges_per_step": g4.m, "ratio": "1:3",
                      "eps_ppm": 50000, "parallelism": "single GPU"},
           "cut": r4.cut, "load": [r4.load[0], r4.load[1]], "time": [r4.time[0], r4.time[1]],
           "feasible": r4.feasible, "levels": r4.levels,
           "median_step_ms": round(statistics.median(step_ms), 4),
           "create_ms": round(create_ms, 3),
           "matches_oracle_digest": digest == exp.get("part_sha256")
           and r4.cut == int(exp.get("cut", -1)),
           "alg_bytes_per_step": b_alg,
           "alg_bytes_frac_of_hbm_peak": round(b_alg / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS,
                                               5),
           "roofline": roofline}

    # CPU baseline: the serial oracle on the same workload, one thread, one
    # whole partition (the unit of the metric)
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.partition(g4, oracle.Options(**L4M_OPTS))
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(g4.m / tc, 1), "unit": "edges/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one whole partition of the 4M-vertex layered DAG, "
                                         f"single-threaded: {tc:.1f} s",
                               "cpu_model": cpu_model_name(), "nproc": os.cpu_count()}
        out["parity_with_oracle"] = bool(np.array_equal(got4, ref.part)) and r4.cut == ref.cut \
            and (r4.load[0], r4.load[1]) == ref.load
        del ref
    h4.close()
    del p4

    # host memory in and out (PCIe included): gp_create from host arrays,
    # partition, assignment back to the host
    if not args.no_extra:
        e2e = []
        xa, ad = np.ascontiguousarray(g4.xadj, np.int32), np.ascontiguousarray(g4.adjncy, np.int32)
        aw = np.ascontiguousarray(g4.adjwgt, np.int64)
        vw = np.ascontiguousarray(g4.vwgt, np.int64).reshape(-1)
        hp = np.empty(g4.n, np.int8)
        for _ in range(3):
            t0 = time.perf_counter()
            hh = gp.Graph(g4.n, xa, ad, aw, vw)
            hh.partition(o4, part=hp)
            hh.close()
            e2e.append(time.perf_counter() - t0)
        te = statistics.median(e2e)
        out["host_end_to_end"] = {"ms": round(te * 1e3, 3), "edges_per_s": round(g4.m / te, 1),
                                  "note": "host arrays in through gp_create, host assignment "
                                          "out (PCIe included), median of 3"}
    del g4

    if not args.no_extra:
        out["cholesky64_lu48"], graphs2 = step2_secondary(gp, dagen, torch, dev, args)

    # batched form: 4,096 uneven DAGs in one persistent launch
    if not args.no_extra:
        graphs_b = dagen.batch(4096, 100, 50000, 0)
        bb = dagen.concat(graphs_b)
        dev_b = gp.batch_to_device(bb, dev)
        pb = torch.empty(int(bb.voff[-1]), dtype=torch.int8, device=dev)
        bt = gp.Batch()
        ob = gp.options(**STEP2_OPTS)
        # the autotuner checks every configuration gives identical bytes and keeps the fastest
        _, resb, chosen, tune_ms = bt.autotune(*dev_b, opts=ob, part=pb, reps=1)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, resb = bt.partition(*dev_b, opts=ob, part=pb)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        tb = statistics.median(times)
        mb = int(bb.eoff[-1]) // 2
        out["batch4096"] = {"graphs": 4096, "vertices": int(bb.voff[-1]), "edges": mb,
                            "ms": round(tb * 1e3, 3), "edges_per_s": round(mb / tb, 1),
                            "cut_sum": int(sum(r.cut for r in resb)),
                            "all_ok": all(r.status == 0 for r in resb),
                            "feasible": int(sum(r.feasible for r in resb)),
                            "autotuned": {"workgroups": chosen[0], "chunk": chosen[1],
                                          "order_mode": chosen[2], "team_width_shift": chosen[3],
                                          "tuning_ms_per_call": round(tune_ms, 3)}}
        out["batch4096"]["timeline"] = batch_timeline(bt, bb, chosen)
        gotb = pb.cpu().numpy()
        bt.close()
        del dev_b, pb
        if not args.no_cpu:
            # the serial oracle over the same graphs, one graph per host thread
            # (the graphs are independent; ctypes releases the GIL); every
            # graph's assignment and result compared
            import oracle
            nthr = min(os.cpu_count() or 1, 16)
            oo_b = oracle.Options(**STEP2_OPTS)
            t0 = time.perf_counter()
            with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
                refs = list(ex.map(lambda g: oracle.partition(g, oo_b), graphs_b))
            tcb = time.perf_counter() - t0
            same = all(np.array_equal(gotb[bb.voff[i]:bb.voff[i + 1]], r.part)
                       and resb[i].cut == r.cut and (resb[i].load[0], resb[i].load[1]) == r.load
                       for i, r in enumerate(refs))
            out["batch4096"]["cpu_oracle_threads"] = {
                "threads": nthr, "ms": round(tcb * 1e3, 1), "edges_per_s": round(mb / tcb, 1)}
            out["batch4096"]["parity_with_oracle"] = bool(same)
            del refs
        del graphs_b

    # learned coarsest-level proposal vs the plain bisection on its evaluation
    # DAGs: the 1M-vertex layered DAG (1:3, 5 %), Cholesky T=64 and LU T=48
    # (1:4, 3 %)
    wpath = os.path.join(ROOT, "paper_1502_07451_amd", "mpnn_weights.bin")
    if not args.no_extra and os.path.exists(wpath):
        from paper_1502_07451_amd import learn
        w = learn.load_weights(wpath)
        out["learned"] = (learn.gain_test(w, [dagen.config_layered1m()], L4M_OPTS, dev, reps=3)
                          + learn.gain_test(w, graphs2, STEP2_OPTS, dev, reps=3))
    # schedule simulation (the paper's runtime comparison): eager, dmda-like
    # and the partition on 3 CPU workers + 1 GPU worker, tiled Cholesky T=16
    # (b = 512, 2 MiB tiles), time unit = one flop at CPU speed, the link
    # moving one byte per unit; GPU speed 4x (small gap) and 50x (large gap)
    if not args.no_extra:
        import numpy as np
        sched = []
        for rate in (4, 50):
            g = dagen.cholesky(16, 512, rate=rate)
            tc, tg = int(g.vwgt[:, 0].sum()) // 3, int(g.vwgt[:, 1].sum())
            _, (r0, r1) = gp.ratio_from_times(tc, tg)
            hg = gp.Graph(g.n, g.xadj, g.adjncy, g.adjwgt, np.ascontiguousarray(g.vwgt))
            part, pres = hg.partition(gp.options(ratio=(r0, r1), eps_ppm=30000))
            hg.close()
            row = {"dag": "cholesky_T16", "gpu_speedup": rate, "ratio": [r0, r1],
                   "gp_cut": pres.cut}
            for name, pol in (("eager", gp.SIM_EAGER), ("dmda", gp.SIM_DMDA), ("gp", gp.SIM_GP)):
                res, _, _ = gp.simulate(g, pol, part=part, ncpu=3, ngpu=1, latency=0, bw=1)
                row[name] = {"makespan": res.makespan, "transfers": res.transfers,
                             "bytes": res.bytes, "tasks_cpu_gpu": [res.tasks[0], res.tasks[1]]}
            sched.append(row)
        out["schedule"] = sched
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
