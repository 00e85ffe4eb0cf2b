#!/usr/bin/env python3
"""Benchmark: task-DAG dependencies (edges) partitioned per second on one MI355X.

Workload (one step): the two-way CPU:GPU partition (ratio 1:4, eps 3 %) of
the tiled Cholesky DAG with T=64 (45,760 tasks, 131,040 dependencies) and the
tiled LU DAG with T=48 (38,024 tasks, 109,416 dependencies), 1024x1024 tiles,
+-10 % per-task cost jitter, 8 MiB per dependency.  Each step calls
gp_partition once per graph on device-resident inputs (the graphs were
handed to gp_create beforehand; its time is reported as create_ms).  The two
calls run concurrently, each on its own stream and host thread.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import ctypes
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ensure_built():
    if not all(os.path.exists(os.path.join(ROOT, p)) for p in (
            "paper_1502_07451_amd/libgp.so", "dagen/libdagen.so")):
        import __graft_entry__
        __graft_entry__.build()


KERNEL_SOURCES = ("gp_dev.h", "gp_internal.h", "gp_kernels.hip", "gp_phases.h")


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or the kernel sources have changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_cholesky64_lu48_traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        kv = dict(l.split(" = ", 1) for l in f.read().splitlines() if " = " in l)
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1502_07451_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if kv.get("kernel") != kernel or kv.get("source_sha256") != h.hexdigest():
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 4M-vertex layered DAG and the 4,096-graph batch")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only warmup + timed steps (for profiler runs)")
    ap.add_argument("--layered4m-kernels", action="store_true",
                    help="only two partitions of the 4M-vertex layered DAG (for counter runs)")
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
    if args.layered4m_kernels:
        g4 = dagen.config_layered4m()
        h4 = gp.create(g4, dev)
        p4 = torch.empty(g4.n, dtype=torch.int8, device=dev)
        o4 = gp.options(ratio=(1, 3), eps_ppm=50000)
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r4 = h4.partition(o4, part=p4)
            torch.cuda.synchronize()
            log(f"layered4m partition: {(time.perf_counter() - t0) * 1e3:.3f} ms, cut {r4.cut}")
        if args.copy_probe > 0:
            src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            log(f"copy probe: 3 copies of {args.copy_probe} MiB")
        h4.close()
        return
    graphs = dagen.config_cholesky64_lu48()
    edges = sum(g.m for g in graphs)
    dev_arrays = [gp.to_device(g, dev) for g in graphs]
    torch.cuda.synchronize()
    # the DAGs of a step are independent: each has its own HIP stream (default
    # priority) and host thread, so their latency-bound levels overlap
    streams = [torch.cuda.Stream(device=dev) for _ in graphs]
    t0 = time.perf_counter()
    handles = [gp.Graph(*a, stream=ctypes.c_void_p(s.cuda_stream))
               for a, s in zip(dev_arrays, streams)]
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    opts = gp.options(ratio=(1, 4), eps_ppm=30000)
    parts = [torch.empty(g.n, dtype=torch.int8, device=dev) for g in graphs]
    torch.cuda.synchronize()
    results = [None] * len(graphs)
    pool = concurrent.futures.ThreadPoolExecutor(max_workers=len(graphs))

    def run_one(i):
        _, results[i] = handles[i].partition(opts, part=parts[i])

    def step():
        for f in [pool.submit(run_one, i) for i in range(len(graphs))]:
            f.result()

    def step_serial():
        for i in range(len(graphs)):
            run_one(i)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    value = edges / (ms_per_step / 1e3)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {args.copy_probe} MiB")
        del src, dst
    if args.kernels_only:
        log(f"{args.steps} steps, {ms_per_step:.3f} ms/step, {value:.4g} edges/s")
        return

    # roofline: the same steps again with HIP events around every launch
    for h in handles:
        h.profile(True)
    prof_steps = max(3, min(args.steps, 10))
    for _ in range(prof_steps):
        step_serial()
    torch.cuda.synchronize()
    agg = aggregate([h.profile_read(reset=True) for h in handles])
    for h in handles:
        h.profile(False)
    total_ms = sum(a["ms"] for a in agg.values())
    log(f"{'kernel':28s} {'launch':>7s} {'exec':>6s} {'ms/step':>9s} {'share':>6s} {'GB/s':>8s}")
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1]["ms"]):
        gbs = a["bytes"] / (a["ms"] * 1e-3) / 1e9 if a["ms"] > 0 and a["bytes"] > 0 else 0.0
        log(f"{name:28s} {a['launches'] // prof_steps:7d} {a['executed'] // prof_steps:6d} "
            f"{a['ms'] / prof_steps:9.4f} {a['ms'] / total_ms:6.1%} {gbs:8.1f}")
    # dominant kernel among those whose algorithmic bytes are defined
    cand = {k: v for k, v in agg.items() if v["bytes"] > 0}
    dom_name, dom = max(cand.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom_name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": dom_name, "avg_launch_us": round(avg_ms * 1e3, 3),
                "alg_bytes_per_launch": round(bytes_per_launch),
                "kernel_share_of_step": round(dom["ms"] / total_ms, 4)}
    if dom_name == "k_init_trials":
        # what bounds it: one vertex per step of a serial chain
        roofline["limiter"] = ("serial greedy picks: dependent LDS round trips and two "
                               "block barriers per pick, not HBM bandwidth")

    out = {"metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic",
           "config": {"workload": "cholesky64+lu48: tiled Cholesky T=64 (45,760 tasks, "
                                  "131,040 deps) + tiled LU T=48 (38,024 tasks, 109,416 deps), "
                                  "1024x1024 tiles, +-10% jitter, 8 MiB/dep",
                      "ratio": "1:4", "eps_ppm": 30000, "edges_per_step": edges,
                      "parallelism": "single GPU"},
           "cut": [r.cut for r in results],
           "load": [[r.load[0], r.load[1]] for r in results],
           "feasible": [r.feasible for r in results],
           "levels": [r.levels for r in results],
           "create_ms": round(create_ms, 3),
           "roofline": roofline}

    # secondary: end to end from host memory (gp_create over PCIe, partition,
    # assignment back to the host), one DAG after the other
    if not args.no_extra:
        e2e = []
        for _ in range(3):
            t0 = time.perf_counter()
            for g in graphs:
                hh = gp.Graph(g.n, np.ascontiguousarray(g.xadj, np.int32),
                              np.ascontiguousarray(g.adjncy, np.int32),
                              np.ascontiguousarray(g.adjwgt, np.int64),
                              np.ascontiguousarray(g.vwgt, np.int64).reshape(-1))
                hp = np.empty(g.n, np.int8)
                hh.partition(opts, part=hp)
                hh.close()
            e2e.append(time.perf_counter() - t0)
        te = statistics.median(e2e)
        out["host_end_to_end"] = {"ms": round(te * 1e3, 3), "edges_per_s": round(edges / te, 1),
                                  "note": "host arrays in, host assignment out, serial"}

    # larger single-graph case: the 4M-vertex layered DAG
    if not args.no_extra:
        g4 = dagen.config_layered4m()
        h4 = gp.create(g4, dev)
        p4 = torch.empty(g4.n, dtype=torch.int8, device=dev)
        o4 = gp.options(ratio=(1, 3), eps_ppm=50000)
        _, r4 = h4.partition(o4, part=p4)
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r4 = h4.partition(o4, part=p4)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t4 = statistics.median(times)
        # algorithmic bytes of the pipeline at one matching round and one
        # refinement pass per level: per level S = 4(n+1) + 12*2m + 16n read by
        # matching, contraction and refinement, the next level written once,
        # plus match, cmap and part (10 B per vertex)
        _, _, tr4 = h4.partition(o4, part=p4, trace_cap=64)
        S = [4 * (int(r[0]) + 1) + 12 * int(r[1]) + 16 * int(r[0]) for r in tr4]
        b_alg = sum(3 * S[l] + (S[l + 1] if l + 1 < len(S) else 0) + 10 * int(tr4[l][0])
                    for l in range(len(S) - 1))
        exp = {}
        gpath = os.path.join(ROOT, "tests", "golden", "layered4m_1to3_eps5.txt")
        with open(gpath) as f:
            exp = dict(l.split("=", 1) for l in f.read().split("\n") if "=" in l)
        digest = hashlib.sha256(p4.cpu().numpy().tobytes()).hexdigest()
        out["layered4m"] = {"edges": g4.m, "ms": round(t4 * 1e3, 3),
                            "edges_per_s": round(g4.m / t4, 1), "cut": r4.cut,
                            "levels": r4.levels,
                            "matches_oracle_digest": digest == exp.get("part_sha256")
                            and r4.cut == int(exp.get("cut", -1)),
                            "alg_bytes": b_alg,
                            "alg_bytes_frac_of_hbm_peak": round(b_alg / t4 / 1e9 / HBM_PEAK_GBS, 5)}
        h4.close()
        del p4

    # batched form: 4,096 uneven DAGs in one persistent launch
    if not args.no_extra:
        graphs_b = dagen.batch(4096, 100, 50000, 0)
        bb = dagen.concat(graphs_b)
        dev_b = gp.batch_to_device(bb, dev)
        pb = torch.empty(int(bb.voff[-1]), dtype=torch.int8, device=dev)
        bt = gp.Batch()
        ob = gp.options(ratio=(1, 4), eps_ppm=30000)
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
                                          "order_mode": chosen[2],
                                          "tuning_ms_per_call": round(tune_ms, 3)}}
        bt.close()
        del dev_b, pb
        if not args.no_cpu:
            # the serial oracle over the same 4,096 graphs, one graph per host
            # thread (the graphs are independent; ctypes releases the GIL)
            import oracle
            nthr = min(os.cpu_count() or 1, 16)
            oo_b = oracle.Options(ratio=(1, 4), eps_ppm=30000)
            t0 = time.perf_counter()
            with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
                cuts = list(ex.map(lambda g: oracle.partition(g, oo_b).cut, graphs_b))
            tcb = time.perf_counter() - t0
            out["batch4096"]["cpu_oracle_threads"] = {
                "threads": nthr, "ms": round(tcb * 1e3, 1), "edges_per_s": round(mb / tcb, 1),
                "cut_sum_equal": int(sum(cuts)) == out["batch4096"]["cut_sum"]}
        del graphs_b

    # learned coarsest-level proposal vs the plain bisection on the step's DAGs
    wpath = os.path.join(ROOT, "paper_1502_07451_amd", "mpnn_weights.bin")
    if not args.no_extra and os.path.exists(wpath):
        from paper_1502_07451_amd import learn
        out["learned"] = learn.gain_test(learn.load_weights(wpath), graphs,
                                         dict(ratio=(1, 4), eps_ppm=30000), dev, reps=3)

    # CPU baseline: the serial oracle on the same workload, on the host
    if not args.no_cpu:
        import oracle
        oo = oracle.Options(ratio=(1, 4), eps_ppm=30000)
        reps, t_cpu = 0, []
        parity = True
        t_start = time.perf_counter()
        while reps < 3 or (time.perf_counter() - t_start < 10.0 and reps < 50):
            t0 = time.perf_counter()
            refs = [oracle.partition(g, oo) for g in graphs]
            t_cpu.append(time.perf_counter() - t0)
            reps += 1
        got = [p.cpu().numpy() for p in parts]
        for g, r, gpart, gres in zip(graphs, refs, got, results):
            parity &= bool(np.array_equal(gpart, r.part)) and gres.cut == r.cut
        tc = statistics.median(t_cpu)
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next((l.split(":", 1)[1].strip() for l in f
                                  if l.startswith("model name")), "")
        except OSError:
            pass
        out["cpu_baseline"] = {"value": round(edges / tc, 1), "unit": "edges/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the whole step (both DAGs), {reps} repetitions, "
                                         f"median {tc * 1e3:.1f} ms, single-threaded",
                               "cpu_model": cpu_model, "nproc": os.cpu_count()}
        out["parity_with_oracle"] = parity
    for h in handles:
        h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
