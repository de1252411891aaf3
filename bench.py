"""Benchmark: stepping-SSSP throughput on one MI355X.

One "step" of this benchmark is one whole solve of the hot path (init,
then ExtDist -> Extract -> Relax/WriteMin -> Update until the queue is
empty). The default workload is the power-law graph: R-MAT scale 24, edge
factor 16 (a = 0.57, b = 0.19, c = 0.19), symmetrised and deduplicated,
weights uniform in [1, 2^18), one source in the largest component,
rho-stepping. The graph is resident in HBM before timing starts.

`--workload knn10000` times the many-query workload instead: a 10-NN graph
of 10^7 points in 1000 Gaussian clusters and 64 sources, all solved in one
launch (a step = one batch of 64 queries), next to the same 64 queries
solved one launch at a time.

Prints one JSON line. `value` is edges relaxed per second (GTEPS, counting
repeated relaxations) over the K timed steps; `roofline` prices the
algorithmic bytes of the stepping kernel against the 8 TB/s HBM peak;
`cpu_baseline` times the CPU oracle (single-threaded binary-heap Dijkstra)
on the same graph and sources.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

METRIC = "edges relaxed/s (GTEPS) + % HBM roofline; p50/p99 query latency batched vs plain"
HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(REPO, "paper_2105_06145_amd", "csrc", f)
               for f in ("stepping.hip", "graph.hip", "internal.h")]
TRAFFIC_FILE = os.path.join(REPO, "profiles", "traffic_stepping_kernel_rmat24.json")

WORKLOADS = {
    "rmat24": "R-MAT scale 24, edge factor 16 (a=.57 b=.19 c=.19), symmetrised, self-loops and duplicates "
              "removed, w ~ U[1, 2^18), one source in the largest component; rho-stepping",
    "road5000": "5000x5000 jittered grid (+-0.4), 10% grid edges deleted, 1% extra edges within 3 cells, "
                "w = round(1000 * length), one source in the largest component; Delta*-stepping",
    "grid256": "256x256 4-neighbour grid, w ~ U[1, 2^16), source 0; rho-stepping rho=4096",
    "knn10000": "10-NN graph of 10^7 points: 1000 Gaussian clusters (sigma 0.01) of 10^4 points in the unit "
                "cube, union-symmetrised, w = max(1, llround(1e6 * dist)), caller vertex order kept; 64 sources "
                "uniform over all vertices, solved together in one launch; rule and parameters autotuned",
}
BATCHED = {"knn10000": 64}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n: int, st: dict, nsrc: int, offset_bytes: int = 8, relabelled: bool = True) -> int:
    """Bytes the method must move for one launch (nsrc solves), from its counters.

    S0, per source: 8n (distance fill) + n/8 (bitmap clear).
    Output in caller ids (relabelled graph), per source: 4n (id map) + 8n (read) + 8n (write).
    Extract, bitmap step: n/8 (flag scan) + 8 q (keys of members).
    Extract, list step:   12 q (list entry + key).
    Explicit lists: 4 per entry written (kept and new members).
    Per extracted vertex: 2 * offset_bytes (row bounds) + 8 (its key) + 8 (F write + read).
    Per relaxed arc:      8 (packed target, weight) + 8 (key of the target).
    Per successful WriteMin: 8 (key write) + 8 (flag word RMW).
    """
    b = nsrc * (8 * n + n // 8 + (20 * n if relabelled else 0))
    b += st["dense_steps"] * (n // 8) + 8 * st["queue_dense"] + 12 * st["queue_list"] + 4 * st["list_appends"]
    b += (2 * offset_bytes + 16) * st["extracted"] + 16 * st["edges_relaxed"] + 16 * st["writemin_success"]
    return b


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, rho: int):
    """HBM bytes per launch from the committed rocprofv3 counters, or None when
    they were taken on other kernel sources, another workload or another rho."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha() or d.get("workload") != workload:
        return None
    rec = d.get("by_rho", {}).get(str(rho))
    return rec.get("traffic_bytes_per_launch") if rec else None


def roofline_entry(b_alg: int, kernel_avg_ms: float, traffic):
    achieved = b_alg / (kernel_avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "stepping_kernel",
            "algorithmic_bytes_per_launch": int(b_alg), "kernel_avg_ms": round(kernel_avg_ms, 4)}


def reachable_arcs(g, dist_row) -> int:
    return int((np.diff(g.offsets)[dist_row != np.uint64(2**64 - 1)]).sum())


def base_record(args, value, ms_per, config, roofline, cpu):
    return {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def run_single(args, torch, sp, w):
    g, src = w.graph, int(w.sources[0])
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    torch.cuda.synchronize()

    rule = "rho" if args.workload != "road5000" else "delta"
    sweep = []
    if rule == "rho":
        if args.workload == "grid256":
            choices = [4096]
        elif args.sweep:
            choices = [1 << int(x) for x in args.sweep.split(",") if x]
        else:
            choices = []
        for rho in choices:
            times = []
            for _ in range(3):
                _, st = sp.solve(G, [src], rule="rho", rho=rho)
                times.append(st["device_ms"])
            sweep.append({"rho": rho, "ms": float(np.median(times)), "steps": int(st["steps"]),
                          "edges_relaxed": int(st["edges_relaxed"]),
                          "gteps": st["edges_relaxed"] / (np.median(times) * 1e6)})
            log(f"  sweep rho=2^{rho.bit_length() - 1}: {np.median(times):.3f} ms, steps {st['steps']}, "
                f"E_r {st['edges_relaxed']}")
        fixed = {"rho": min(sweep, key=lambda r: r["ms"])["rho"] if sweep else (args.rho or 1 << 18)}
    else:
        fixed = {"delta": args.delta}

    out = torch.empty((1, g.n), dtype=torch.int64, device="cuda")
    for _ in range(args.warmup):
        sp.solve(G, [src], rule=rule, out=out, **fixed)

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    edges = 0
    kernel_ms = 0.0
    steps_total = 0
    b_alg = 0
    ev0.record()
    for _ in range(args.steps):
        _, st = sp.solve(G, [src], rule=rule, out=out, **fixed)
        edges += st["edges_relaxed"]
        kernel_ms += st["device_ms"]
        steps_total += st["steps"]
        b_alg += algorithmic_bytes(g.n, st, 1)
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per = total_ms / args.steps
    gteps = edges / (total_ms * 1e6)
    m_reach = reachable_arcs(g, sp.to_numpy_u64(out)[0])

    roofline = roofline_entry(b_alg / args.steps, kernel_ms / args.steps,
                              load_traffic(args.workload, fixed.get("rho", 0)))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        c0 = oracle.now()
        _, settled, scanned = oracle.dijkstra(g.offsets, g.targets, g.weights, src,
                                              max_settled=args.cpu_settle_cap, stats=True)
        secs = oracle.now() - c0
        cpu = {"value": round(scanned / secs / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"one binary-heap Dijkstra solve from the same source ({settled} vertices settled, "
                         f"{scanned} arcs relaxed, {secs:.2f} s, 1 thread)"}

    config = {"workload": WORKLOADS[args.workload], "n": g.n, "m": g.m, "source": src, "rule": rule,
              **fixed, "steps_per_solve": int(steps_total // args.steps),
              "edges_relaxed_per_solve": int(edges // args.steps), "useful_arcs": m_reach}
    res = base_record(args, gteps, ms_per, config, roofline, cpu)
    res["gteps_useful"] = round(m_reach * args.steps / (total_ms * 1e6), 4)
    res["rho_sweep"] = sweep
    G.close()
    return res


def run_batched(args, torch, sp, w):
    """All sources in one launch (teams chosen by the library) against the
    same sources one launch each (one whole-grid team)."""
    g = w.graph
    srcs = [int(x) for x in w.sources]
    nq = len(srcs)
    from paper_2105_06145_amd import autotune as at
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    torch.cuda.synchronize()
    out = torch.empty((nq, g.n), dtype=torch.int64, device="cuda")
    one = torch.empty((1, g.n), dtype=torch.int64, device="cuda")

    def call(cfg, sources, dst, extra_tuning=None):
        tun = {**(cfg.get("tuning") or {}), **(extra_tuning or {})}
        kw = {k: cfg[k] for k in ("rho", "delta") if k in cfg}
        return sp.solve(G, sources, rule=cfg["rule"], tuning=tun or None, out=dst, **kw)

    default = {"rule": "rho", "rho": args.rho or int(w.params["rho"])}
    if args.tune_budget > 0:
        # Batched: the parameter search times the whole batch. Plain: it times
        # the first 8 queries one launch each, with one whole-grid team.
        t0 = time.time()
        cfg_b = at.Tuner(budget_s=args.tune_budget).tune(G, srcs)
        log(f"autotune batched ({time.time() - t0:.1f}s): {cfg_b}")

        def plain_measure(cfg):
            return sum(call(cfg, [s], one, {"teams": 1})[1]["device_ms"] for s in srcs[:8])
        t0 = time.time()
        w_med = G.summary["weight_q10_50_90"][1] or 1
        cfg_p = at.Tuner(budget_s=args.tune_budget, measure=plain_measure).search(G.n, 1, w_med)
        log(f"autotune plain ({time.time() - t0:.1f}s): {cfg_p}")
    else:
        cfg_b = cfg_p = default
    for _ in range(args.warmup):
        call(cfg_b, srcs, out)
    call(cfg_p, srcs[:1], one, {"teams": 1})

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    edges = kernel_ms = b_alg = 0
    ev0.record()
    for _ in range(args.steps):
        _, st = call(cfg_b, srcs, out)
        edges += st["edges_relaxed"]
        kernel_ms += st["device_ms"]
        b_alg += algorithmic_bytes(g.n, st, nq, relabelled=False)
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per = total_ms / args.steps
    teams = int(st["teams"])
    dist = sp.to_numpy_u64(out)
    m_reach = sum(reachable_arcs(g, dist[i]) for i in range(nq))

    # The same queries, one launch each.
    plain_edges = 0
    lat = []
    ev0.record()
    for s in srcs:
        _, st1 = call(cfg_p, [s], one, {"teams": 1})
        plain_edges += st1["edges_relaxed"]
        lat.append(st1["device_ms"])
    ev1.record()
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1)

    roofline = roofline_entry(b_alg / args.steps, kernel_ms / args.steps, None)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        c0 = oracle.now()
        scanned_total = 0
        for s in srcs:
            _, _, scanned = oracle.dijkstra(g.offsets, g.targets, g.weights, s, stats=True)
            scanned_total += scanned
        secs = oracle.now() - c0
        cpu = {"value": round(scanned_total / secs / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"the same {nq} queries, one binary-heap Dijkstra each ({scanned_total} arcs relaxed, "
                         f"{secs:.2f} s, 1 thread, {nq / secs:.2f} queries/s)"}

    strip = lambda c: {k: v for k, v in c.items() if k in ("rule", "rho", "delta", "tuning")}
    config = {"workload": WORKLOADS[args.workload], "n": g.n, "m": g.m, "queries": nq, **strip(cfg_b),
              "teams": teams, "edges_relaxed_per_batch": int(edges // args.steps), "useful_arcs": m_reach,
              "tuned": args.tune_budget > 0}
    res = base_record(args, edges / (total_ms * 1e6), ms_per, config, roofline, cpu)
    res["gteps_useful"] = round(m_reach * args.steps / (total_ms * 1e6), 4)
    res["queries_per_s"] = round(nq * args.steps / (total_ms * 1e-3), 1)
    res["plain"] = {"what": f"the same {nq} queries, one launch each, whole grid per query", "config": strip(cfg_p),
                    "total_ms": round(plain_ms, 3), "queries_per_s": round(nq / (plain_ms * 1e-3), 1),
                    "gteps": round(plain_edges / (plain_ms * 1e6), 4),
                    "gteps_useful": round(m_reach / (plain_ms * 1e6), 4),
                    "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                    "latency_ms_p99": round(float(np.percentile(lat, 99)), 4)}
    res["batched_speedup"] = round(plain_ms / ms_per, 3)
    G.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--rho", type=int, default=0, help="rho for the timed solves (0 = the workload's default)")
    ap.add_argument("--delta", type=int, default=1 << 13)
    ap.add_argument("--sweep", default="", metavar="LOG2_LIST",
                    help="e.g. 16,17,18,19,20,21,22: time 3 solves per rho first and use the fastest")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-budget", type=float, default=20.0,
                    help="seconds of parameter search per mode for the batched workload (0 = workload defaults)")
    ap.add_argument("--cpu-settle-cap", type=int, default=0,
                    help="stop the CPU oracle after this many settled vertices (0 = full solve)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (5 times) and exit; "
                         "used to scale the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen
    import paper_2105_06145_amd as sp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    t0 = time.time()
    w = graphgen.workload(args.workload, sources=BATCHED.get(args.workload, 1))
    log(f"workload {args.workload}: n={w.graph.n} m={w.graph.m} sources={len(w.sources)} "
        f"(generated in {time.time() - t0:.1f}s)")
    if args.workload in BATCHED:
        res = run_batched(args, torch, sp, w)
    else:
        res = run_single(args, torch, sp, w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
