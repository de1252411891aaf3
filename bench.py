"""Benchmark: stepping-SSSP throughput on one MI355X.

One "step" of this benchmark is one whole solve of the hot path (init,
then ExtDist -> Extract -> Relax/WriteMin -> Update until the queue is
empty). The default workload is the power-law graph: R-MAT scale 24, edge
factor 16 (a = 0.57, b = 0.19, c = 0.19), symmetrised and deduplicated,
weights uniform in [1, 2^18), ten seeded sources in the largest component,
rho-stepping. The graph is resident in HBM before timing starts. rho is
swept over 2^16 .. 2^22 first with the paper's rule (one solve per source
each; `rho_sweep`, fastest in `paper_rule`), then with hub deferral at the
autotuner's settings around the fastest rho (`hub_defer_sweep`: vertices of
high out-degree extracted only at keys up to a much smaller sampled rank);
the K timed solves use the fastest configuration of both.

The default line also carries the metric's other workloads, each under its
own key: `road_delta_sweep` (the 5000 x 5000 road grid, Delta*-stepping with
Delta = 2^10 .. 2^16 and Bellman-Ford: time, steps, time per step; then
Delta and the local-expansion budget together around the fastest),
`knn_batched` (a 10-NN graph of 10^7 points, 64 queries in one launch
against the same queries one launch each) and `latency` (a short serving
run: R-MAT scale 22 and a 2000 x 2000 road grid resident, Poisson arrivals,
p50/p99 of the serving launches against a one-query-at-a-time loop);
`--extras` selects them.

`--workload knn10000` times the many-query workload alone (with an optional
parameter search); `--workload serve` runs the serving comparison at full
length (a closed loop over a prefix of the trace for the saturation rates,
then the open loop over the whole trace); `road5000` and `grid256` time
single solves.

Prints one JSON line. `value` is edges relaxed per second (GTEPS, counting
repeated relaxations) over the K timed steps, `gteps_useful` arcs out of
reachable vertices per second; `roofline` prices the algorithmic bytes of
the stepping kernel against the 8 TB/s HBM peak; `cpu_baseline` times the
CPU oracle (single-threaded binary-heap Dijkstra, median of 3) on the same
graph.
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
               for f in ("stepping.hip", "graph.hip", "internal.h", "hint_code.h")]
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
WORKLOADS["serve"] = ("serving: R-MAT scale 22 (edge factor 16, w ~ U[1, 2^18)) and a 2000x2000 road-like grid "
                      "(road recipe) both resident; each query picks R-MAT with probability 0.7, else the grid, and "
                      "a uniform source in that graph's largest component; Poisson arrivals")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n: int, st: dict, nsrc: int, offset_bytes: int = 8) -> int:
    """Bytes the method must move for one launch (nsrc solves), from its
    counters, by the roofline's accounting of the path:

    S0, per source:        8 n (distance fill) + n / 8 (bitmap clear).
    Dense (bitmap) steps:  n / 8 (flag scan) per step + 8 per queued member (keys).
    Per extracted vertex:  2 * offset_bytes (row bounds) + 8 (its key) + 8 (F write + read).
    Per relaxed arc:       8 (packed target, weight) + 8 (key of the target).
    Per successful WriteMin: 8 (key write) + 4 (flag word); explicit-list
                           mode: + 4 per list entry written.
    """
    b = nsrc * (8 * n + n // 8)
    b += st["dense_steps"] * (n // 8) + 8 * st["queue_dense"]
    b += (2 * offset_bytes + 16) * st["extracted"] + 16 * st["edges_relaxed"]
    b += 12 * st["writemin_success"] + 4 * st["list_appends"]
    return b


def implementation_bytes(n: int, st: dict, nsrc: int, offset_bytes: int = 8, relabelled: bool = True) -> int:
    """The same with what this implementation adds to the method's bytes: the
    copy of each row back to the caller's vertex ids (4 n id map + 8 n read +
    8 n write per source on relabelled graphs), the list steps' reads of the
    queue (4 per entry + 8 per key) and 8-byte flag words (+ 4 per success)."""
    b = algorithmic_bytes(n, st, nsrc, offset_bytes)
    b += nsrc * (20 * n if relabelled else 0) + 12 * st["queue_list"] + 4 * st["writemin_success"]
    return b


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_key(rho: int, tuning) -> str:
    """Key of a configuration in the traffic file: rho, plus the hub-deferral
    setting when there is one and a list divisor other than the default
    ("2097152:defer32/1000", "2097152:defer32/1000:list256")."""
    key = str(rho)
    if tuning and tuning.get("hub_defer_degree"):
        key += f":defer{tuning['hub_defer_degree']}/{tuning['hub_defer_div']}"
    if tuning and tuning.get("list_divisor", 64) != 64:
        key += f":list{tuning['list_divisor']}"
    return key


def load_traffic(workload: str, key: str):
    """HBM bytes per launch from the committed rocprofv3 counters, or None when
    they were taken on other kernel sources, another workload or another
    configuration (traffic_key)."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha() or d.get("workload") != workload:
        return None
    rec = d.get("by_rho", {}).get(key)
    return rec.get("traffic_bytes_per_launch") if rec else None


def roofline_entry(b_alg: int, kernel_avg_ms: float, traffic):
    achieved = b_alg / (kernel_avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "stepping_kernel",
            "algorithmic_bytes_per_launch": int(b_alg), "kernel_avg_ms": round(kernel_avg_ms, 4)}


def host_cpu() -> dict:
    """CPU model and core counts of the host the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "cpu_count": os.cpu_count()}


def oracle_baseline(g, src: int, runs: int = 3) -> dict:
    """The oracle (single-threaded binary-heap Dijkstra) from one source,
    timed `runs` times; the rate is arcs scanned per second of the median."""
    import oracle
    secs = []
    settled = scanned = 0
    for _ in range(runs):
        c0 = oracle.now()
        _, settled, scanned = oracle.dijkstra(g.offsets, g.targets, g.weights, src, stats=True)
        secs.append(oracle.now() - c0)
    med = float(np.median(secs))
    return {"value": round(scanned / med / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"one binary-heap Dijkstra solve from the first source ({settled} vertices settled, "
                      f"{scanned} arcs relaxed), timed {runs} times on 1 thread: median {med:.2f} s "
                      f"(runs {', '.join(f'{x:.2f}' for x in secs)} s)",
            **host_cpu()}


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


def stream_copy_gbs(torch, mib: int = 1024, reps: int = 5) -> float:
    """Measured device-copy bandwidth (bytes read + written per second), the
    practical ceiling beside the 8 TB/s spec peak."""
    nbytes = mib << 20
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def measure_ceilings(torch, g, relax_arcs: int, relax_ms: float) -> dict:
    """The memory-system rates that bound Relax, measured by the ceiling
    microbenchmarks (libsssp_ceilings.so) over tables of this graph's size:
    random 2-byte gathers (the filter's key-bound read per arc) and random
    64-bit atomic minima (WriteMin), with indices uniform over the vertices
    and, separately, distributed as the graph's arc targets (a random arc's
    target, numbered by decreasing degree as the library numbers vertices).
    Beside them, Relax's own rate: arcs relaxed per second of Relax phase."""
    import ctypes

    from paper_2105_06145_amd import _native
    L = _native.ceilings_lib()
    n = g.n
    count = 1 << 27
    rng = np.random.default_rng(12345)
    deg = np.diff(g.offsets)
    order = np.argsort(-deg, kind="stable")
    rank = np.empty(n, dtype=np.int32)
    rank[order] = np.arange(n, dtype=np.int32)
    arcs = rng.integers(0, g.m, count)
    idx_deg = torch.from_numpy(rank[g.targets[arcs]]).cuda()
    idx_uni = torch.randint(0, n, (count,), dtype=torch.int32, device="cuda")
    del arcs, order, rank
    t16 = torch.zeros(n, dtype=torch.int16, device="cuda")
    t64 = torch.full((n,), (1 << 62), dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def rate(call, reps=3):
        assert call() == 0  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            assert call() == 0
        e1.record()
        torch.cuda.synchronize()
        return round(count * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 2)

    vp = ctypes.c_void_p
    out = {"unit": "G accesses/s", "accesses_per_launch": count, "table_entries": n}
    for name, idx in (("uniform", idx_uni), ("arc_targets", idx_deg)):
        out[f"gather16_{name}"] = rate(lambda: L.sssp_ceiling_gather16(vp(idx.data_ptr()), count, vp(t16.data_ptr()),
                                                                       vp(sink.data_ptr()), st))
        out[f"atomic_min64_{name}"] = rate(lambda: L.sssp_ceiling_atomic_min64(vp(idx.data_ptr()), count,
                                                                               vp(t64.data_ptr()), st))
    # Gathers that always hit L2: the index stream walks the table slice by
    # slice (2^18 entries = 512 KB per slice, uniform within it), so every
    # XCD's L2 holds the slice being read. What binning the arcs by target
    # range (to make the key-bound reads L2-resident) could at best reach.
    slice_entries = 1 << 18
    nsl = max(1, n // slice_entries)
    per = count // nsl
    idx_l2 = ((torch.arange(count, device="cuda", dtype=torch.int64) // per).clamp(max=nsl - 1) * slice_entries
              + torch.randint(0, min(n, slice_entries), (count,), device="cuda")).to(torch.int32)
    out["gather16_l2_slices"] = rate(lambda: L.sssp_ceiling_gather16(vp(idx_l2.data_ptr()), count, vp(t16.data_ptr()),
                                                                     vp(sink.data_ptr()), st))
    out["l2_slice_entries"] = slice_entries
    del idx_l2
    out["relax_arcs_per_s"] = round(relax_arcs / (relax_ms * 1e-3) / 1e9, 2)
    out["relax_frac_of_gather16_arc_targets"] = round(out["relax_arcs_per_s"] / out["gather16_arc_targets"], 3)
    del idx_deg, idx_uni, t16, t64, sink
    torch.cuda.synchronize()
    return out


def run_single(args, torch, sp, w):
    g = w.graph
    srcs = [int(x) for x in w.sources]
    src = srcs[0]
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    torch.cuda.synchronize()
    out = torch.empty((1, g.n), dtype=torch.int64, device="cuda")

    rule = "rho" if args.workload != "road5000" else "delta"
    sweep, defer_sweep = [], []
    m_reach_of = {}
    tuning = None  # tuning of the timed solves (hub deferral), or None

    def sweep_point(rho, tun):
        """One solve per source (the timed solves' sources), averaged."""
        times, balg, edges_r, steps_r, useful = [], [], [], [], []
        for s_ in srcs:
            _, st = sp.solve(G, [s_], rule="rho", rho=rho, tuning=tun, out=out)
            if s_ not in m_reach_of:
                m_reach_of[s_] = reachable_arcs(g, sp.to_numpy_u64(out)[0])
            times.append(st["device_ms"])
            balg.append(algorithmic_bytes(g.n, st, 1))
            edges_r.append(st["edges_relaxed"])
            steps_r.append(st["steps"])
            useful.append(m_reach_of[s_])
        ms = float(np.mean(times))
        r = {"rho": rho, "ms": round(ms, 4), "steps": int(np.mean(steps_r)),
             "edges_relaxed": int(np.mean(edges_r)),
             "gteps": round(float(np.mean(edges_r)) / (ms * 1e6), 4),
             "gteps_useful": round(float(np.mean(useful)) / (ms * 1e6), 4),
             "roofline_frac": round(float(np.mean(balg)) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        if tun:
            r["hub_defer"] = {"degree": tun["hub_defer_degree"], "div": tun["hub_defer_div"]}
        log(f"  sweep rho=2^{rho.bit_length() - 1} {tun or ''}: {ms:.3f} ms, steps {r['steps']}, "
            f"E_r {r['edges_relaxed']}, frac {r['roofline_frac']}")
        return r

    if rule == "rho":
        if args.workload == "grid256":
            choices = [4096]
        elif args.sweep:
            choices = [1 << int(x) for x in args.sweep.split(",") if x]
        else:
            choices = []
        for rho in choices:
            sweep.append(sweep_point(rho, None))
        fixed = {"rho": min(sweep, key=lambda r: r["ms"])["rho"] if sweep else (args.rho or 1 << 18)}
        if args.rho:
            fixed = {"rho": args.rho}
        if args.defer:
            parts = [int(x) for x in args.defer.split(",")]
            tuning = {"hub_defer_degree": parts[0], "hub_defer_div": parts[1]}
            if len(parts) > 2:
                tuning["list_divisor"] = parts[2]
        elif sweep and args.defer_sweep and args.workload == "rmat24":
            # Hub deferral: the autotuner's candidates around the fastest rho
            # of the paper's rule; the timed solves use the fastest of all.
            from paper_2105_06145_amd import autotune as at
            for rho, deg, div in at.defer_candidates(fixed["rho"]):
                defer_sweep.append(sweep_point(rho, {"hub_defer_degree": deg, "hub_defer_div": div}))
            best_d = min(defer_sweep, key=lambda r: r["ms"])
            # The explicit-list switch around the best setting (the
            # autotuner's next knob): a list kept only for smaller queues
            # suits the deferred queue, which stays large for longer.
            base_tun = {"hub_defer_degree": best_d["hub_defer"]["degree"], "hub_defer_div": best_d["hub_defer"]["div"]}
            for ld in (16, 256):
                r = sweep_point(best_d["rho"], {**base_tun, "list_divisor": ld})
                r["list_divisor"] = ld
                defer_sweep.append(r)
            best_d = min(defer_sweep, key=lambda r: r["ms"])
            if best_d["ms"] < min(sweep, key=lambda r: r["ms"])["ms"] and not args.rho:
                fixed = {"rho": best_d["rho"]}
                tuning = {"hub_defer_degree": best_d["hub_defer"]["degree"],
                          "hub_defer_div": best_d["hub_defer"]["div"]}
                if "list_divisor" in best_d:
                    tuning["list_divisor"] = best_d["list_divisor"]
        if tuning:
            fixed["tuning"] = tuning
    else:
        fixed = {"delta": args.delta or int(w.params["delta"])}

    for i in range(args.warmup):
        sp.solve(G, [srcs[i % len(srcs)]], rule=rule, out=out, **fixed)

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    edges = 0
    kernel_ms = 0.0
    steps_total = 0
    b_alg = b_impl = 0
    extracted = successes = 0
    relax_ms = 0.0
    # Step i solves from source i mod K (the paper averages over sources;
    # all of them lie in the largest component).
    ev0.record()
    for i in range(args.steps):
        _, st = sp.solve(G, [srcs[i % len(srcs)]], rule=rule, out=out, **fixed)
        edges += st["edges_relaxed"]
        kernel_ms += st["device_ms"]
        steps_total += st["steps"]
        extracted += st["extracted"]
        successes += st["writemin_success"]
        relax_ms += st["phase_ms"][3]
        b_alg += algorithmic_bytes(g.n, st, 1)
        b_impl += implementation_bytes(g.n, st, 1)
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per = total_ms / args.steps
    gteps = edges / (total_ms * 1e6)
    m_reach = 0
    for i in range(args.steps):
        s_ = srcs[i % len(srcs)]
        if s_ not in m_reach_of:
            sp.solve(G, [s_], rule=rule, out=out, **fixed)
            m_reach_of[s_] = reachable_arcs(g, sp.to_numpy_u64(out)[0])
        m_reach += m_reach_of[s_]

    roofline = roofline_entry(b_alg / args.steps, kernel_ms / args.steps,
                              load_traffic(args.workload, traffic_key(fixed.get("rho", 0), tuning)))
    roofline["implementation_bytes_per_launch"] = int(b_impl / args.steps)
    copy_gbs = stream_copy_gbs(torch)
    roofline["stream_copy_gbs"] = round(copy_gbs, 1)
    roofline["frac_of_stream"] = round(roofline["achieved"] / copy_gbs, 4)
    if args.workload == "rmat24" and not args.no_ceilings:
        try:
            roofline["ceilings"] = measure_ceilings(torch, g, edges, relax_ms)
        except Exception as e:
            roofline["ceilings"] = {"error": f"{type(e).__name__}: {e}"}

    cpu = None if args.no_cpu_baseline else oracle_baseline(g, src, args.cpu_runs)

    config = {"workload": WORKLOADS[args.workload], "n": g.n, "m": g.m,
              "sources": srcs if len(srcs) > 1 else src, "rule": rule,
              **{k: v for k, v in fixed.items() if k != "tuning"},
              "hub_defer": ({"degree": tuning["hub_defer_degree"], "div": tuning["hub_defer_div"]}
                            if tuning else None),
              "list_divisor": (tuning or {}).get("list_divisor", 64),
              "steps_per_solve": int(steps_total // args.steps),
              "edges_relaxed_per_solve": int(edges // args.steps),
              "writemin_success_per_solve": int(successes // args.steps),
              "useful_arcs_per_solve": int(m_reach // args.steps)}
    res = base_record(args, gteps, ms_per, config, roofline, cpu)
    res["gteps_useful"] = round(m_reach / (total_ms * 1e6), 4)
    res["extracted_per_vertex"] = round(extracted / args.steps / g.n, 4)  # X / n
    res["relaxed_per_arc"] = round(edges / args.steps / g.m, 4)           # E_r / m
    if sweep:
        best = min(sweep, key=lambda r: r["ms"])
        res["rho_sweep"] = {"per_rho": sweep, "fastest_rho": best["rho"],
                            "fastest_frac": best["roofline_frac"],
                            "what": "the paper's rho rule: one solve per source per rho, averaged"}
        res["paper_rule"] = {k: best[k] for k in ("rho", "ms", "steps", "edges_relaxed", "gteps", "gteps_useful",
                                                  "roofline_frac")}
    if defer_sweep:
        bd = min(defer_sweep, key=lambda r: r["ms"])
        res["hub_defer_sweep"] = {
            "per_setting": defer_sweep,
            "fastest": {k: bd[k] for k in ("rho", "hub_defer", "ms", "list_divisor") if k in bd},
            "what": ("rho with hub deferral (vertices of out-degree >= degree extracted only at keys up to the "
                     "sampled (rho / div)-th key), one solve per source each; the timed solves use the fastest "
                     "configuration of both sweeps (fewer arcs relaxed for the same distances, so GTEPS and the "
                     "roofline fraction count less work)")}
    G.close()
    torch.cuda.synchronize()
    return res


def run_road_sweep(args, torch, sp):
    """Delta*-stepping over Delta = 2^10 .. 2^16 and Bellman-Ford on the road
    workload, one solve each from its seeded source: time, steps, time per
    step (the paper's Delta and BF rows; Sec. 6 on road graphs). Then the
    autotuner's joint candidates of Delta and local-expansion budget around
    the fastest Delta."""
    import graphgen
    w = graphgen.workload("road5000", sources=1)
    g = w.graph
    src = int(w.sources[0])
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    out = torch.empty((1, g.n), dtype=torch.int64, device="cuda")
    sp.solve(G, [src], rule="delta", delta=1 << 15, out=out)  # warm-up
    m_reach = reachable_arcs(g, sp.to_numpy_u64(out)[0])
    rows = []
    for lg in list(range(10, 17)) + ["bf"]:
        kw = {"rule": "bf"} if lg == "bf" else {"rule": "delta", "delta": 1 << lg}
        _, st = sp.solve(G, [src], out=out, **kw)
        ms = st["device_ms"]
        rows.append({"delta": None if lg == "bf" else 1 << lg, "rule": kw["rule"], "ms": round(ms, 3),
                     "steps": int(st["steps"]), "us_per_step": round(ms * 1e3 / max(1, st["steps"]), 2),
                     "edges_relaxed": int(st["edges_relaxed"]), "gteps": round(st["edges_relaxed"] / (ms * 1e6), 4),
                     "gteps_useful": round(m_reach / (ms * 1e6), 4),
                     "local_vertices": int(st["local_vertices"])})
        log(f"  road5000 {kw}: {ms:.2f} ms, {st['steps']} steps")
    best = min((r for r in rows if r["rule"] == "delta"), key=lambda r: r["ms"])
    # Delta and the local-expansion budget together (the autotuner's joint
    # step), around the fastest Delta at the default budget.
    from paper_2105_06145_amd import autotune as at
    joint = []
    for d, budget in at.local_candidates(best["delta"]):
        _, st = sp.solve(G, [src], rule="delta", delta=d, tuning={"local_budget": budget}, out=out)
        ms = st["device_ms"]
        joint.append({"delta": d, "local_budget": budget, "ms": round(ms, 3), "steps": int(st["steps"]),
                      "edges_relaxed": int(st["edges_relaxed"]), "local_vertices": int(st["local_vertices"]),
                      "gteps_useful": round(m_reach / (ms * 1e6), 4)})
        log(f"  road5000 delta {d}, local budget {budget}: {ms:.2f} ms, {st['steps']} steps")
    G.close()
    torch.cuda.synchronize()
    jbest = min(joint, key=lambda r: r["ms"])
    return {"workload": WORKLOADS["road5000"], "n": g.n, "m": g.m, "source": src, "useful_arcs": m_reach,
            "per_rule": rows, "fastest_delta": best["delta"],
            "delta_and_local_budget": {"per_pair": joint, "default_budget": at.DEFAULT_LOCAL_BUDGET,
                                       "fastest": {k: jbest[k] for k in ("delta", "local_budget", "ms")}}}


def run_knn_compare(args, torch, sp):
    """The batched workload at fixed settings (from an earlier tuning run):
    64 queries in one launch against the same 64 queries one launch each."""
    import graphgen
    w = graphgen.workload("knn10000", sources=64)
    la = argparse.Namespace(**vars(args))
    la.tune_budget, la.no_cpu_baseline, la.steps, la.warmup = 0.0, True, 3, 1
    la.workload = "knn10000"
    r = run_batched(la, torch, sp, w, cfg_fixed=({"rule": "delta", "delta": 1898},
                                                 {"rule": "delta", "delta": 3796}))
    keep = ("queries_per_s", "batched_speedup", "gteps_useful", "plain", "ms_per_step", "value")
    res = {k: r[k] for k in keep}
    res["config"] = {k: r["config"][k] for k in ("n", "m", "queries", "rule", "delta", "teams")}
    res["workload"] = WORKLOADS["knn10000"]
    res["settings"] = ("fixed, from an earlier tuning run of this workload: Delta*-stepping with Delta = 1898 "
                       "for the batch, 3796 for the single launches")
    return res


def run_batched(args, torch, sp, w, cfg_fixed=None):
    """All sources in one launch (teams chosen by the library) against the
    same sources one launch each (one whole-grid team). cfg_fixed: (batched,
    plain) settings to use instead of the defaults or a tuning run."""
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
    if cfg_fixed is not None:
        cfg_b, cfg_p = cfg_fixed
    elif args.tune_budget > 0:
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
        b_alg += algorithmic_bytes(g.n, st, nq)
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
                         f"{secs:.2f} s, 1 thread, {nq / secs:.2f} queries/s)", **host_cpu()}

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


def np_row_hash(d: np.ndarray) -> int:
    """Checksum of a distance row, as sssp_row_hash defines it (for oracle rows)."""
    v = np.arange(d.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = d.astype(np.uint64) ^ (v * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        return int(z.sum(dtype=np.uint64))


def run_serve(args, torch, sp):
    """Continuous-batching servers (one persistent launch per graph, requests
    joining as teams free up) against a one-query-at-a-time loop of plain
    solves, on the same query trace: closed loop (all queries queued at once)
    for saturation throughput, then open loop with Poisson arrivals at 0.8 x
    the plain loop's saturation rate."""
    import graphgen
    from paper_2105_06145_amd import autotune as at
    side = torch.cuda.Stream()  # keep work off the NULL stream while servers run
    torch.cuda.set_stream(side)
    t0 = time.time()
    gr = graphgen.rmat(22, 16, seed=5001)
    gd = graphgen.road(2000, 2000, seed=5002)
    graphs = [gr, gd]
    lcc = [graphgen.largest_component(g) for g in graphs]
    log(f"serve graphs: rmat22 n={gr.n} m={gr.m}, road2000 n={gd.n} m={gd.m} ({time.time() - t0:.1f}s)")
    G = [sp.Graph.from_csr(gr.offsets, gr.targets, gr.weights),
         sp.Graph.from_csr(gd.offsets, gd.targets, gd.weights, reorder=False)]
    nq = args.queries
    rng = np.random.default_rng(5003)
    which = (rng.random(nq) >= 0.7).astype(np.int64)  # 0: R-MAT (p = 0.7), 1: grid
    pools = [np.flatnonzero(m) for m in lcc]
    src = np.array([int(pools[k][rng.integers(0, pools[k].size)]) for k in which], dtype=np.int64)
    gaps = rng.exponential(1.0, nq)  # unit-rate Poisson process, scaled below

    # Parameters: tuned on a batch of the trace's sources per graph (served),
    # and on 8 single queries per graph (plain).
    cfg_s, cfg_p = [], []
    if args.tune_budget <= 0:
        # Settings a full tuning run of this workload chose for one query at a
        # time on the whole grid. The servers' rho and Delta are per team (a
        # group of k teams uses k times them): the whole-grid values divided
        # by the server's team count, so a request that arrives at a quiet
        # server, solved by all its teams, runs with the plain loop's values.
        # R-MAT: rho = 2^19 with hub deferral (degree 64, rank rho / 300),
        # 6.7 against 9.6 ms per query for the paper's rule at its best rho
        # (2^17) on the whole grid; --serve-no-defer keeps the paper's rule.
        if args.serve_defer:
            rmat_rho, rmat_tun = 1 << 19, {"hub_defer_degree": 64, "hub_defer_div": 300}
        else:
            rmat_rho, rmat_tun = 1 << 17, {}
        cfg_p = [{"rule": "rho", "rho": rmat_rho, "tuning": dict(rmat_tun)},
                 {"rule": "delta", "delta": 67584, "tuning": {}}]
        nteams = [int(x) for x in args.serve_teams.split(",")]
        cfg_s = [{"rule": "rho", "rho": args.serve_rho or max(1, rmat_rho // nteams[0]), "tuning": dict(rmat_tun)},
                 {"rule": "delta", "delta": args.serve_delta or max(1, 67584 // nteams[1]), "tuning": {}}]
    for k in ((0, 1) if args.tune_budget > 0 else ()):
        ks = [int(x) for x in src[which == k][:32]]
        tb = at.Tuner(budget_s=args.tune_budget / 2)
        cfg_s.append(tb.tune(G[k], ks, rules=("rho",) if k == 0 else ("delta",)))

        def plain_measure(cfg, k=k, ks=ks):
            kw = {x: cfg[x] for x in ("rho", "delta") if x in cfg}
            tun = {**(cfg.get("tuning") or {}), "teams": 1}
            return sum(sp.solve(G[k], [s], rule=cfg["rule"], tuning=tun, **kw)[1]["device_ms"] for s in ks[:8])
        cfg_p.append(at.Tuner(budget_s=args.tune_budget / 2, measure=plain_measure).search(
            G[k].n, 1, G[k].summary["weight_q10_50_90"][1] or 1, rules=("rho",) if k == 0 else ("delta",)))
        log(f"graph {k}: served {cfg_s[k]}, plain {cfg_p[k]}")

    def params(cfg):
        return {x: cfg[x] for x in ("rule", "rho", "delta") if x in cfg}

    out1 = [torch.empty((1, g.n), dtype=torch.int64, device="cuda") for g in graphs]

    def plain_loop(arrive, count):
        """One query at a time, whole grid each; returns (latencies, hashes, makespan)."""
        lat = np.zeros(count)
        hashes = [0] * count
        start = time.perf_counter()
        for i in range(count):
            k = int(which[i])
            now = time.perf_counter() - start
            if now < arrive[i]:
                time.sleep(arrive[i] - now)
            tun = {**(cfg_p[k].get("tuning") or {}), "teams": 1}
            sp.solve(G[k], [int(src[i])], tuning=tun, out=out1[k], stream=side, **params(cfg_p[k]))
            hashes[i] = sp.row_hash(out1[k][0], stream=side)
            lat[i] = time.perf_counter() - start - arrive[i]
            if (i + 1) % 200 == 0:
                log(f"  plain: {i + 1}/{count} queries, {time.perf_counter() - start:.1f}s")
        return lat, hashes, time.perf_counter() - start

    serve_teams = [int(x) for x in args.serve_teams.split(",")]
    serve_bpc = [int(x) for x in args.serve_bpc.split(",")]
    serve_gmax = [int(x) for x in args.serve_group_max.split(",")]
    serve_gmin = [int(x) for x in args.serve_group_min.split(",")]
    # The admission budget, split between the two servers in proportion to
    # their grids.
    budget = int(args.serve_budget_gib * (1 << 30))
    budgets = [budget * serve_bpc[0] // sum(serve_bpc), budget * serve_bpc[1] // sum(serve_bpc)]

    def served_loop(arrive, count):
        """Both graphs' budget servers running; queries enqueued at arrival and
        admitted as rows of the budget free up (a finished query's row is
        released as soon as it is polled); returns (latencies, hashes,
        makespan, stats, most rows in use)."""
        servers = [sp.BudgetServer(G[k], budgets[k], tuning={**(cfg_s[k].get("tuning") or {}),
                                                             "blocks_per_cu": serve_bpc[k], "teams": serve_teams[k],
                                                             "group_max": serve_gmax[k], "group_min": serve_gmin[k]},
                                   hash_rows=True, stream=side, **params(cfg_s[k])) for k in (0, 1)]
        ticket = [{}, {}]
        lat = np.zeros(count)
        hashes = [0] * count
        nxt = done = 0
        peak_rows = [0, 0]
        start = time.perf_counter()
        last_log = last_done = start
        try:
            while done < count:
                now_abs = time.perf_counter()
                if now_abs - last_log > 5.0:
                    last_log = now_abs
                    log(f"  served: {done}/{count} queries, {now_abs - start:.1f}s")
                if now_abs - last_done > 60.0:
                    # Both servers must be resident at once; a tool that runs
                    # kernels one at a time (a counter-collecting profiler)
                    # leaves the second waiting for the first to go idle.
                    raise RuntimeError(f"serving stalled at {done}/{count} queries")
                now = now_abs - start
                while nxt < count and arrive[nxt] <= now:
                    k = int(which[nxt])
                    ticket[k][servers[k].enqueue(int(src[nxt]))] = nxt
                    nxt += 1
                for k in (0, 1):
                    S = servers[k]
                    fin = S.poll()
                    if fin:
                        c = S.counts()
                        peak_rows[k] = max(peak_rows[k], c["admitted"] + c["held"])
                    for t, h in fin:
                        i = ticket[k].pop(t)
                        lat[i] = time.perf_counter() - start - arrive[i]
                        hashes[i] = h
                        S.release(t)
                        done += 1
                        last_done = time.perf_counter()
            makespan = time.perf_counter() - start
            rows_avail = [S.counts()["rows"] for S in servers]
            stats = [S.stop() for S in servers]
        finally:
            for S in servers:
                try:
                    S.stop()
                except Exception:
                    pass
            for S in servers:
                S.close()
        return lat, hashes, makespan, stats, {"rows": rows_avail, "peak_rows_in_use": peak_rows}

    # Closed loop (the trace's first queries all queued at t = 0): saturation
    # rates of both systems.
    nc = min(nq, args.closed_queries) if args.closed_queries > 0 else nq
    zero = np.zeros(nc)
    lat_p0, hash_p, span_p0 = plain_loop(zero, nc)
    rate_plain = nc / span_p0
    log(f"plain closed loop: {span_p0:.2f}s, {rate_plain:.1f} q/s")
    lat_s0, hash_s0, span_s0, _, _ = served_loop(zero, nc)
    log(f"served closed loop: {span_s0:.2f}s, {nc / span_s0:.1f} q/s")
    # Open loop over the whole trace at 0.8 x the plain saturation rate.
    lam = 0.8 * rate_plain
    arrive = np.cumsum(gaps) / lam
    lat_p1, hash_p1, span_p1 = plain_loop(arrive, nq)
    lat_s1, hash_s1, span_s1, sstats, rowinfo = served_loop(arrive, nq)
    log(f"open loop lambda={lam:.1f}/s: plain p50 {np.median(lat_p1) * 1e3:.1f} ms, served p50 "
        f"{np.median(lat_s1) * 1e3:.1f} ms")
    same = all(hash_p1[i] == hash_s1[i] for i in range(nq)) and \
        all(hash_p[i] == hash_s0[i] == hash_p1[i] for i in range(nc))
    # Oracle sample.
    checked = 0
    if not args.no_cpu_baseline:
        import oracle
        c0 = oracle.now()
        for k in (0, 1):
            for i in np.flatnonzero(which == k)[:args.oracle_sample]:
                d = oracle.dijkstra(graphs[k].offsets, graphs[k].targets, graphs[k].weights, int(src[i]))
                assert np_row_hash(d) == hash_s1[i], f"query {i}: served row differs from the oracle"
                checked += 1
        csecs = oracle.now() - c0
    edges_served = sum(st["edges_relaxed"] for st in sstats)

    def pct(x, q):
        return round(float(np.percentile(x, q)) * 1e3, 3)

    res = {
        "metric": METRIC,
        "value": round(nq / span_s1, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": nq,
        "warmup": 0,
        "ms_per_step": round(span_s1 * 1e3 / nq, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["serve"], "queries": nq, "closed_loop_queries": nc,
                   "admission_budget_bytes": budgets, "result_rows": rowinfo["rows"],
                   "peak_rows_in_use": rowinfo["peak_rows_in_use"],
                   "server_teams": serve_teams, "server_blocks_per_cu": serve_bpc, "server_group_max": serve_gmax, "server_group_min": serve_gmin,
                   "served": [params(c) | {"tuning": c.get("tuning")} for c in cfg_s],
                   "plain": [params(c) | {"tuning": c.get("tuning")} for c in cfg_p]},
        "closed_loop": {"queries": nc, "plain_qps": round(rate_plain, 2), "served_qps": round(nc / span_s0, 2),
                        "speedup": round(span_p0 / span_s0, 3)},
        "open_loop": {"lambda_qps": round(lam, 2),
                      "plain_qps": round(nq / span_p1, 2), "served_qps": round(nq / span_s1, 2),
                      "plain_ms": {"p50": pct(lat_p1, 50), "p99": pct(lat_p1, 99)},
                      "served_ms": {"p50": pct(lat_s1, 50), "p99": pct(lat_s1, 99)},
                      "by_graph_p50_ms": {"rmat": [pct(lat_p1[which == 0], 50), pct(lat_s1[which == 0], 50)],
                                          "grid": [pct(lat_p1[which == 1], 50), pct(lat_s1[which == 1], 50)],
                                          "order": ["plain", "served"]},
                      "served_gteps": round(edges_served / (span_s1 * 1e9), 4)},
        "same_alone_and_in_the_mix": same,
        "oracle_checked": checked,
        "roofline": None,
        "cpu_baseline": None if args.no_cpu_baseline else {
            "value": round(checked / csecs, 3), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{checked} of the trace's queries, one binary-heap Dijkstra each ({csecs:.1f} s, 1 thread)"},
    }
    for g in G:
        g.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--rho", type=int, default=0, help="rho for the timed solves (0 = the workload's default)")
    ap.add_argument("--delta", type=int, default=0, help="Delta for the road workload (0 = its default, 2^15)")
    ap.add_argument("--sweep", default="16,17,18,19,20,21,22", metavar="LOG2_LIST",
                    help="rho values (log2) timed first, one solve per source each; the timed solves use the "
                         "fastest ('' = no sweep)")
    ap.add_argument("--defer", default="", metavar="DEGREE,DIV[,LIST_DIVISOR]",
                    help="hub deferral (and optionally the explicit-list divisor) for the timed solves "
                         "(skips the deferral sweep)")
    ap.add_argument("--no-defer-sweep", dest="defer_sweep", action="store_false",
                    help="time the fastest rho of the paper's rule only")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="rmat24: skip the gather / atomic-minimum ceiling microbenchmarks")
    ap.add_argument("--cpu-runs", type=int, default=3, help="timed runs of the CPU oracle (the median is reported)")
    ap.add_argument("--extras", default="road,knn,latency",
                    help="rmat24: further workloads whose figures join the line (road: Delta / BF sweep on "
                         "road5000; knn: 64 batched queries against 64 single launches; latency: a short "
                         "serving run); '' = none")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sources", type=int, default=10,
                    help="rmat24: seeded sources in the largest component; timed solve i uses source i mod K")
    ap.add_argument("--queries", type=int, default=600, help="serving: queries in the trace")
    ap.add_argument("--latency-queries", type=int, default=1000,
                    help="rmat24: queries of the short serving run whose p50/p99 join the line (0 = skip)")
    ap.add_argument("--closed-queries", type=int, default=2000,
                    help="serving: queries of the closed-loop (saturation) runs, a prefix of the trace (0 = all)")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0,
                    help="serving: device-memory admission budget (GiB), split between the servers in "
                         "proportion to their grids")
    ap.add_argument("--serve-bpc", default="2,2",
                    help="serving: workgroups per CU of the R-MAT and grid servers (sum at most 4)")
    ap.add_argument("--serve-group-max", default="8,16",
                    help="serving: most teams per request on the R-MAT and grid servers (0 = all of them; "
                         "half of each server by default, so a request that arrives while another runs "
                         "finds idle teams)")
    ap.add_argument("--serve-group-min", default="4,4",
                    help="serving: fewest teams per request on the R-MAT and grid servers (a request waits "
                         "while fewer are idle rather than run on one or two teams)")
    ap.add_argument("--serve-teams", default="16,32",
                    help="serving: teams of the R-MAT and grid servers (with --serve-bpc 2,2 on 256 CUs: 16 "
                         "R-MAT teams of 32 workgroups, 32 grid teams of 16); a request takes a group of "
                         "idle teams, all of them when it is alone")
    ap.add_argument("--serve-rho", type=int, default=0,
                    help="serving: the R-MAT server's rho per team (0 = 2^17 / its teams)")
    ap.add_argument("--serve-delta", type=int, default=0,
                    help="serving: the grid server's Delta per team (0 = 67584 / its teams)")
    ap.add_argument("--serve-no-defer", dest="serve_defer", action="store_false",
                    help="serving: the paper's rho rule for the R-MAT queries (default: hub deferral)")
    ap.add_argument("--oracle-sample", type=int, default=4, help="serving: queries per graph checked by the oracle")
    ap.add_argument("--tune-budget", type=float, default=20.0,
                    help="seconds of parameter search per mode for the batched and serving workloads "
                         "(0 = the workload defaults, or for serving the settings of an earlier full search)")
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

    if args.workload == "serve":
        print(json.dumps(run_serve(args, torch, sp)), flush=True)
        return
    t0 = time.time()
    nsrc = BATCHED.get(args.workload, args.sources if args.workload == "rmat24" else 1)
    w = graphgen.workload(args.workload, sources=nsrc)
    log(f"workload {args.workload}: n={w.graph.n} m={w.graph.m} sources={len(w.sources)} "
        f"(generated in {time.time() - t0:.1f}s)")
    if args.workload in BATCHED:
        res = run_batched(args, torch, sp, w)
    else:
        res = run_single(args, torch, sp, w)
        extras = [x for x in args.extras.split(",") if x] if args.workload == "rmat24" else []
        del w
        # Further workloads of the metric, each in its own key; a failure in
        # one is recorded there and leaves the throughput line standing.
        if "road" in extras:
            try:
                res["road_delta_sweep"] = run_road_sweep(args, torch, sp)
            except Exception as e:
                res["road_delta_sweep"] = {"error": f"{type(e).__name__}: {e}"}
        if "knn" in extras:
            try:
                res["knn_batched"] = run_knn_compare(args, torch, sp)
            except Exception as e:
                res["knn_batched"] = {"error": f"{type(e).__name__}: {e}"}
        if "latency" in extras and args.latency_queries > 0:
            # The metric's latency half: a short serving run (both graphs of the
            # serving workload resident) against the one-at-a-time loop.
            la = argparse.Namespace(**vars(args))
            la.queries, la.tune_budget, la.oracle_sample = args.latency_queries, 0.0, 1
            la.closed_queries = args.latency_queries
            try:
                srv = run_serve(la, torch, sp)
                res["latency"] = {k: srv[k] for k in ("closed_loop", "open_loop", "same_alone_and_in_the_mix",
                                                       "oracle_checked")}
                res["latency"]["workload"] = srv["config"]["workload"]
                res["latency"]["queries"] = la.queries
            except Exception as e:  # the throughput line above stands on its own
                res["latency"] = {"error": f"{type(e).__name__}: {e}"}
    torch.cuda.synchronize()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
