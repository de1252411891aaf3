"""Per-graph parameter search for the stepping solver.

The stepping rules reach the same distances for every parameter (Sec. 3.2,
Table 2); rho, Delta and the kernel's tuning knobs change only the number of
steps and the redundant work, and the best values depend on the graph (the
paper picks rho per graph and motivates a rule that needs no preprocessing).
This module searches them by timing real solves on the device:

  1. the rule parameter, from large to small (large values mean few steps,
     small ones many; the time is taken to fall and then rise along the way,
     so the sweep stops once two values in a row are more than 5% slower
     than the best; a flat stretch, such as rho above every queue size, does
     not stop it):
     rho over powers of four from n down to 2^8, Delta over the median arc
     weight times powers of four; then the neighbouring powers of two;
  2. for batches, the number of teams the persistent grid is split into;
  3. on graphs that relax locally (average out-degree below the library's
     super-sparse threshold, Sec. 6 on large neighbour sets), the rule
     parameter and the local-expansion budget together: a larger Delta (or
     rho) puts more hops into one step, and with the default budget the
     expansion then stops short of them and the steps multiply, so values
     up to four times the best are tried with budgets grown alike;
  4. on graphs with high-degree vertices (out-degree 32 and up) and the
     rho rule, rho and hub deferral together: deferring the hubs to a much
     smaller threshold removes most of their repeated relaxations, and the
     larger rho it allows cuts the steps, so values up to eight times the
     best are tried with three (degree, divisor) settings;
  5. the hub-degree threshold, the size of the arc chunks hubs are cut into
     (the tile shape of their relaxation), the explicit-list switch, then
     the queue structure (flat array or tournament tree, Sec. 4).

Each candidate is timed `reps` times (median of the kernel time). Results are
cached per (graph fingerprint, batch-size class) in a JSON file, so a graph
seen again, or another graph of the same shape summary, is solved with its
tuned parameters at once.
"""

from __future__ import annotations

import json
import math
import os
import time
from typing import Callable


def batch_class(nsrc: int) -> int:
    """1 for single solves, else the power of two >= nsrc (min 8)."""
    if nsrc <= 1:
        return 1
    return max(8, 1 << (nsrc - 1).bit_length())


def rho_candidates(n: int) -> list[int]:
    """Powers of four from about n down to 2^8, largest first."""
    top = max(8, (max(n, 2) - 1).bit_length())
    return [1 << k for k in range(top - (top - 8) % 2, 7, -2)]


def delta_candidates(w_median: int) -> list[int]:
    """The median arc weight times 4^5 down to 4^-1, largest first."""
    base = max(1, int(w_median))
    return [max(1, base << k) if k >= 0 else max(1, base >> -k) for k in range(10, -3, -2)]


# The library's defaults for local expansion (sssp_tuning.local_budget and
# super_sparse_degree).
DEFAULT_LOCAL_BUDGET = 4096
SUPER_SPARSE_DEGREE = 10


def local_candidates(v0: int) -> list[tuple[int, int]]:
    """(rule parameter, local budget) pairs tried around the best parameter
    v0 found with the default budget: v0 with twice the budget, 2 * v0 with
    2 and 4 times it, 4 * v0 with 4 and 8 times it."""
    b = DEFAULT_LOCAL_BUDGET
    return [(v0, 2 * b), (2 * v0, 2 * b), (2 * v0, 4 * b), (4 * v0, 4 * b), (4 * v0, 8 * b)]


# (hub_defer_degree, hub_defer_div) settings tried with rho.
DEFER_SETTINGS = [(32, 1000), (64, 300), (128, 100)]


def defer_candidates(v0: int) -> list[tuple[int, int, int]]:
    """(rho, hub_defer_degree, hub_defer_div) triples tried around the best
    rho v0 found without deferral: v0, 2 v0, 4 v0 and 8 v0 with each setting
    (deferral moves the best rho up by about 4x, and the best rho of the
    paper's rule is flat over a factor of two or more)."""
    return [(v, deg, div) for v in (v0, 2 * v0, 4 * v0, 8 * v0) for deg, div in DEFER_SETTINGS]


def has_hubs(degree_log2_hist) -> bool:
    """Whether a graph has vertices of out-degree 32 or more (its log2
    out-degree histogram reaches bin 5)."""
    return len(degree_log2_hist or []) > 5 and any(degree_log2_hist[5:])


def relaxes_locally(n: int, m: int) -> bool:
    """Whether the library runs local expansion on a graph of this size
    (average out-degree below the super-sparse threshold)."""
    return n > 0 and m < SUPER_SPARSE_DEGREE * n


def team_candidates(nsrc: int, grid: int = 1024) -> list[int]:
    out, t = [], 8
    while t <= grid and t < 2 * max(nsrc, 8):
        out.append(t)
        t *= 2
    return out


class Tuner:
    """Coordinate search over (rule parameter, teams, local_budget, hub
    deferral, hub_degree, chunk_edges, list_divisor, queue).

    `measure(config) -> ms` times one configuration; by default it runs the
    solver on the given graph and sources. A config is a dict with keys rule,
    rho or delta, and tuning (a dict of sssp_tuning fields).
    """

    def __init__(self, cache_path: str | None = None, budget_s: float = 60.0, reps: int = 2,
                 measure: Callable[[dict], float] | None = None, log: Callable[[str], None] | None = None):
        self.cache_path = cache_path
        self.budget_s = budget_s
        self.reps = reps
        self._measure = measure
        self._log = log or (lambda s: None)
        self.history: list[tuple[dict, float]] = []

    # -- cache ------------------------------------------------------------
    def _load(self) -> dict:
        if not self.cache_path or not os.path.exists(self.cache_path):
            return {}
        with open(self.cache_path) as f:
            return json.load(f)

    def _store(self, key: str, value: dict):
        if not self.cache_path:
            return
        d = self._load()
        d[key] = value
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    @staticmethod
    def key(fingerprint: str, nsrc: int) -> str:
        return f"{fingerprint}/{batch_class(nsrc)}"

    def lookup(self, fingerprint: str, nsrc: int) -> dict | None:
        return self._load().get(self.key(fingerprint, nsrc))

    # -- search -----------------------------------------------------------
    def _eval(self, cfg: dict, best: list) -> float:
        ms = self._measure(cfg)
        self.history.append((cfg, ms))
        self._log(f"autotune {json.dumps(cfg, sort_keys=True)}: {ms:.3f} ms")
        if ms < best[1]:
            best[0], best[1] = cfg, ms
        return ms

    def search(self, n: int, nsrc: int, w_median: int, rules=("rho", "delta"), grid: int = 1024,
               local: bool = False, hubs: bool = False) -> dict:
        t0 = time.monotonic()
        best = [None, math.inf]

        def out_of_time():
            return time.monotonic() - t0 > self.budget_s

        def with_tuning(cfg, **kw):
            c = dict(cfg)
            c["tuning"] = {**cfg.get("tuning", {}), **kw}
            return c

        base_tuning = {"teams": 0} if nsrc > 1 else {}
        # 1. rule parameter: coarse (x4), then the two neighbours (x2).
        for rule in rules:
            if rule == "rho":
                name, cands = "rho", rho_candidates(n)
            elif rule == "delta":
                name, cands = "delta", delta_candidates(w_median)
            else:
                self._eval({"rule": rule, "tuning": dict(base_tuning)}, best)
                continue
            scores = {}
            worse = 0
            for v in cands:
                if (out_of_time() and best[0] is not None) or worse >= 2:
                    break
                scores[v] = self._eval({"rule": rule, name: v, "tuning": dict(base_tuning)}, best)
                worse = worse + 1 if scores[v] > 1.05 * min(scores.values()) else 0
            if not scores:
                continue
            v0 = min(scores, key=scores.get)
            for v in (v0 // 2, v0 * 2):
                if v >= 1 and v not in scores and not out_of_time():
                    scores[v] = self._eval({"rule": rule, name: v, "tuning": dict(base_tuning)}, best)
        # 3. rule parameter and local-expansion budget together.
        if local and best[0] is not None and best[0]["rule"] in ("rho", "delta"):
            name = best[0]["rule"]
            for v, budget in local_candidates(best[0][name]):
                if out_of_time():
                    break
                self._eval({"rule": name, name: v, "tuning": {**base_tuning, "local_budget": budget}}, best)
        # 4. rho and hub deferral together.
        if hubs and best[0] is not None and best[0]["rule"] == "rho":
            for v, deg, div in defer_candidates(best[0]["rho"]):
                if out_of_time():
                    break
                tun = {**best[0].get("tuning", {}), "hub_defer_degree": deg, "hub_defer_div": div}
                self._eval({"rule": "rho", "rho": v, "tuning": tun}, best)
        # 2., 5. kernel knobs, one at a time around the best so far.
        knobs = []
        if nsrc > 1:
            knobs.append(("teams", team_candidates(nsrc, grid)))
        knobs.append(("hub_degree", [256, 1024, 4096]))
        knobs.append(("chunk_edges", [1024, 4096, 16384]))
        knobs.append(("list_divisor", [16, 64, 256]))
        knobs.append(("queue", [1]))
        for knob, values in knobs:
            start = best[0]
            for v in values:
                if out_of_time():
                    break
                if start.get("tuning", {}).get(knob) == v:
                    continue
                self._eval(with_tuning(start, **{knob: v}), best)
        cfg = dict(best[0])
        cfg["ms"] = best[1]
        cfg["evaluations"] = len(self.history)
        return cfg

    def tune(self, graph, sources, rules=("rho", "delta"), force: bool = False) -> dict:
        """Tuned configuration for solving `sources` on `graph` (a Graph):
        from the cache when present, else searched now and cached."""
        nsrc = len(sources)
        fp = graph.fingerprint
        if not force:
            hit = self.lookup(fp, nsrc)
            if hit is not None:
                return hit
        if self._measure is None:
            from . import solve

            def measure(cfg):
                kw = {k: v for k, v in cfg.items() if k in ("rho", "delta")}
                times = []
                for _ in range(self.reps):
                    _, st = solve(graph, sources, rule=cfg["rule"], tuning=cfg.get("tuning") or None, **kw)
                    times.append(st["device_ms"])
                times.sort()
                return times[len(times) // 2]
            self._measure = measure
        w_median = graph.summary.get("weight_q10_50_90", [0, 1, 0])[1] or 1
        cfg = self.search(graph.n, nsrc, w_median, rules, local=relaxes_locally(graph.n, getattr(graph, "m", 0)),
                          hubs=has_hubs(graph.summary.get("degree_log2_hist")))
        self._store(self.key(fp, nsrc), cfg)
        return cfg


def solve_tuned(graph, sources, tuner: Tuner, **kw):
    """Solve with the tuner's configuration for this graph and batch size."""
    from . import solve
    cfg = tuner.tune(graph, sources)
    params = {k: v for k, v in cfg.items() if k in ("rho", "delta")}
    return solve(graph, sources, rule=cfg["rule"], tuning=cfg.get("tuning") or None, **params, **kw)
