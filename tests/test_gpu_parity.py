"""Parity of the HIP stepping loop with the CPU oracle, through the C ABI.

Distances are integers, so the bar is bit-exact equality with the oracle's
Dijkstra on the same seeded graph, for every rule and parameter (all stepping
rules reach the same array: Sec. 3.2 and Table 2). Step-level properties are
checked where the paper fixes them: the theta = min rule's exact step count,
Lemma 5.1's extraction bound, Bellman-Ford's k_n + 1 steps and Thm. 5.5's
Delta* step bound.
"""

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

INF = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.fixture(scope="module")
def sp(torch_cuda):
    import paper_2105_06145_amd as sp
    return sp


def run(sp, g, sources, **kw):
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    try:
        dist, st = sp.solve(G, sources, **kw)
        return sp.to_numpy_u64(dist), st
    finally:
        G.close()


def ref(g, s):
    return oracle.dijkstra(g.offsets, g.targets, g.weights, int(s))


def assert_same(got, exp, what=""):
    if not np.array_equal(got, exp):
        bad = np.flatnonzero(got != exp)
        v = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} vertices differ; first {v}: gpu {int(got[v])} oracle {int(exp[v])}")


RULES = [("rho", {"rho": 1}), ("rho", {"rho": 3}), ("rho", {"rho": 64}), ("rho", {"rho": 1 << 30}),
         ("rho", {"rho": 8, "tuning": {"hub_defer_degree": 2, "hub_defer_div": 4}}),
         ("rho", {"rho": 3, "tuning": {"hub_defer_degree": 1, "hub_defer_div": 0xFFFFFFFF}}),
         ("rho_exact", {"rho": 1}), ("rho_exact", {"rho": 7}), ("rho_exact", {"rho": 100}),
         ("delta", {"delta": 1}), ("delta", {"delta": 777}), ("delta", {"delta": 1 << 40}), ("bf", {}),
         ("min", {})]


def tiny_graph(rng):
    n = int(rng.integers(1, 130))
    m = int(rng.integers(0, 5 * n + 1))
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    wmax = int(rng.choice([1, 5, 1000, 2**32 - 1]))
    w = rng.integers(1, wmax + 1, m, dtype=np.int64)
    w[rng.random(m) < 0.1] = 0
    return graphgen.from_arcs(n, src, dst, w)


def test_tiny_random_graphs_all_rules(sp):
    rng = np.random.default_rng(2024)
    for i in range(120):
        g = tiny_graph(rng)
        s = int(rng.integers(0, g.n))
        exp = ref(g, s)
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
        for rule, kw in RULES:
            dist, _ = sp.solve(G, [s], rule=rule, seed=i, **kw)
            assert_same(sp.to_numpy_u64(dist)[0], exp, f"graph {i} n={g.n} m={g.m} rule {rule} {kw}")
            if i % 4 == 0:
                dist, _ = sp.solve(G, [s], rule=rule, seed=i, snapshot_keys=True, **kw)
                assert_same(sp.to_numpy_u64(dist)[0], exp, f"graph {i} rule {rule} {kw} snapshot keys")
        G.close()


def test_grid256_rho4096(sp):
    w = graphgen.workload("grid256")
    g = w.graph
    got, st = run(sp, g, w.sources[:1], rule="rho", rho=4096)
    exp = ref(g, w.sources[0])
    assert_same(got[0], exp, "grid256 rho=4096")
    assert oracle.certificate(g.offsets, g.targets, g.weights, int(w.sources[0]), got[0]) == (0, -1)
    assert st["steps"] > 1 and st["edges_relaxed"] >= g.m


def test_theta_min_exact_loop_counts(sp):
    # w >= 1: each step extracts exactly the queue minimum's ties, all final.
    g = graphgen.grid2d(96, 80, 1, 40, seed=5)
    for s in (0, 4000):
        exp = ref(g, s)
        got, st = run(sp, g, [s], rule="min")
        assert_same(got[0], exp, "min rule")
        assert st["steps"] == oracle.distinct_finite(exp)
        assert st["extracted"] == int((exp != INF).sum())
        assert st["edges_relaxed"] == oracle.reachable_arcs(g.offsets, exp)
        assert st["local_vertices"] == 0  # nothing lands at or below theta = min when w >= 1


NO_LOCAL = dict(local_budget=0xFFFFFFFF)  # Alg. 1 as printed: every relaxed vertex went through Extract


def test_extraction_bound_lemma_5_1(sp):
    # Positive weights: vertex v is extracted at most max(1, hop[v]) times.
    # Without local expansion every reachable vertex is extracted; with it,
    # vertices relaxed inside a step need no extraction, and the bound holds.
    g = graphgen.road(120, 120, seed=8)
    s = int(graphgen.pick_sources(g.n, 1, 9, graphgen.largest_component(g))[0])
    exp = ref(g, s)
    hop, kn = oracle.hop_depth(g.offsets, g.targets, g.weights, s, exp)
    bound = np.maximum(hop, 1)
    bound[hop < 0] = 0
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for rule, kw in [("rho", {"rho": 512}), ("delta", {"delta": 4000}), ("bf", {})]:
        for tun in (NO_LOCAL, None):
            dist, st = sp.solve(G, [s], rule=rule, extract_counts=True, tuning=tun, **kw)
            assert_same(sp.to_numpy_u64(dist)[0], exp, rule)
            cnt = st["extract_counts"].cpu().numpy()[0]
            assert np.all(cnt <= bound), (rule, tun, int(np.argmax(cnt - bound)))
            if tun is NO_LOCAL:
                assert np.all(cnt[hop >= 0] >= 1)
            assert int(cnt.sum()) == st["extracted"]
    G.close()


def test_step_bounds_bf_and_delta_star(sp):
    g = graphgen.road(150, 150, seed=10)
    s = int(graphgen.pick_sources(g.n, 1, 11, graphgen.largest_component(g))[0])
    exp = ref(g, s)
    _, kn = oracle.hop_depth(g.offsets, g.targets, g.weights, s, exp)
    L = int(g.weights.max())
    got, st = run(sp, g, [s], rule="bf")
    assert_same(got[0], exp, "bf")
    assert st["steps"] <= kn + 1
    for delta in (1 << 10, 1 << 13, 1 << 16):
        got, st = run(sp, g, [s], rule="delta", delta=delta)
        assert_same(got[0], exp, f"delta {delta}")
        assert st["steps"] <= -(-kn * L // delta) + kn + 1


def test_rho_small_queue_extracts_everything(sp):
    g = graphgen.rmat(13, 8, seed=12)
    s = int(np.argmax(g.degrees()))
    exp = ref(g, s)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for rho in (16, 300, 5000):
        dist, st = sp.solve(G, [s], rule="rho", rho=rho, trace=4096)
        assert_same(sp.to_numpy_u64(dist)[0], exp, f"rho {rho}")
        recs = st["trace"]
        assert len(recs) == st["steps"]
        large_seen = 0  # steps whose queue exceeded rho / 10: the first two use rho / 10
        for r in recs:
            rho10 = max(1, rho // 10)
            rho_eff = rho10 if large_seen < 2 else rho
            if r["q"] > rho10:
                large_seen += 1
            if r["q"] <= rho_eff:
                assert r["extracted"] == r["q"] and not (r["flags"] & 4)
            else:
                assert r["flags"] & 4 and r["samples"] > 0
                assert 1 <= r["extracted"] <= r["q"]
        assert sum(r["extracted"] for r in recs) == st["extracted"]
        assert sum(r["edges"] for r in recs) == st["edges_relaxed"]
    G.close()


@pytest.mark.parametrize("name", ["rmat16", "road300", "knn30"])
def test_medium_workloads_every_rule(sp, name):
    if name == "knn30":
        g = graphgen.knn(30, 400, 0.01, 10, 1e6, seed=4001)
        srcs = graphgen.pick_sources(g.n, 2, 4003)
    else:
        w = graphgen.workload(name, sources=2)
        g, srcs = w.graph, w.sources
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for s in srcs:
        exp = ref(g, s)
        for rule, kw in [("rho", {"rho": 1 << 8}), ("rho", {"rho": 1 << 14}), ("delta", {"delta": 1 << 12}),
                         ("delta", {"delta": 1 << 17}), ("bf", {})]:
            dist, _ = sp.solve(G, [s], rule=rule, **kw)
            assert_same(sp.to_numpy_u64(dist)[0], exp, f"{name} src {s} {rule} {kw}")
    G.close()


def test_tuning_variants_do_not_change_distances(sp):
    g = graphgen.rmat(15, 16, seed=14)
    s = int(np.argmax(g.degrees()))
    exp = ref(g, s)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    variants = [dict(hub_degree=1, chunk_edges=64), dict(hub_degree=64, chunk_edges=64),
                dict(list_divisor=0xFFFFFFFF), dict(list_divisor=1), dict(no_filter=1), dict(blocks_per_cu=1),
                dict(sample_cap=16, probe_cap=16), dict(hub_degree=1 << 20), dict(local_budget=0xFFFFFFFF),
                dict(local_budget=1), dict(local_budget=16, super_sparse_degree=1 << 20),
                dict(local_budget=1 << 20, super_sparse_degree=1 << 20, list_divisor=1)]
    for tv in variants:
        for rule, kw in [("rho", {"rho": 2048}), ("bf", {})]:
            dist, _ = sp.solve(G, [s], rule=rule, tuning=tv, **kw)
            assert_same(sp.to_numpy_u64(dist)[0], exp, f"tuning {tv} {rule}")
    G.close()
    # The caller's vertex order kept internally (no degree renumbering).
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    for rule, kw in [("rho", {"rho": 2048}), ("delta", {"delta": 3000}), ("bf", {})]:
        dist, st = sp.solve(G, [s], rule=rule, extract_counts=True, **kw)
        assert_same(sp.to_numpy_u64(dist)[0], exp, f"keep order {rule}")
        assert int(st["extract_counts"].sum()) == st["extracted"]
    G.close()


def test_local_expansion_on_road_graphs(sp):
    """Local expansion (Sec. 6, large neighbour sets) leaves every distance
    as it is and, on a high-diameter graph, needs far fewer steps."""
    g = graphgen.road(120, 120, seed=23)
    s = 777
    exp = ref(g, s)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    for rule, kw in [("delta", {"delta": 2000}), ("delta", {"delta": 200000}), ("bf", {}), ("rho", {"rho": 64})]:
        steps = {}
        for name, tun in [("off", dict(local_budget=0xFFFFFFFF)), ("on", None), ("small", dict(local_budget=8)),
                          ("all", dict(super_sparse_degree=1 << 20, local_budget=1 << 16))]:
            dist, st = sp.solve(G, [s], rule=rule, tuning=tun, **kw)
            assert_same(sp.to_numpy_u64(dist)[0], exp, f"{rule} {kw} local {name}")
            steps[name] = st["steps"]
            if name == "off":
                assert st["local_vertices"] == 0
            if name == "all":
                assert st["local_vertices"] > 0
        assert steps["all"] < steps["off"], (rule, kw, steps)
    G.close()


def test_local_expansion_row_mode_and_its_fallbacks(sp, torch_cuda):
    """Local expansion lists carry each vertex's row from the arc that
    listed it (row mode); without those rows (borrowed arrays), with the
    repeated-push skip, with more teams and with a budget that overflows the
    LDS lists, the next round reads the offsets. Every form gives the
    oracle's distances."""
    import torch
    g = graphgen.road(150, 150, seed=29)
    srcs = [11, 9000, 20000]
    exp = [ref(g, s) for s in srcs]
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    off_d = torch.from_numpy(g.offsets.astype(np.int64)).cuda()
    tgt_d = torch.from_numpy(g.targets.astype(np.int32)).cuda()
    wt_d = torch.from_numpy(g.weights.astype(np.uint32).view(np.int32)).cuda()
    B = sp.Graph.from_csr(off_d, tgt_d, wt_d, borrow=True)
    try:
        for graph, name in ((G, "copied"), (B, "borrowed")):
            for tun in ({}, {"repeat_skip": 1}, {"teams": 8}, {"local_budget": 1 << 16, "super_sparse_degree": 1 << 20},
                        {"local_budget": 3}):
                for rule, kw in (("delta", {"delta": 3000}), ("rho", {"rho": 128})):
                    d, st = sp.solve(graph, srcs, rule=rule, tuning=tun or None, **kw)
                    got = sp.to_numpy_u64(d)
                    for i, s in enumerate(srcs):
                        assert_same(got[i], exp[i], f"{name} {tun} {rule} source {s}")
    finally:
        G.close()
        B.close()


def test_bidirectional_relaxation(sp):
    """Pull-then-push relaxation (Sec. 6) on symmetric graphs leaves every
    distance as it is; it is refused on graphs not declared undirected, and
    an asymmetric graph declared undirected is rejected."""
    for g, s, rules in [(graphgen.rmat(14, 16, seed=24), None, [("rho", {"rho": 1000}), ("bf", {})]),
                        (graphgen.road(90, 90, seed=25), 4000, [("delta", {"delta": 3000}), ("rho", {"rho": 64})])]:
        s = int(np.argmax(g.degrees())) if s is None else s
        exp = ref(g, s)
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, undirected=True)
        for rule, kw in rules:
            for tun in (dict(pull=1), dict(pull=1, hub_degree=16, chunk_edges=64), dict(pull=1, local_budget=64),
                        dict(pull=0xFFFFFFFF)):
                dist, _ = sp.solve(G, [s], rule=rule, tuning=tun, **kw)
                assert_same(sp.to_numpy_u64(dist)[0], exp, f"{rule} {kw} {tun}")
            dist, _ = sp.solve(G, [s, 0, 5], rule=rule, tuning=dict(pull=1, teams=8), **kw)
            for i, src in enumerate([s, 0, 5]):
                assert_same(sp.to_numpy_u64(dist)[i], ref(g, src), f"batched pull {rule} row {i}")
        G.close()
    g = graphgen.rmat(10, 8, seed=26)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    with pytest.raises(sp.SSSPError) as ei:
        sp.solve(G, [0], tuning=dict(pull=1))
    assert ei.value.status == 1
    G.close()
    one_way = graphgen.from_arcs(4, [0, 1, 2], [1, 2, 3], [5, 5, 5])
    with pytest.raises(sp.SSSPError) as ei:
        sp.Graph.from_csr(one_way.offsets, one_way.targets, one_way.weights, undirected=True)
    assert ei.value.status == 2 and "symmetric" in str(ei.value)


TREE = dict(queue=1)  # tournament-tree LaB-PQ (Sec. 4.2, Alg. 2)


def test_tournament_tree_queue_parity(sp):
    """The tournament-tree queue gives the oracle's distances for every rule,
    with one team or many, and refuses unknown queue kinds."""
    rng = np.random.default_rng(60)
    for i in range(50):
        g = tiny_graph(rng)
        s = int(rng.integers(0, g.n))
        exp = ref(g, s)
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
        for rule, kw0 in RULES:
            for tun0 in (TREE, dict(queue=1, teams=8)):
                kw = {k: v for k, v in kw0.items() if k != "tuning"}
                tun = {**kw0.get("tuning", {}), **tun0}
                dist, _ = sp.solve(G, [s, 0], rule=rule, seed=i, tuning=tun, **kw)
                assert_same(sp.to_numpy_u64(dist)[0], exp, f"tree, graph {i} n={g.n} {rule} {kw} {tun}")
                assert_same(sp.to_numpy_u64(dist)[1], ref(g, 0), f"tree, graph {i} source 0 {rule} {kw} {tun}")
        G.close()
    for g, rules in [(graphgen.rmat(15, 16, seed=61), [("rho", {"rho": 256}), ("rho", {"rho": 1 << 14}),
                                                       ("rho_exact", {"rho": 2000}), ("delta", {"delta": 50000}),
                                                       ("bf", {})]),
                     (graphgen.road(120, 120, seed=62), [("delta", {"delta": 3000}), ("rho", {"rho": 64}),
                                                         ("min", {})])]:
        s = int(np.argmax(g.degrees()))
        exp = ref(g, s)
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
        for rule, kw in rules:
            for tun in (TREE, dict(queue=1, hub_degree=16, chunk_edges=64), dict(queue=1, local_budget=64),
                        dict(queue=1, no_filter=1)):
                dist, _ = sp.solve(G, [s], rule=rule, tuning=tun, **kw)
                assert_same(sp.to_numpy_u64(dist)[0], exp, f"tree {rule} {kw} {tun}")
        G.close()
    G = sp.Graph.from_csr(*(lambda t: (t.offsets, t.targets, t.weights))(graphgen.grid2d(8, 8, seed=63)))
    with pytest.raises(sp.SSSPError) as ei:
        sp.solve(G, [0], tuning=dict(queue=2))
    assert ei.value.status == 1
    G.close()


def test_tournament_tree_extracts_what_the_flat_array_extracts(sp):
    """With keys fixed at extraction (repeatable runs), the tree and the flat
    array are two implementations of one LaB-PQ: every step sees the same
    threshold, queue size, extracted set size and relaxed arcs."""
    for g, s, rules in [(graphgen.road(100, 100, seed=64), 5000, [("delta", {"delta": 2500}), ("bf", {}), ("min", {})]),
                        (graphgen.rmat(13, 8, seed=65), None, [("delta", {"delta": 40000}), ("bf", {})])]:
        s = int(np.argmax(g.degrees())) if s is None else s
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
        for rule, kw in rules:
            traces = {}
            for name, tun in (("flat", None), ("tree", TREE)):
                dist, st = sp.solve(G, [s], rule=rule, tuning=tun, snapshot_keys=True, trace=1 << 16,
                                    extract_counts=True, **kw)
                assert_same(sp.to_numpy_u64(dist)[0], ref(g, s), f"{name} {rule}")
                traces[name] = ([(r["theta"], r["q"], r["extracted"], r["edges"]) for r in st["trace"]],
                                st["extract_counts"].cpu().numpy())
            a, b = traces["flat"][0], traces["tree"][0]
            first = next((i for i in range(min(len(a), len(b))) if a[i] != b[i]), min(len(a), len(b)))
            assert a == b, (rule, len(a), len(b), first, a[max(0, first - 1):first + 2], b[max(0, first - 1):first + 2])
            assert np.array_equal(traces["flat"][1], traces["tree"][1]), rule
        G.close()


def test_exact_rho_selection_on_a_star(sp):
    """With the exact rho-th key (NEXT-4 rule), a star whose leaf weights are
    a permutation of 1..N is settled rho leaves per step: the trace shows
    exactly rho extractions per step until at most rho leaves remain, and
    ties at theta are all extracted. (Local expansion is off: it would settle
    the whole star in the source's step.)"""
    N = 1000
    rng = np.random.default_rng(27)
    w = rng.permutation(N) + 1
    g = graphgen.from_arcs(N + 1, np.zeros(N, dtype=np.int64), np.arange(1, N + 1), w)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    for rho in (1, 7, 64, 999, 1000):
        dist, st = sp.solve(G, [0], rule="rho_exact", rho=rho, trace=4096, tuning=NO_LOCAL)
        assert_same(sp.to_numpy_u64(dist)[0], ref(g, 0), f"star rho {rho}")
        ext = [r["extracted"] for r in st["trace"]]
        assert ext[0] == 1 and sum(ext) == N + 1, (rho, ext[:5])
        qs = [r["q"] for r in st["trace"]]
        for r, q in zip(st["trace"][1:], qs[1:]):
            assert r["extracted"] == min(rho, q), (rho, r)
            assert bool(r["flags"] & 8) == (q > rho)
    G.close()
    # Ties: weights 1..10 each used 100 times; rho = 150 lands inside the
    # second weight class, so the step takes every leaf of weights 1 and 2.
    w = np.repeat(np.arange(1, 11), 100)
    g = graphgen.from_arcs(1001, np.zeros(1000, dtype=np.int64), np.arange(1, 1001), w)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    dist, st = sp.solve(G, [0], rule="rho_exact", rho=150, trace=64, tuning=NO_LOCAL)
    assert_same(sp.to_numpy_u64(dist)[0], ref(g, 0), "star ties")
    assert st["trace"][1]["extracted"] == 200 and st["trace"][1]["theta"] == 2
    G.close()


def test_crowded_bitmap_words_extract_each_member_once(sp):
    """Bitmap Extract below n/4 queued deals a round's members out over the
    workgroup. A star whose leaves fill 768 consecutive bitmap words (plus a
    word of 37 members and 3,000 words of one member) puts thousands of
    members in one workgroup's round when teams are small; every leaf's key
    is final when it is queued, so each leaf must be extracted exactly once
    whatever the threshold splits (a bit cleared by mistake leaves it never
    extracted, a bit left set extracts it twice)."""
    n = 1 << 18
    rng = np.random.default_rng(31)
    full = np.arange(0, 768 * 64)
    ragged = np.arange(768 * 64, 768 * 64 + 37)
    singles = (np.arange(1000, 4000) * 64 + rng.integers(0, 64, 3000))
    leaves = np.concatenate([full, ragged, singles])
    src = n - 1
    w = rng.permutation(leaves.size) + 1
    g = graphgen.from_arcs(n, np.full(leaves.size, src, dtype=np.int64), leaves, w)
    exp = ref(g, src)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    tun = dict(NO_LOCAL, blocks_per_cu=1, teams=16)
    dense_lane_steps = 0
    for rule, kw in [("rho", {"rho": 2000}), ("rho", {"rho": 40000}), ("rho_exact", {"rho": 5000}),
                     ("delta", {"delta": 9000}), ("bf", {}), ("min", {})]:
        dist, st = sp.solve(G, [src], rule=rule, tuning=tun, trace=1 << 16, extract_counts=True, **kw)
        assert_same(sp.to_numpy_u64(dist)[0], exp, f"crowded {rule} {kw}")
        xc = st["extract_counts"].cpu().numpy()[0]
        assert xc[src] == 1 and np.all(xc[leaves] == 1), (rule, kw, int(xc[leaves].min()), int(xc[leaves].max()))
        assert int(xc.sum()) == leaves.size + 1, (rule, kw)
        dense_lane_steps += sum(1 for r in st["trace"] if (r["flags"] & 1) and n // 64 < r["q"] < n // 4)
    assert dense_lane_steps > 0
    G.close()


def test_seeds_and_repeats_agree(sp):
    g = graphgen.rmat(14, 16, seed=15)
    s = int(np.argmax(g.degrees()))
    exp = ref(g, s)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for seed in range(8):
        dist, _ = sp.solve(G, [s], rule="rho", rho=500, seed=seed)
        assert_same(sp.to_numpy_u64(dist)[0], exp, f"seed {seed}")
    G.close()


def test_edge_cases(sp):
    # single vertex, no arcs
    g = graphgen.from_arcs(1, [], [], [])
    got, st = run(sp, g, [0])
    assert got.tolist() == [[0]] and st["steps"] == 1
    # isolated source in a bigger graph
    g = graphgen.from_arcs(200, [1, 2], [2, 3], [4, 5])
    got, _ = run(sp, g, [0], rule="bf")
    assert got[0][0] == 0 and np.all(got[0][1:] == INF)
    # self-loops and parallel arcs only
    g = graphgen.from_arcs(3, [0, 0, 0, 1, 1], [0, 1, 1, 1, 2], [0, 9, 4, 1, 0])
    for rule, kw in RULES:
        got, _ = run(sp, g, [0], rule=rule, **kw)
        assert got[0].tolist() == [0, 4, 4]
    # distances beyond 2^32: a 300-arc path of maximal weights
    n = 301
    g = graphgen.from_arcs(n, np.arange(300), np.arange(1, 301), np.full(300, 2**32 - 1))
    got, _ = run(sp, g, [0], rule="rho", rho=7)
    assert_same(got[0], (np.arange(n, dtype=np.uint64) * np.uint64(2**32 - 1)), "max weights")
    # vertex counts around a bitmap word boundary
    for n in (63, 64, 65, 127, 128, 129):
        rng = np.random.default_rng(n)
        g = graphgen.from_arcs(n, rng.integers(0, n, 4 * n), rng.integers(0, n, 4 * n),
                               rng.integers(0, 100, 4 * n))
        got, _ = run(sp, g, [n - 1], rule="rho", rho=5)
        assert_same(got[0], ref(g, n - 1), f"n={n}")


def test_multiple_sources_rows(sp):
    g = graphgen.road(80, 80, seed=16)
    srcs = [0, 17, 5000, 6399, 17]
    got, st = run(sp, g, srcs, rule="delta", delta=3000)
    assert got.shape == (5, g.n)
    for i, s in enumerate(srcs):
        assert_same(got[i], ref(g, s), f"row {i}")


def test_int32_offsets_and_device_input(sp, torch_cuda):
    torch = torch_cuda
    g = graphgen.rmat(12, 16, seed=17)
    s = int(np.argmax(g.degrees()))
    exp = ref(g, s)
    G = sp.Graph.from_csr(g.offsets.astype(np.int32), g.targets, g.weights)
    dist, _ = sp.solve(G, [s], rule="rho", rho=256)
    assert_same(sp.to_numpy_u64(dist)[0], exp, "int32 offsets")
    G.close()
    off = torch.from_numpy(g.offsets).cuda()
    tgt = torch.from_numpy(g.targets).cuda()
    w = torch.from_numpy(g.weights.view(np.int32)).cuda()
    G = sp.Graph.from_csr(off, tgt, w)
    dist, _ = sp.solve(G, [s], rule="bf")
    assert_same(sp.to_numpy_u64(dist)[0], exp, "device input")
    G.close()
    G = sp.Graph.from_csr(off.to(torch.int32), tgt, w)
    dist, _ = sp.solve(G, [s], rule="delta", delta=5000)
    assert_same(sp.to_numpy_u64(dist)[0], exp, "device input int32 offsets")
    G.close()


def test_device_validation_rejects_bad_graph(sp, torch_cuda):
    torch = torch_cuda
    off = torch.tensor([0, 2, 3, 3], dtype=torch.int64, device="cuda")
    tgt = torch.tensor([1, 7, 0], dtype=torch.int32, device="cuda")  # 7 >= n
    w = torch.ones(3, dtype=torch.int32, device="cuda")
    with pytest.raises(sp.SSSPError) as ei:
        sp.Graph.from_csr(off, tgt, w)
    assert ei.value.status == 2 and "index 1" in str(ei.value)
    off2 = torch.tensor([0, 2, 1, 3], dtype=torch.int64, device="cuda")
    with pytest.raises(sp.SSSPError):
        sp.Graph.from_csr(off2, torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda"), w)


def test_step_limit_and_bad_params(sp):
    g = graphgen.from_arcs(50, np.arange(49), np.arange(1, 50), np.ones(49))
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    with pytest.raises(sp.SSSPError) as ei:
        sp.solve(G, [0], rule="bf", max_steps=5, tuning=NO_LOCAL)
    assert ei.value.status == 6
    dist, st = sp.solve(G, [0], rule="bf", max_steps=50, tuning=NO_LOCAL)
    assert st["steps"] == 50  # 49 steps settle the path, one more empties Q
    # Local expansion walks the whole path within the first step.
    dist, st = sp.solve(G, [0], rule="bf", max_steps=5)
    assert st["steps"] <= 2 and st["local_vertices"] >= 49
    assert sp.to_numpy_u64(dist)[0].tolist() == list(range(50))
    for bad in (dict(rule="rho", rho=0), dict(rule="delta", delta=0)):
        with pytest.raises(sp.SSSPError) as ei:
            sp.solve(G, [0], **bad)
        assert ei.value.status == 1
    with pytest.raises(sp.SSSPError):
        sp.solve(G, [50])
    G.close()


def test_batched_teams_match_oracle(sp):
    """Many sources in one launch, for team counts that put each team inside
    one XCD (multiples of 8) and counts that do not (1 and 2)."""
    g = graphgen.rmat(13, 16, seed=21)
    rng = np.random.default_rng(21)
    srcs = [int(x) for x in rng.integers(0, g.n, 37)] + [0, 0]
    exp = {s: ref(g, s) for s in set(srcs)}
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for teams in (0, 1, 2, 8, 16, 64, 256):
        for rule, kw in [("rho", {"rho": 300}), ("delta", {"delta": 40000}), ("bf", {})]:
            dist, st = sp.solve(G, srcs, rule=rule, tuning=dict(teams=teams), **kw)
            got = sp.to_numpy_u64(dist)
            for i, s in enumerate(srcs):
                assert_same(got[i], exp[s], f"teams {teams} rule {rule} row {i} source {s}")
            assert st["teams"] == (teams or 64)
    G.close()


def test_batched_counts_equal_sum_of_single_solves(sp):
    """With snapshot keys, Relax uses the key each vertex was extracted with,
    so for rules whose thresholds do not depend on sampling (Delta*,
    Bellman-Ford, theta = min) each solve extracts the same sets whether its
    source runs alone or among others: step, extraction and relaxation totals of a batch are the sums
    over single solves, and the first source's trace is the same record for
    record (apart from the count of successful WriteMins, which depends on
    the order in which concurrent WriteMins land, and the phase times)."""
    g = graphgen.road(60, 60, seed=22)
    srcs = [0, 3599, 1234, 77, 2500, 999, 42, 3000, 1800, 5]
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for rule, kw in [("delta", {"delta": 2500}), ("bf", {}), ("min", {})]:
        tot = {"steps": 0, "extracted": 0, "edges_relaxed": 0}
        for s in srcs:
            _, st = sp.solve(G, [s], rule=rule, snapshot_keys=True, **kw)
            for k in tot:
                tot[k] += st[k]
        _, single = sp.solve(G, srcs[:1], rule=rule, trace=4096, snapshot_keys=True, **kw)
        for teams in (8, 16, 2):
            dist, st = sp.solve(G, srcs, rule=rule, tuning=dict(teams=teams), trace=4096,
                                extract_counts=True, snapshot_keys=True, **kw)
            for k in tot:
                assert st[k] == tot[k], (rule, teams, k)
            strip = lambda recs: [{k: v for k, v in r.items() if k not in ("successes", "extract_ns", "relax_ns")}
                                  for r in recs]
            assert strip(st["trace"][:single["steps"]]) == strip(single["trace"]), (rule, teams)
            counts = st["extract_counts"].cpu().numpy()
            assert counts.sum() == st["extracted"]
            got = sp.to_numpy_u64(dist)
            for i, s in enumerate(srcs):
                assert_same(got[i], ref(g, s), f"{rule} teams {teams} row {i}")
                if rule == "min":  # theta = min settles each reachable vertex exactly once
                    assert np.array_equal(counts[i], (got[i] != INF).astype(np.int32)), (teams, i)
    G.close()


def test_batched_knn_many_queries(sp):
    """The query workload: a kNN graph kept in the caller's vertex order and 64
    sources solved in one launch, auto team count."""
    w = graphgen.workload("knn10", sources=64)
    g = w.graph
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    dist, st = sp.solve(G, w.sources, rule="rho", rho=1 << 12)
    got = sp.to_numpy_u64(dist)
    assert st["teams"] == 64
    for i, s in enumerate(w.sources):
        assert_same(got[i], ref(g, s), f"knn row {i}")
    # Same answers one source at a time.
    for i in (0, 31, 63):
        d1, _ = sp.solve(G, w.sources[i:i + 1], rule="rho", rho=1 << 12)
        assert_same(sp.to_numpy_u64(d1)[0], got[i], f"knn single {i}")
    G.close()


def test_bad_team_counts_rejected(sp):
    g = graphgen.from_arcs(10, np.arange(9), np.arange(1, 10), np.ones(9))
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for teams in (3, 1 << 20):
        with pytest.raises(sp.SSSPError) as ei:
            sp.solve(G, [0, 1], tuning=dict(teams=teams))
        assert ei.value.status == 1 and "teams" in str(ei.value)
    G.close()


# ---------------------------------------------------------------------------
# Full-size workloads (the configurations the benchmark times).

@pytest.fixture(scope="module")
def rmat24():
    return graphgen.workload("rmat24", sources=2)


@pytest.fixture(scope="module")
def road5000():
    return graphgen.workload("road5000", sources=1)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_rmat24_rho_sweep(sp, rmat24):
    g = rmat24.graph
    s = int(rmat24.sources[0])
    exp = ref(g, s)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    for rho in (1 << 16, 1 << 18, 1 << 22):  # 2^18: the benchmark's setting
        dist, st = sp.solve(G, [s], rule="rho", rho=rho)
        got = sp.to_numpy_u64(dist)[0]
        assert_same(got, exp, f"rmat24 rho=2^{rho.bit_length() - 1}")
        print(f"rmat24 rho={rho} steps={st['steps']} edges={st['edges_relaxed']} ms={st['device_ms']:.2f}",
              flush=True)
    assert oracle.certificate(g.offsets, g.targets, g.weights, s, got) == (0, -1)
    # the tournament-tree queue and the stream-ordered call at full size
    dist, st = sp.solve(G, [s], rule="rho", rho=1 << 16, tuning={"queue": 1})
    assert_same(sp.to_numpy_u64(dist)[0], exp, "rmat24 tournament tree rho=2^16")
    print(f"rmat24 tree rho=65536 steps={st['steps']} ms={st['device_ms']:.2f}", flush=True)
    # hub deferral at the benchmark's deferral setting
    dist, st = sp.solve(G, [s], rule="rho", rho=1 << 21, tuning={"hub_defer_degree": 32, "hub_defer_div": 1000})
    assert_same(sp.to_numpy_u64(dist)[0], exp, "rmat24 hub deferral rho=2^21")
    print(f"rmat24 deferral rho=2^21 steps={st['steps']} edges={st['edges_relaxed']} ms={st['device_ms']:.2f}",
          flush=True)
    pending = sp.solve_async(G, [s], rule="rho", rho=1 << 18)
    dist, _ = pending.wait()
    assert_same(sp.to_numpy_u64(dist)[0], exp, "rmat24 asynchronous solve")
    # second source: certificate only (linear time)
    s2 = int(rmat24.sources[1])
    dist, _ = sp.solve(G, [s2], rule="rho", rho=1 << 20)
    assert oracle.certificate(g.offsets, g.targets, g.weights, s2, sp.to_numpy_u64(dist)[0]) == (0, -1)
    G.close()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_road5000_delta_star_and_bf(sp, road5000):
    g = road5000.graph
    s = int(road5000.sources[0])
    exp = ref(g, s)
    G = sp.Graph.from_csr(g.offsets.astype(np.int32), g.targets, g.weights)
    for rule, kw in [("delta", {"delta": 1 << 10}), ("delta", {"delta": 1 << 15}), ("delta", {"delta": 1 << 16}),
                     ("delta", {"delta": 1 << 16, "tuning": {"local_budget": 8192}}), ("bf", {})]:
        dist, st = sp.solve(G, [s], rule=rule, **kw)
        got = sp.to_numpy_u64(dist)[0]
        assert_same(got, exp, f"road5000 {rule} {kw}")
        print(f"road5000 {rule} {kw} steps={st['steps']} ms={st['device_ms']:.1f}", flush=True)
    G.close()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_knn10000_batched_rows(sp):
    """The batched benchmark configuration: 64 sources on the 10^7-point kNN
    graph in one launch. Four rows against the oracle, every row against the
    linear-time certificate."""
    w = graphgen.workload("knn10000", sources=64)
    g = w.graph
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    for rule, kw in [("rho", {"rho": 4096}), ("delta", {"delta": 1898, "tuning": {"teams": 64}})]:
        dist, st = sp.solve(G, w.sources, rule=rule, **kw)
        got = sp.to_numpy_u64(dist)
        print(f"knn10000 {rule} {kw}: teams={st['teams']} ms={st['device_ms']:.1f}", flush=True)
        for i in (0, 21, 42, 63):
            assert_same(got[i], ref(g, w.sources[i]), f"knn10000 {rule} row {i}")
        for i, s in enumerate(w.sources):
            assert oracle.certificate(g.offsets, g.targets, g.weights, int(s), got[i]) == (0, -1), (rule, i)
    G.close()


@pytest.mark.parametrize("teams", [1, 8])
def test_repeat_skip_keeps_distances(sp, teams):
    """Pushes skipped because the tail's key has not changed since its last
    push (per vertex, and per hub chunk with small hub rows and chunks) leave
    every distance as the oracle's, and on a graph where keys do repeat some
    arcs are skipped."""
    g = graphgen.rmat(14, 16, seed=81)
    srcs = [3, 4000, 11111]
    exp = [ref(g, s) for s in srcs]
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    try:
        skipped_any = 0
        for rule, kw in (("rho", {"rho": 64}), ("rho", {"rho": 2048}), ("delta", {"delta": 5000}), ("bf", {})):
            for tun in ({"hub_degree": 64, "chunk_edges": 64}, {}):
                on = {**tun, "repeat_skip": 1, "teams": teams}
                off = {**tun, "repeat_skip": 0xFFFFFFFF, "teams": teams}
                d_on, st_on = sp.solve(G, srcs, rule=rule, tuning=on, **kw)
                d_off, st_off = sp.solve(G, srcs, rule=rule, tuning=off, **kw)
                got_on, got_off = sp.to_numpy_u64(d_on), sp.to_numpy_u64(d_off)
                for i in range(len(srcs)):
                    assert_same(got_on[i], exp[i], f"{rule} {kw} {on} source {srcs[i]}")
                    assert_same(got_off[i], exp[i], f"{rule} {kw} {off} source {srcs[i]}")
                assert st_off["repeat_skipped"] == 0
                skipped_any += st_on["repeat_skipped"]
        assert skipped_any > 0
    finally:
        G.close()


@pytest.mark.parametrize("teams", [1, 8])
def test_hub_deferral_keeps_distances(sp, teams):
    """Hub deferral (high-degree vertices extracted only at keys <= theta_h in
    sampled rho steps) leaves every distance as the oracle's, with the tree
    queue, snapshot keys and tiny hub chunks too, and on a power-law graph
    relaxes fewer arcs."""
    g = graphgen.rmat(14, 16, seed=81)
    srcs = [3, 4000, 11111]
    exp = [ref(g, s) for s in srcs]
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    try:
        arcs = {}
        for rho in (16, 2048, 1 << 20):
            for tun in ({}, {"hub_defer_degree": 16, "hub_defer_div": 1000}, {"hub_defer_degree": 64},
                        {"hub_defer_degree": 1, "hub_defer_div": 4},
                        {"hub_defer_degree": 16, "hub_defer_div": 1000, "queue": 1},
                        {"hub_defer_degree": 2, "hub_defer_div": 0xFFFFFFFF, "hub_degree": 64, "chunk_edges": 64}):
                tv = {**tun, "teams": teams}
                for snap in (False, True):
                    d, st = sp.solve(G, srcs, rule="rho", rho=rho, tuning=tv, snapshot_keys=snap)
                    got = sp.to_numpy_u64(d)
                    for i in range(len(srcs)):
                        assert_same(got[i], exp[i], f"rho {rho} {tv} snapshot {snap} source {srcs[i]}")
                    if rho == 2048 and not snap and "queue" not in tun:
                        arcs[(tun.get("hub_defer_degree"), tun.get("hub_defer_div"))] = st["edges_relaxed"]
        assert arcs[(16, 1000)] < arcs[(None, None)], arcs
    finally:
        G.close()
    # Ignored on graphs kept in the caller's order; with local expansion on a
    # road-like graph (low-degree hubs deferred) the distances stay.
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    try:
        d, _ = sp.solve(G, srcs, rule="rho", rho=2048, tuning={"hub_defer_degree": 16, "teams": teams})
        for i in range(len(srcs)):
            assert_same(sp.to_numpy_u64(d)[i], exp[i], f"keep order source {srcs[i]}")
    finally:
        G.close()
    r = graphgen.road(60, 60, seed=5)
    rs = [0, 1234]
    G = sp.Graph.from_csr(r.offsets, r.targets, r.weights)
    try:
        for tun in ({"hub_defer_degree": 4, "hub_defer_div": 100}, {"hub_defer_degree": 1, "hub_defer_div": 3}):
            d, st = sp.solve(G, rs, rule="rho", rho=64, tuning={**tun, "teams": teams})
            for i, s in enumerate(rs):
                assert_same(sp.to_numpy_u64(d)[i], ref(r, s), f"road {tun} source {s}")
    finally:
        G.close()


def test_sampled_steps_draw_appendix_b_sample_size(sp):
    """rho-stepping draws App. B's sample size s = ceil(10 (q / rho' + log q))
    (log q = 1 + log2(q + 1)) in every sampled step: exactly s from the
    explicit list, and from the bitmap about 1.25 s n / q probes of which
    the queued ones are kept (their count near probes * q / n, at least s on
    average). rho' is rho / 10 in the first two steps whose queue exceeds
    rho / 10 (Sec. 6), else rho."""
    import math
    g = graphgen.rmat(16, 16, seed=83)
    n = g.n
    src = int(graphgen.pick_sources(n, 1, 84, graphgen.largest_component(g))[0])
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    try:
        checked = 0
        for rho in (64, 512, 4096):
            d, st = sp.solve(G, [src], rule="rho", rho=rho, trace=4096)
            assert_same(sp.to_numpy_u64(d)[0], ref(g, src), f"rho {rho}")
            rho10 = max(1, rho // 10)
            large = 0
            for r in st["trace"]:
                q = r["q"]
                rho_eff = rho10 if large < 2 else rho
                if q > rho10:
                    large += 1
                sampled = bool(r["flags"] & 4)
                assert sampled == (q > rho_eff), (rho, r)
                if not sampled:
                    continue
                s = math.ceil(10.0 * (q / rho_eff + 1.0 + math.log2(q + 1.0)))
                if r["flags"] & 1:  # bitmap step: rejection probing
                    probes = min(1 << 16, math.ceil(s * n / q * 1.25))
                    mean = probes * q / n
                    if probes < (1 << 16):
                        assert mean >= s
                    assert abs(r["samples"] - mean) <= 6 * math.sqrt(mean) + 1, (rho, q, s, r["samples"], mean)
                else:  # explicit list: exactly s samples
                    assert r["samples"] == min(s, 1 << 16), (rho, q, s, r["samples"])
                checked += 1
        assert checked > 10
    finally:
        G.close()


def test_borrowed_device_arrays_are_used_in_place(sp, torch_cuda):
    """SSSP_BORROW_DEVICE: the caller's device targets and weights are read in
    place (no packed copy): distances match the oracle, the graph holds no
    arc storage of its own, and weights changed in the caller's tensor are
    the weights of the next solve."""
    torch = torch_cuda
    g = graphgen.rmat(13, 16, seed=85)
    off = torch.from_numpy(g.offsets.astype(np.int64)).cuda()
    tgt = torch.from_numpy(g.targets.astype(np.int32)).cuda()
    w = torch.from_numpy(g.weights.view(np.int32).copy()).cuda()
    srcs = [0, 17, 4000]
    for undirected, tun in ((False, None), (True, {"pull": 1})):
        G = sp.Graph.from_csr(off, tgt, w, borrow=True, undirected=undirected)
        copied = sp.Graph.from_csr(off, tgt, w, reorder=False)
        try:
            # Graph storage: offsets only, against offsets and 8-byte arcs.
            assert G.device_bytes() == 8 * (g.n + 1)
            assert copied.device_bytes() == 8 * (g.n + 1) + 8 * g.m
            d, _ = sp.solve(G, srcs, rule="rho", rho=256, tuning=tun)
            got = sp.to_numpy_u64(d)
            for i, s in enumerate(srcs):
                assert_same(got[i], ref(g, s), f"borrowed, source {s}")
            w.mul_(3)  # in place, both arcs of a pair alike
            d, _ = sp.solve(G, srcs, rule="delta", delta=3000, tuning=tun)
            got = sp.to_numpy_u64(d)
            w3 = g.weights * np.uint32(3)
            for i, s in enumerate(srcs):
                assert_same(got[i], oracle.dijkstra(g.offsets, g.targets, w3, s), f"weights x3, source {s}")
            w.div_(3, rounding_mode="floor")
        finally:
            G.close()
            copied.close()
