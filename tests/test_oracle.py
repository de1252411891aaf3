"""Pins of the CPU oracle against things other than itself: hand-derived
fixtures, closed forms, brute force on tiny graphs, an independent library
(scipy) and planted mistakes that the certificate must reject. CPU only."""

import os

import numpy as np
import pytest

import graphgen
import oracle

INF = np.uint64(0xFFFFFFFFFFFFFFFF)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_fixture(name):
    lines = [ln.split("#")[0].strip() for ln in open(os.path.join(GOLDEN, name))]
    lines = [ln for ln in lines if ln]
    it = iter(lines)
    n = src = None
    arcs, dist, hop = [], None, None
    for ln in it:
        if ln.startswith("n "):
            n = int(ln.split()[1])
        elif ln.startswith("source "):
            src = int(ln.split()[1])
        elif ln == "arcs":
            continue
        elif ln == "dist":
            dist = [INF if x == "inf" else np.uint64(int(x)) for x in next(it).split()]
        elif ln == "hop":
            hop = [int(x) for x in next(it).split()]
        else:
            u, v, w = (int(x) for x in ln.split())
            arcs.append((u, v, w))
    a = np.array(arcs, dtype=np.int64)
    g = graphgen.from_arcs(n, a[:, 0], a[:, 1], a[:, 2])
    return g, src, np.array(dist, dtype=np.uint64), np.array(hop, dtype=np.int32)


@pytest.mark.parametrize("name", ["diamond.txt", "zero_cycle.txt"])
def test_golden_fixtures(name):
    g, s, dist, hop = load_fixture(name)
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
    assert np.array_equal(d, dist)
    assert np.array_equal(oracle.bellman_ford(g.offsets, g.targets, g.weights, s), dist)
    assert np.array_equal(oracle.floyd_warshall(g.offsets, g.targets, g.weights)[s], dist)
    h, k = oracle.hop_depth(g.offsets, g.targets, g.weights, s, d)
    assert np.array_equal(h, hop)
    assert k == hop.max()
    assert oracle.certificate(g.offsets, g.targets, g.weights, s, d) == (0, -1)


def random_tiny(rng, n, m, wmax, zero_frac=0.1):
    """Random digraph with multi-edges, self-loops and zero weights."""
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    w = rng.integers(1, wmax + 1, m)
    w[rng.random(m) < zero_frac] = 0
    return graphgen.from_arcs(n, src, dst, w)


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 65))
    m = int(rng.integers(0, 4 * n + 1))
    g = random_tiny(rng, n, m, int(rng.choice([1, 3, 100, 2**32 - 1])))
    D = oracle.floyd_warshall(g.offsets, g.targets, g.weights)
    for s in range(n):
        d = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
        assert np.array_equal(d, D[s]), (seed, s)
        assert np.array_equal(oracle.bellman_ford(g.offsets, g.targets, g.weights, s), D[s])
        assert oracle.certificate(g.offsets, g.targets, g.weights, s, d)[0] == 0


def test_brute_force_max_weights_no_overflow():
    # A path of 60 arcs of weight 2^32 - 1: distances reach 60 * (2^32 - 1).
    n = 61
    g = graphgen.from_arcs(n, np.arange(60), np.arange(1, 61), np.full(60, 2**32 - 1))
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, 0)
    assert d[60] == np.uint64(60 * (2**32 - 1))
    assert np.array_equal(d, oracle.floyd_warshall(g.offsets, g.targets, g.weights)[0])


def test_closed_form_unit_grid():
    # Unit weights on a W x H 4-neighbour grid: d = c * (|dx| + |dy|).
    W, H = 37, 23
    g = graphgen.grid2d(W, H, 1, 2, seed=3)  # weights uniform in [1, 2) -> all 1
    assert np.all(g.weights == 1)
    for sx, sy in [(0, 0), (18, 11), (36, 22)]:
        s = sy * W + sx
        d = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
        x = np.arange(W * H) % W
        y = np.arange(W * H) // W
        assert np.array_equal(d, (np.abs(x - sx) + np.abs(y - sy)).astype(np.uint64))
        hop, k = oracle.hop_depth(g.offsets, g.targets, g.weights, s, d)
        assert np.array_equal(hop, (np.abs(x - sx) + np.abs(y - sy)).astype(np.int32))
        assert k == max(sx, W - 1 - sx) + max(sy, H - 1 - sy)


def test_closed_form_path_star_complete_components():
    rng = np.random.default_rng(5)
    # Path: prefix sums.
    w = rng.integers(0, 1000, 99)
    g = graphgen.from_arcs(100, np.arange(99), np.arange(1, 100), w)
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, 0)
    assert np.array_equal(d, np.concatenate([[0], np.cumsum(w)]).astype(np.uint64))
    hop, k = oracle.hop_depth(g.offsets, g.targets, g.weights, 0, d)
    assert k == 99 and np.array_equal(hop, np.arange(100, dtype=np.int32))
    assert oracle.distinct_finite(d) == len(np.unique(d))
    # Star from the centre: d = w; from a leaf: w_leaf + w_other (undirected).
    w = rng.integers(1, 50, 20)
    src = np.concatenate([np.zeros(20, int), np.arange(1, 21)])
    dst = np.concatenate([np.arange(1, 21), np.zeros(20, int)])
    g = graphgen.from_arcs(21, src, dst, np.concatenate([w, w]))
    assert np.array_equal(oracle.dijkstra(g.offsets, g.targets, g.weights, 0)[1:], w.astype(np.uint64))
    d3 = oracle.dijkstra(g.offsets, g.targets, g.weights, 3)
    exp = (w + w[2]).astype(np.uint64)
    exp[2] = 0
    assert d3[0] == w[2] and np.array_equal(d3[1:], exp)
    # Complete digraph with unit weights: 1 everywhere but the source.
    n = 30
    uu, vv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = uu != vv
    g = graphgen.from_arcs(n, uu[keep], vv[keep], np.ones(keep.sum()))
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, 7)
    exp = np.ones(n, np.uint64)
    exp[7] = 0
    assert np.array_equal(d, exp)
    # Two components: the far side stays unreachable.
    g = graphgen.from_arcs(6, [0, 1, 3, 4], [1, 2, 4, 5], [1, 1, 1, 1])
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, 0)
    assert list(d[:3]) == [0, 1, 2] and np.all(d[3:] == INF)
    assert oracle.reachable_arcs(g.offsets, d) == 2


def test_chain_with_shortcuts():
    # Chain 0->1->...->k with unit arcs, plus parallel shortcuts i->i+2 of
    # weight 3 (never better) and 0->k of weight k (a tie with the chain).
    k = 50
    src = list(range(k)) + list(range(k - 1)) + [0]
    dst = list(range(1, k + 1)) + list(range(2, k + 1)) + [k]
    w = [1] * k + [3] * (k - 1) + [k]
    g = graphgen.from_arcs(k + 1, src, dst, w)
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, 0)
    assert np.array_equal(d, np.arange(k + 1, dtype=np.uint64))
    hop, kn = oracle.hop_depth(g.offsets, g.targets, g.weights, 0, d)
    assert hop[k] == 1 and kn == k - 1


@pytest.mark.parametrize("make", [
    lambda: graphgen.rmat(12, 16, seed=11),
    lambda: graphgen.road(60, 60, seed=12),
    lambda: graphgen.grid2d(50, 40, 1, 1 << 16, seed=13),
    lambda: graphgen.knn(20, 50, 0.01, 10, 1e6, seed=14),
])
def test_scipy_cross_check(make):
    # scipy's Dijkstra works in float64, exact for these integer sums (< 2^53).
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    g = make()
    A = csr_matrix((g.weights.astype(np.float64), g.targets, g.offsets), shape=(g.n, g.n))
    rng = np.random.default_rng(1)
    for s in rng.integers(0, g.n, 3):
        d = oracle.dijkstra(g.offsets, g.targets, g.weights, int(s))
        ref = sp_dijkstra(A, directed=True, indices=int(s))
        fin = np.isfinite(ref)
        assert np.array_equal(fin, d != INF)
        assert np.array_equal(ref[fin].astype(np.uint64), d[fin])


def test_certificate_rejects_planted_mistakes():
    g = graphgen.road(40, 40, seed=21)
    s = int(np.flatnonzero(g.degrees() > 0)[17])
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
    assert oracle.certificate(g.offsets, g.targets, g.weights, s, d) == (0, -1)
    fin = np.flatnonzero((d != INF) & (np.arange(g.n) != s))
    rng = np.random.default_rng(2)
    for v in rng.choice(fin, 20, replace=False):
        up = d.copy()
        up[v] += np.uint64(1)  # too large: the arc from its tight parent is tense
        code, bad = oracle.certificate(g.offsets, g.targets, g.weights, s, up)
        assert code == 2 and bad == v
        lo = d.copy()
        lo[v] -= np.uint64(1)  # too small: no tight path reaches it
        code, _ = oracle.certificate(g.offsets, g.targets, g.weights, s, lo)
        assert code in (2, 3)
    bad_src = d.copy()
    bad_src[s] = 1
    assert oracle.certificate(g.offsets, g.targets, g.weights, s, bad_src)[0] == 1
    # A finite value on an unreachable vertex (isolated component).
    g2 = graphgen.from_arcs(4, [0, 2], [1, 3], [5, 5])
    d2 = oracle.dijkstra(g2.offsets, g2.targets, g2.weights, 0)
    d2[2] = 7
    d2[3] = 12
    assert oracle.certificate(g2.offsets, g2.targets, g2.weights, 0, d2) == (3, 2)
    # All-INF except the source: arcs out of the source are tense.
    d3 = np.full(g.n, INF)
    d3[s] = 0
    assert oracle.certificate(g.offsets, g.targets, g.weights, s, d3)[0] == 2


def test_certificate_zero_weight_cycle_needs_search():
    # 0 -> 1 (5); cycle 2 <-> 3 with weight 0, not reachable from 0. Claiming
    # d(2) = d(3) = 1 leaves no tense arc, and each has a "tight" in-arc from
    # the other, but no tight path from the source: condition (iii) catches it.
    g = graphgen.from_arcs(4, [0, 2, 3], [1, 3, 2], [5, 0, 0])
    d = np.array([0, 5, 1, 1], dtype=np.uint64)
    assert oracle.certificate(g.offsets, g.targets, g.weights, 0, d)[0] == 3


def test_bounded_dijkstra_prefix():
    g = graphgen.rmat(12, 16, seed=31)
    s = int(np.argmax(g.degrees()))
    full, settled, scanned = oracle.dijkstra(g.offsets, g.targets, g.weights, s, stats=True)
    part, k, sc = oracle.dijkstra(g.offsets, g.targets, g.weights, s, max_settled=100, stats=True)
    assert k == 100 and sc <= scanned and settled == int((full != INF).sum())
    assert scanned == oracle.reachable_arcs(g.offsets, full)
    # The 100 settled vertices carry final distances; nothing is below truth.
    assert int((part == full).sum()) >= 100
    assert np.all(part >= full)


def test_theta_min_quantities():
    # For w >= 1 the theta = min rule (Table 2, Dijkstra row) takes one step
    # per distinct finite distance; helpers used by the GPU tests.
    g = graphgen.grid2d(10, 10, 1, 2, seed=1)
    d = oracle.dijkstra(g.offsets, g.targets, g.weights, 0)
    assert oracle.distinct_finite(d) == 19  # x + y in 0..18
    assert oracle.reachable_arcs(g.offsets, d) == g.m
