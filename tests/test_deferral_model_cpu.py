"""Hub deferral (an extension of the rho rule) on a plain CPU model of the
stepping loop (Alg. 1 with the rho rule of Table 2, exact rank instead of
sampling): every step extracts the queued vertices with key <= theta, except
that vertices of out-degree >= D need key <= theta_h, the (rho / div)-th
smallest key. The smallest key is always extracted, so the loop ends, and it
ends with the oracle's distances whatever D and div are, on graphs with zero
weights, ties and multi-edges (CPU; independent of the HIP path)."""

import numpy as np

import graphgen
import oracle

INF = np.iinfo(np.uint64).max


def model_rho_stepping(g, src, rho, D=None, div=None):
    n = g.n
    off = g.offsets.astype(np.int64)
    deg = np.diff(off)
    dist = np.full(n, INF, dtype=np.uint64)
    dist[src] = 0
    inq = np.zeros(n, dtype=bool)
    inq[src] = True
    steps = relaxed = 0
    while inq.any():
        qv = np.flatnonzero(inq)
        keys = dist[qv]
        theta = INF if qv.size <= rho else np.partition(keys, rho - 1)[rho - 1]
        sel = keys <= theta
        if D is not None and qv.size > rho:
            k = max(1, rho // div)
            theta_h = np.partition(keys, k - 1)[k - 1]
            assert theta_h >= keys.min()
            sel &= (deg[qv] < D) | (keys <= theta_h)
        ext = qv[sel]
        assert ext.size > 0  # progress: the smallest key is always extracted
        inq[ext] = False
        for u in ext:  # WriteMin with the current key (any order is valid)
            du = dist[u]
            for e in range(off[u], off[u + 1]):
                v = g.targets[e]
                nd = du + np.uint64(g.weights[e])
                relaxed += 1
                if nd < dist[v]:
                    dist[v] = nd
                    inq[v] = True
        steps += 1
    return dist, steps, relaxed


def test_deferral_keeps_distances_on_tiny_graphs():
    rng = np.random.default_rng(77)
    for i in range(60):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(0, 6 * n + 1))
        w = rng.integers(0, 50, m)
        w[rng.random(m) < 0.2] = 0
        g = graphgen.from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m), w)
        s = int(rng.integers(0, n))
        exp = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
        for rho, D, div in ((1, 1, 1), (2, 1, 4), (5, 2, 3), (3, 3, 1000), (8, 1, 2)):
            got, _, _ = model_rho_stepping(g, s, rho, D, div)
            assert np.array_equal(got, exp), (i, rho, D, div)


def test_deferral_relaxes_fewer_arcs_on_a_power_law_graph():
    g = graphgen.rmat(11, 16, seed=5)
    s = int(np.argmax(np.diff(g.offsets)))
    exp = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
    base, steps0, rel0 = model_rho_stepping(g, s, 256)
    dfr, steps1, rel1 = model_rho_stepping(g, s, 256, D=32, div=30)
    assert np.array_equal(base, exp) and np.array_equal(dfr, exp)
    assert rel1 < rel0, (rel1, rel0)
