"""Seeded generators: determinism, shape and the published SplitMix64 values. CPU only."""

import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def digest(g):
    h = hashlib.sha256()
    for a in (g.offsets, g.targets, g.weights):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def check_symmetric_simple(g):
    off, tgt, w = g.offsets, g.targets, g.weights
    assert off[0] == 0 and off[-1] == g.m and np.all(np.diff(off) >= 0)
    assert np.all((tgt >= 0) & (tgt < g.n))
    src = np.repeat(np.arange(g.n), np.diff(off))
    assert not np.any(src == tgt), "self-loop"
    # rows sorted strictly => no duplicates
    same_row = src[1:] == src[:-1]
    assert np.all(tgt[1:][same_row] > tgt[:-1][same_row])
    # symmetric with equal weights
    fwd = np.lexsort((tgt, src))
    rev = np.lexsort((src, tgt))
    assert np.array_equal(src[fwd], tgt[rev]) and np.array_equal(tgt[fwd], src[rev])
    assert np.array_equal(w[fwd], w[rev])


def test_splitmix64_published_values():
    # First outputs of SplitMix64 seeded with 0 (Steele, Lea and Flood 2014;
    # the same sequence as java.util.SplittableRandom(0).nextLong()).
    assert [int(x) for x in graphgen.splitmix64(0, 3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_grid_shape_and_weights():
    g = graphgen.grid2d(256, 256, 1, 1 << 16, seed=1001)
    assert g.n == 65536 and g.m == 2 * 2 * 256 * 255 == 261120
    assert g.weights.min() >= 1 and g.weights.max() < (1 << 16)
    check_symmetric_simple(g)
    assert digest(g) == digest(graphgen.grid2d(256, 256, 1, 1 << 16, seed=1001))
    assert digest(g) != digest(graphgen.grid2d(256, 256, 1, 1 << 16, seed=1002))


def test_rmat_shape():
    g = graphgen.rmat(14, 16, seed=5)
    assert g.n == 1 << 14
    assert 0 < g.m <= 2 * 16 * (1 << 14)
    assert g.weights.min() >= 1 and g.weights.max() < (1 << 18)
    check_symmetric_simple(g)
    deg = g.degrees()
    assert deg.max() > 50 * deg.mean()  # power-law hubs
    assert digest(g) == digest(graphgen.rmat(14, 16, seed=5))
    # Without relabelling the hubs sit at low ids (quadrant a = 0.57 dominates).
    g0 = graphgen.rmat(14, 16, seed=5, relabel=False)
    assert np.argmax(g0.degrees()) < 64
    assert g0.m == g.m  # relabelling permutes, it does not change the multiset


def test_road_shape():
    W = 200
    g = graphgen.road(W, W, seed=9)
    n_grid = 2 * W * W - 2 * W
    expected = 2 * (0.9 * n_grid + 0.01 * n_grid)
    assert abs(g.m - expected) / expected < 0.02
    check_symmetric_simple(g)
    # Weights are rounded 1000 x lengths of jittered unit steps: in [200, ~4300].
    assert g.weights.min() >= 1 and g.weights.max() <= int(1000 * np.hypot(3.8, 3.8)) + 1
    lcc = graphgen.largest_component(g)
    assert lcc.sum() > 0.95 * g.n


def test_knn_shape():
    g = graphgen.knn(30, 200, 0.01, 10, 1e6, seed=4)
    assert g.n == 6000
    deg = g.degrees()
    assert deg.min() >= 10  # every point keeps its own 10 neighbours
    check_symmetric_simple(g)
    lab, k = graphgen.components(g)
    assert k >= 1 and lab.max() == k - 1


def test_largest_component_and_sources():
    g = graphgen.from_arcs(7, [0, 1, 1, 2, 4, 5], [1, 0, 2, 1, 5, 4], [1] * 6)
    lcc = graphgen.largest_component(g)
    assert list(np.flatnonzero(lcc)) == [0, 1, 2]
    src = graphgen.pick_sources(g.n, 50, 3, lcc)
    assert set(src.tolist()) <= {0, 1, 2}
    assert np.array_equal(src, graphgen.pick_sources(g.n, 50, 3, lcc))


def test_thread_count_independence():
    code = ("import sys; sys.path.insert(0, %r); import graphgen, hashlib;"
            "g = graphgen.rmat(13, 8, seed=77); r = graphgen.road(90, 70, seed=78);"
            "print(hashlib.sha256(g.targets.tobytes() + g.weights.tobytes() + r.targets.tobytes()"
            " + r.weights.tobytes()).hexdigest())") % REPO
    outs = []
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert outs[0] == outs[1]


@pytest.mark.parametrize("name", ["grid256", "rmat12", "road100", "knn20"])
def test_workload_recipes(name):
    w = graphgen.workload(name, sources=3)
    assert w.sources.shape == (3,)
    assert np.all((w.sources >= 0) & (w.sources < w.graph.n))
