"""Stream-ordered solves (sssp_solve_async / query / wait / cancel) through
the C ABI: the same distances as the synchronous call (bit-exact against the
oracle), visible to work queued after the launch on the same stream, one
pending solve per graph, and cancellation that ends a long solve at a step
boundary with upper bounds in the rows under way."""

import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

SENTINEL = np.uint64(0xFFFFFFFFFFFFFFFE)


@pytest.fixture(scope="module")
def sp(torch_cuda):
    import paper_2105_06145_amd as sp
    return sp


def path_graph(n):
    """0 - 1 - ... - (n-1), unit weights both ways: the theta = min rule takes
    one step per vertex (n steps)."""
    u = np.arange(n - 1)
    return graphgen.from_arcs(n, np.concatenate([u, u + 1]), np.concatenate([u + 1, u]), np.ones(2 * (n - 1)))


def test_async_matches_oracle_and_is_stream_ordered(sp, torch_cuda):
    torch = torch_cuda
    g = graphgen.rmat(14, 16, seed=50)
    srcs = [int(np.argmax(g.degrees())), 3, 77, 1000]
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for tun in ({}, {"teams": 8}):
            p = sp.solve_async(G, srcs, rule="rho", rho=2048, tuning=tun)
            copy = p.out.clone()  # queued after the launch on the same stream
            out, st = p.wait()
            side.synchronize()
            for i, s in enumerate(srcs):
                exp = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
                assert np.array_equal(sp.to_numpy_u64(out)[i], exp), (tun, i)
                assert np.array_equal(sp.to_numpy_u64(copy)[i], exp), ("stream-ordered copy", tun, i)
            assert st["steps"] > 0 and st["extracted"] >= len(srcs) and st["device_ms"] > 0
            _, st2 = sp.solve(G, srcs, rule="rho", rho=2048, tuning=tun)
            assert st2["teams"] == st["teams"]
    G.close()


def test_query_and_one_pending_solve_per_graph(sp, torch_cuda):
    torch = torch_cuda
    g = graphgen.road(80, 80, seed=51)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        p = sp.solve_async(G, [5], rule="delta", delta=3000)
        for call in (lambda: sp.solve(G, [0]), lambda: sp.solve_async(G, [0]),
                     lambda: sp.Server(G, torch.empty((1, g.n), dtype=torch.int64, device="cuda"))):
            with pytest.raises(sp.SSSPError) as ei:
                call()
            assert ei.value.status == 1 and "pending" in str(ei.value)
        rc = sp.sssp_graph_destroy(G._h)
        assert rc == 1  # refused while pending
        t_end = time.monotonic() + 30
        while not p.done():
            assert time.monotonic() < t_end
            time.sleep(0.001)
        out, _ = p.wait()
        assert np.array_equal(sp.to_numpy_u64(out)[0], oracle.dijkstra(g.offsets, g.targets, g.weights, 5))
        # nothing pending any more
        for fn in (sp.sssp_solve_wait, ):
            assert fn(G._h, None) == 1
        assert sp.sssp_solve_cancel(G._h) == 1
        assert sp.sssp_solve_query(G._h)[0] == 1
        # enqueue-time errors leave nothing pending
        with pytest.raises(sp.SSSPError):
            sp.solve_async(G, [g.n])
        with pytest.raises(sp.SSSPError):
            sp.solve_async(G, [0], rule="rho", rho=0)
        d, _ = sp.solve(G, [5], rule="bf")
        assert np.array_equal(sp.to_numpy_u64(d)[0], oracle.dijkstra(g.offsets, g.targets, g.weights, 5))
        # run-time errors come from wait
        p = sp.solve_async(G, [5], rule="delta", delta=3000, max_steps=2)
        with pytest.raises(sp.SSSPError) as ei:
            p.wait()
        assert ei.value.status == 6
    G.close()


def test_cancel_ends_a_long_solve(sp, torch_cuda):
    torch = torch_cuda
    n = 200_000
    g = path_graph(n)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    exact = np.arange(n, dtype=np.uint64)  # distance from vertex 0
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        # One source, whole grid: about n steps of a few microseconds each.
        out = torch.empty((1, n), dtype=torch.int64, device="cuda")
        t0 = time.monotonic()
        p = sp.solve_async(G, [0], rule="min", out=out)
        time.sleep(0.05)
        p.cancel()
        with pytest.raises(sp.SSSPError) as ei:
            p.wait()
        elapsed = time.monotonic() - t0
        assert ei.value.status == sp.N.SSSP_ERR_CANCELLED
        row = sp.to_numpy_u64(out)[0]
        assert np.all(row >= exact)  # upper bounds (unreached: UINT64_MAX)
        assert row[0] == 0 and np.any(row == np.uint64(2**64 - 1))  # stopped part-way
        print(f"cancelled after {elapsed * 1e3:.0f} ms", flush=True)
        # Teams: sources not yet started leave their rows unwritten.
        srcs = list(range(0, 64 * 100, 100))
        out = torch.full((len(srcs), n), -2, dtype=torch.int64, device="cuda")
        p = sp.solve_async(G, srcs, rule="min", tuning={"teams": 8}, out=out)
        time.sleep(0.05)
        p.cancel()
        with pytest.raises(sp.SSSPError) as ei:
            p.wait()
        assert ei.value.status == sp.N.SSSP_ERR_CANCELLED
        rows = sp.to_numpy_u64(out)
        started = 0
        for i, s in enumerate(srcs):
            if np.all(rows[i] == SENTINEL):
                continue
            started += 1
            assert np.all(rows[i] >= np.abs(np.arange(n, dtype=np.int64) - s).astype(np.uint64)), i
        assert 1 <= started < len(srcs)
        # the graph is usable again
        d, _ = sp.solve(G, [n - 1], rule="delta", delta=1 << 12)
        assert np.array_equal(sp.to_numpy_u64(d)[0], exact[::-1])
    G.close()
