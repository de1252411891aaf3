"""Serving launches (sssp_server_*): requests posted while the kernel runs,
checked against the oracle row by row, and the row checksum against an
independent numpy implementation of its definition (a sum of SplitMix64
finaliser mixes)."""

import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp(torch_cuda):
    import paper_2105_06145_amd as sp
    return sp


def np_row_hash(d: np.ndarray) -> int:
    v = np.arange(d.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = d.astype(np.uint64) ^ (v * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        return int(z.sum(dtype=np.uint64))


@pytest.fixture
def side_stream(torch_cuda):
    """Run the test on a non-blocking stream: while a server runs, work on the
    legacy NULL stream would wait for the server's (blocking) stream."""
    s = torch_cuda.cuda.Stream()
    with torch_cuda.cuda.stream(s):
        yield s
    s.synchronize()


def serve_all(sp, server, sources, check, deadline_s=30.0):
    """Post every source (one free row each, rows reused once done) and call
    check(index, row_tensor, checksum) as requests finish."""
    nrows = server.rows.shape[0]
    free = list(range(nrows))
    pending = {}
    nxt = done = 0
    t_end = time.monotonic() + deadline_s
    while done < len(sources):
        while free and nxt < len(sources):
            r = free.pop()
            t = server.submit(int(sources[nxt]), r)
            pending[t] = (nxt, r)
            nxt += 1
        for t, h in server.poll():
            i, r = pending.pop(t)
            check(i, server.rows[r], h)
            free.append(r)
            done += 1
        assert time.monotonic() < t_end, f"{done} of {len(sources)} requests finished before the deadline"
    return done


def test_row_hash_matches_definition(sp, torch_cuda):
    torch = torch_cuda
    rng = np.random.default_rng(5)
    for n in (1, 63, 1000, 123457):
        d = rng.integers(0, 2**63, n, dtype=np.uint64)
        d[rng.random(n) < 0.2] = np.uint64(2**64 - 1)
        t = torch.from_numpy(d.view(np.int64)).cuda()
        assert sp.row_hash(t) == np_row_hash(d), n


@pytest.mark.parametrize("case", ["rmat", "road", "rmat-tree", "rmat-fixed-teams", "rmat-defer", "rmat-group-min"])
def test_server_matches_oracle(sp, torch_cuda, side_stream, case):
    torch = torch_cuda
    if case.startswith("rmat"):
        g = graphgen.rmat(13, 16, seed=41)
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
        kw = dict(rule="rho", rho=2048)
        if case == "rmat-tree":
            kw["tuning"] = {"queue": 1}  # tournament-tree LaB-PQ (Sec. 4.2)
        if case == "rmat-fixed-teams":
            kw["tuning"] = {"group_max": 1}  # one team per request
        if case == "rmat-group-min":
            kw["tuning"] = {"group_min": 4, "group_max": 8}  # requests wait for four idle teams
        if case == "rmat-defer":
            kw["tuning"] = {"hub_defer_degree": 16, "hub_defer_div": 100}  # hub deferral, per-group rho
    else:
        g = graphgen.road(70, 70, seed=42)
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
        kw = dict(rule="delta", delta=4000)
    rng = np.random.default_rng(43)
    sources = rng.integers(0, g.n, 150)
    exp = {int(s): oracle.dijkstra(g.offsets, g.targets, g.weights, int(s)) for s in set(sources.tolist())}
    rows = torch.empty((12, g.n), dtype=torch.int64, device="cuda")
    server = sp.Server(G, rows, ring_capacity=16, hash_rows=True, **kw)
    seen = []

    def check(i, row, h):
        got = sp.to_numpy_u64(row)
        e = exp[int(sources[i])]
        assert np.array_equal(got, e), f"request {i} source {sources[i]}"
        assert h == np_row_hash(e), f"request {i}: checksum"
        seen.append(i)

    serve_all(sp, server, sources, check)
    st = server.stop()
    assert sorted(seen) == list(range(len(sources)))
    assert st["teams"] >= 8 and st["steps"] > 0 and st["extracted"] >= len(sources)
    server.close()
    G.close()


def test_two_servers_side_by_side_same_alone_and_in_the_mix(sp, torch_cuda, side_stream):
    """Two graphs served at once on separate streams; every served row's
    checksum equals the checksum of the same query solved alone."""
    torch = torch_cuda
    g1 = graphgen.rmat(14, 16, seed=44)
    g2 = graphgen.road(90, 90, seed=45)
    G1 = sp.Graph.from_csr(g1.offsets, g1.targets, g1.weights)
    G2 = sp.Graph.from_csr(g2.offsets, g2.targets, g2.weights, reorder=False)
    rng = np.random.default_rng(46)
    s1 = rng.integers(0, g1.n, 60)
    s2 = rng.integers(0, g2.n, 40)
    alone = {}
    for G, g, ss, kw in ((G1, g1, s1, dict(rule="rho", rho=4096)), (G2, g2, s2, dict(rule="delta", delta=5000))):
        for s in set(ss.tolist()):
            d, _ = sp.solve(G, [int(s)], **kw)
            alone[(g.n, int(s))] = sp.row_hash(d[0])
    # Both servers ordered after the same stream: each still runs on a queue of its own.
    st1 = st2 = torch.cuda.current_stream()
    rows1 = torch.empty((8, g1.n), dtype=torch.int64, device="cuda")
    rows2 = torch.empty((8, g2.n), dtype=torch.int64, device="cuda")
    tun = dict(blocks_per_cu=2)
    A = sp.Server(G1, rows1, rule="rho", rho=4096, tuning=tun, hash_rows=True, stream=st1)
    B = sp.Server(G2, rows2, rule="delta", delta=5000, tuning=tun, hash_rows=True, stream=st2)
    # Interleave: post to both before collecting from either.
    free = {A: list(range(8)), B: list(range(8))}
    src = {A: s1, B: s2}
    nxt = {A: 0, B: 0}
    pending = {A: {}, B: {}}
    done = 0
    t_end = time.monotonic() + 30
    while done < len(s1) + len(s2):
        for S in (A, B):
            while free[S] and nxt[S] < len(src[S]):
                r = free[S].pop()
                pending[S][S.submit(int(src[S][nxt[S]]), r)] = (nxt[S], r)
                nxt[S] += 1
            for t, h in S.poll():
                i, r = pending[S].pop(t)
                n = S.rows.shape[1]
                assert h == alone[(n, int(src[S][i]))], ("A" if S is A else "B", i)
                free[S].append(r)
                done += 1
        assert time.monotonic() < t_end
    t_stop = time.monotonic()
    A.stop()
    B.stop()
    assert time.monotonic() - t_stop < 5.0  # closing the ring ends the launches at once
    A.close()
    B.close()
    G1.close()
    G2.close()


def test_server_errors_and_idle_limit(sp, torch_cuda, side_stream):
    torch = torch_cuda
    g = graphgen.road(30, 30, seed=47)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    rows = torch.empty((2, g.n), dtype=torch.int64, device="cuda")
    S = sp.Server(G, rows, rule="bf", ring_capacity=2)
    with pytest.raises(sp.SSSPError):
        S.submit(g.n, 0)  # source out of range
    with pytest.raises(sp.SSSPError):
        S.submit(0, 2)  # row out of range
    with pytest.raises(sp.SSSPError):
        sp.solve(G, [0])  # the graph is serving
    with pytest.raises(sp.SSSPError):
        sp.Server(G, rows)  # one server per graph
    S.submit(0, 0)
    S.submit(1, 1)
    with pytest.raises(sp.SSSPError) as ei:
        S.submit(2, 0)  # row 0 is held until its request is polled done
    assert "busy" in str(ei.value)
    got = []
    t_end = time.monotonic() + 60
    while len(got) < 2:
        got += S.poll()
        assert time.monotonic() < t_end
    S.stop()
    S.stop()  # idempotent
    with pytest.raises(sp.SSSPError):
        S.submit(0, 0)
    S.close()
    d, _ = sp.solve(G, [0])  # usable again
    assert np.array_equal(sp.to_numpy_u64(d)[0], oracle.dijkstra(g.offsets, g.targets, g.weights, 0))
    # A server whose teams wait longer than idle_ms for work takes no more
    # requests and ends by itself.
    S = sp.Server(G, rows, rule="bf", idle_ms=100)
    time.sleep(1.0)
    with pytest.raises(sp.SSSPError) as ei:
        S.submit(0, 0)
    assert ei.value.status == 5
    S.stop()
    S.close()
    G.close()
