"""Serving with admission by a device-memory budget (sssp_server_start_budget),
elastic groups of teams, the idle limit while a team is busy, and the
two-graph serving workload (R-MAT scale 22 and a 2000 x 2000 road grid
resident) checked element by element: against the oracle on sampled queries,
and every served row against the same query solved alone."""

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


@pytest.fixture
def side_stream(torch_cuda):
    """Run the test on a non-blocking stream: while a server runs, work on the
    legacy NULL stream would wait for the server's (blocking) stream."""
    s = torch_cuda.cuda.Stream()
    with torch_cuda.cuda.stream(s):
        yield s
    s.synchronize()


def test_budget_admission_blocks_and_resumes(sp, torch_cuda, side_stream):
    torch = torch_cuda
    g = graphgen.rmat(13, 16, seed=51)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    kw = dict(rule="rho", rho=1024)
    # Learn the launch's workspace size, then give it room for 2.5 rows.
    S = sp.BudgetServer(G, 1 << 30, **kw)
    c = S.counts()
    ws, row_bytes = c["workspace_bytes"], c["row_bytes"]
    assert row_bytes == 8 * g.n and c["rows"] >= 2 and c["budget_bytes"] == 1 << 30
    S.stop()
    S.close()
    with pytest.raises(sp.SSSPError) as ei:
        sp.BudgetServer(G, ws + row_bytes - 1, **kw)  # no room for a single row
    assert ei.value.status == 3
    S = sp.BudgetServer(G, ws + 2 * row_bytes + row_bytes // 2, **kw)
    assert S.counts()["rows"] == 2
    srcs = [3, 77, 1000, 5000, 8000, 123, 4095]
    tickets = [S.enqueue(s) for s in srcs]
    assert tickets == list(range(len(srcs)))
    c = S.counts()
    assert c["admitted"] == 2 and c["waiting"] == 5 and c["free_rows"] == 0
    finished = []
    t_end = time.monotonic() + 30
    while len(finished) < 2:
        finished += [t for t, _ in S.poll()]
        assert time.monotonic() < t_end
    assert sorted(finished) == [0, 1]
    # Both rows are held by finished requests: nothing more is admitted.
    time.sleep(0.2)
    assert S.poll() == []
    c = S.counts()
    assert c["held"] == 2 and c["admitted"] == 0 and c["waiting"] == 5 and c["free_rows"] == 0
    exp = {s: oracle.dijkstra(g.offsets, g.targets, g.weights, s) for s in srcs}
    got = {}
    # Taking a row releases it: the next waiting request is admitted.
    got[0] = sp.to_numpy_u64(S.take(0))
    c = S.counts()
    assert c["held"] == 1 and c["admitted"] == 1 and c["waiting"] == 4
    held = [1]
    while len(got) < len(srcs):
        for t in held:
            got[t] = sp.to_numpy_u64(S.take(t))
        held = [t for t, _ in S.poll()]
        assert time.monotonic() < t_end
    for t, s in enumerate(srcs):
        assert np.array_equal(got[t], exp[s]), f"ticket {t} source {s}"
    c = S.counts()
    assert c["held"] == 0 and c["admitted"] == 0 and c["waiting"] == 0 and c["free_rows"] == 2
    with pytest.raises(sp.SSSPError):
        S.take(0)  # already released
    st = S.stop()
    assert st["steps"] > 0
    S.close()
    G.close()


def test_idle_limit_while_a_team_is_busy(sp, torch_cuda, side_stream):
    """One team solves a long request while the others pass the idle limit:
    the launch then takes no more requests, the busy team's request still
    finishes, and polling afterwards reports nothing lost."""
    torch = torch_cuda
    n = 300_000
    src = np.concatenate([np.arange(n - 1), np.arange(1, n)])
    dst = np.concatenate([np.arange(1, n), np.arange(n - 1)])
    w = np.full(src.size, 3, dtype=np.uint32)
    g = graphgen.from_arcs(n, src, dst, w)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights, reorder=False)
    rows = torch.empty((2, n), dtype=torch.int64, device="cuda")
    # One team per request (no groups), so the other teams stay idle; no
    # local expansion, so the request takes one step per vertex.
    S = sp.Server(G, rows, rule="rho", rho=1, tuning={"group_max": 1, "local_budget": 0xFFFFFFFF}, idle_ms=300)
    t0 = S.submit(0, 0)
    time.sleep(1.0)
    with pytest.raises(sp.SSSPError) as ei:
        S.submit(5, 1)
    assert ei.value.status == 5
    done = []
    t_end = time.monotonic() + 60
    while not done:
        done = S.poll()
        assert time.monotonic() < t_end
    assert done[0][0] == t0
    exp = np.arange(n, dtype=np.uint64) * np.uint64(3)
    assert np.array_equal(sp.to_numpy_u64(rows[0]), exp)
    assert S.poll() == []  # nothing outstanding: no error
    S.stop()
    S.close()
    G.close()


def test_elastic_groups_match_the_oracle(sp, torch_cuda, side_stream):
    """Requests posted one at a time (each gets a large group) and in bursts
    (groups shrink to one team each), for several group limits."""
    torch = torch_cuda
    g = graphgen.road(60, 60, seed=52)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    rng = np.random.default_rng(53)
    sources = rng.integers(0, g.n, 40)
    exp = {int(s): oracle.dijkstra(g.offsets, g.targets, g.weights, int(s)) for s in set(sources.tolist())}
    for gm in (0, 2, 8):
        S = sp.BudgetServer(G, 1 << 28, rule="delta", delta=3000, tuning={"group_max": gm, "teams": 16})
        t_end = time.monotonic() + 60
        # One at a time.
        for s in sources[:8]:
            t = S.enqueue(int(s))
            while True:
                fin = S.poll()
                if fin:
                    assert fin[0][0] == t
                    assert np.array_equal(sp.to_numpy_u64(S.take(t)), exp[int(s)]), (gm, int(s))
                    break
                assert time.monotonic() < t_end
        # A burst.
        tick = {S.enqueue(int(s)): int(s) for s in sources[8:]}
        while tick:
            for t, _ in S.poll():
                assert np.array_equal(sp.to_numpy_u64(S.take(t)), exp[tick.pop(t)]), (gm, t)
            assert time.monotonic() < t_end
        S.stop()
        S.close()
    G.close()


def test_serving_rmat22_and_road2000_resident(sp, torch_cuda, side_stream):
    """The serving workload's two graphs resident at once, one budget server
    each; a mixed stream of requests (70% R-MAT). Every served row equals the
    same query solved alone, element by element, and sampled rows equal the
    oracle's."""
    torch = torch_cuda
    gr = graphgen.rmat(22, 16, seed=5001)
    gg = graphgen.road(2000, 2000, seed=5002)
    print(f"graphs: rmat22 n={gr.n} m={gr.m}, road2000 n={gg.n} m={gg.m}", flush=True)
    GR = sp.Graph.from_csr(gr.offsets, gr.targets, gr.weights)
    GG = sp.Graph.from_csr(gg.offsets, gg.targets, gg.weights)
    rng = np.random.default_rng(54)
    lr = graphgen.largest_component(gr)
    lg = graphgen.largest_component(gg)
    nq = 40
    which = rng.random(nq) < 0.7
    srcs = [int(rng.choice(lr)) if r else int(rng.choice(lg)) for r in which]
    kr = dict(rule="rho", rho=1 << 15)
    kg = dict(rule="delta", delta=8448)
    # Alone: each query solved by itself (whole-grid solve), rows kept on the device.
    alone = {}
    for i, (r, s) in enumerate(zip(which, srcs)):
        d, _ = sp.solve(GR if r else GG, [s], **(kr if r else kg))
        alone[i] = d[0]
    print("alone solves done", flush=True)
    SR = sp.BudgetServer(GR, 6 << 30, tuning={"blocks_per_cu": 3}, hash_rows=True, **kr)
    SG = sp.BudgetServer(GG, 2 << 30, tuning={"blocks_per_cu": 1}, hash_rows=True, **kg)
    tick = {}
    for i, (r, s) in enumerate(zip(which, srcs)):
        S = SR if r else SG
        tick[(S is SR, S.enqueue(s))] = i
    served = {}
    t_end = time.monotonic() + 120
    while len(served) < nq:
        for S in (SR, SG):
            for t, h in S.poll():
                served[tick[(S is SR, t)]] = S.take(t)
        assert time.monotonic() < t_end, f"{len(served)} of {nq} served"
    SR.stop()
    SG.stop()
    print("served", flush=True)
    for i in range(nq):
        assert torch.equal(served[i], alone[i]), f"query {i} (source {srcs[i]}): served differs from alone"
    sample = [i for i in range(nq) if which[i]][:2] + [i for i in range(nq) if not which[i]][:2]
    for i in sample:
        g = gr if which[i] else gg
        exp = oracle.dijkstra(g.offsets, g.targets, g.weights, srcs[i])
        assert np.array_equal(sp.to_numpy_u64(served[i]), exp), f"query {i} vs oracle"
    SR.close()
    SG.close()
    GR.close()
    GG.close()
