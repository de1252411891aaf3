"""The allocation-free solve (sssp_solve_noalloc) against sssp_solve, through
the C ABI: same distances, bit for bit, on two calls in a row (the second on
a smaller input), with the oracle's rows beside them; the graph's own
workspace is left alone; a launch whose workspace exceeds the static array is
refused before any device work."""

import ctypes

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp(torch_cuda):
    import paper_2105_06145_amd as sp
    return sp


def _solve_abi(sp, entry, G, sources, params, torch):
    N = sp._native
    src = np.ascontiguousarray(sources, dtype=np.int32)
    out = torch.full((len(src), G.n), -7, dtype=torch.int64, device="cuda")
    st = N.sssp_stats()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = entry(G._h, ctypes.c_void_p(src.ctypes.data), len(src), params, ctypes.c_void_p(out.data_ptr()), stream, st)
    assert rc == N.SSSP_OK, (entry.__name__, rc, N.sssp_last_error())
    return sp.to_numpy_u64(out), st


def _params(sp, rule, **kw):
    p = sp._native.sssp_default_params()
    p.rule = rule
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_noalloc_matches_solve_two_calls_second_smaller(sp, torch_cuda):
    torch = torch_cuda
    N = sp._native
    big = graphgen.rmat(14, 16, whi=1 << 18, seed=71)
    small = graphgen.grid2d(40, 30, 1, 1 << 16, seed=72)
    # Hub deferral on the power-law graph (its benchmark configuration), then
    # the plain rho rule on it, then the small grid: local expansion, which
    # the allocation-free call runs without the graph's target rows.
    defer = N.sssp_tuning()
    defer.hub_defer_degree, defer.hub_defer_div = 64, 300
    cases = [
        (big, [5, 900], _params(sp, N.SSSP_RULE_RHO, rho=4096, seed=3, tuning=ctypes.pointer(defer))),
        (big, [5, 900, 16000], _params(sp, N.SSSP_RULE_RHO, rho=512, seed=3)),
        (small, [17], _params(sp, N.SSSP_RULE_DELTA_STAR, delta=5000)),
    ]
    for g, sources, p in cases:
        print(f"noalloc case n={g.n} m={g.m} sources={sources} rule={p.rule}", flush=True)
        G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
        try:
            before = G.device_bytes()
            got, st_na = _solve_abi(sp, N.sssp_solve_noalloc, G, sources, p, torch)
            # The graph's workspace is neither allocated nor used by this call.
            assert G.device_bytes() == before
            exp, st = _solve_abi(sp, N.sssp_solve, G, sources, p, torch)
            assert np.array_equal(got, exp), f"noalloc differs from sssp_solve on n={g.n}"
            for i, s in enumerate(sources):
                assert np.array_equal(got[i], oracle.dijkstra(g.offsets, g.targets, g.weights, s)), (g.n, s)
            assert st_na.steps > 0 and st_na.teams == st.teams
        finally:
            G.close()


def test_noalloc_refuses_workspace_beyond_the_array(sp, torch_cuda):
    torch = torch_cuda
    N = sp._native
    # 4M vertices and no arcs: about 20 bytes per vertex of workspace for one
    # team already exceed the 64 MiB array.
    n = 4 << 20
    off = np.zeros(n + 1, dtype=np.int64)
    tgt = np.zeros(0, dtype=np.int32)
    w = np.zeros(0, dtype=np.uint32)
    G = sp.Graph.from_csr(off, tgt, w)
    try:
        src = np.array([0], dtype=np.int32)
        out = torch.full((1, n), -7, dtype=torch.int64, device="cuda")
        p = _params(sp, N.SSSP_RULE_BF)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = N.sssp_solve_noalloc(G._h, ctypes.c_void_p(src.ctypes.data), 1, p, ctypes.c_void_p(out.data_ptr()),
                                  stream, None)
        assert rc == N.SSSP_ERR_INVALID_ARGUMENT
        assert "scratch array holds" in N.sssp_last_error()
        torch.cuda.synchronize()
        assert int((out == -7).sum()) == n  # nothing was written
    finally:
        G.close()
