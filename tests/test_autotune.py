"""Parameter search (host logic on a synthetic cost model) and, on the GPU,
tuned solves against the oracle."""

import math

import numpy as np
import pytest

from paper_2105_06145_amd import autotune as at


def cost_model(cfg):
    """A made-up cost with its minimum at rho = 2^14 (or Delta = 4096),
    teams = 32, hub_degree = 4096, chunk_edges = 16384, list_divisor = 64."""
    t = cfg.get("tuning", {})
    if cfg["rule"] == "rho":
        c = 10 + (math.log2(cfg["rho"]) - 14) ** 2
    else:
        c = 12 + (math.log2(cfg["delta"]) - 12) ** 2
    teams = t.get("teams", 0) or 64  # 0: the library's choice for 40 sources
    c += 0 if teams == 32 else 1 + abs(math.log2(teams) - 5)
    c -= 0.5 if t.get("hub_degree") == 4096 else 0
    c -= 0.125 if t.get("chunk_edges") == 16384 else 0
    c += 0 if t.get("list_divisor", 64) == 64 else 0.25
    return c


def test_candidates():
    assert at.rho_candidates(1 << 20) == [1 << k for k in range(20, 7, -2)]
    assert at.rho_candidates((1 << 21) + 5) == [1 << k for k in range(22, 7, -2)]
    assert at.rho_candidates(5) == [256]
    assert at.delta_candidates(1000) == [1024000, 256000, 64000, 16000, 4000, 1000, 250]
    assert at.team_candidates(64) == [8, 16, 32, 64]
    assert at.team_candidates(3) == [8]
    assert [at.batch_class(x) for x in (1, 2, 8, 9, 64, 65)] == [1, 8, 8, 16, 64, 128]


def test_search_finds_the_minimum_of_the_model():
    tu = at.Tuner(measure=cost_model, budget_s=60)
    cfg = tu.search(n=1 << 20, nsrc=40, w_median=1000)
    assert cfg["rule"] == "rho" and cfg["rho"] == 1 << 14
    assert cfg["tuning"]["teams"] == 32 and cfg["tuning"]["hub_degree"] == 4096
    assert cfg["tuning"]["chunk_edges"] == 16384
    assert cfg.get("tuning", {}).get("list_divisor", 64) == 64
    assert cfg["ms"] == pytest.approx(9.375)
    assert cfg["evaluations"] == len(tu.history)


def test_sweep_stops_after_two_slower_values():
    calls = []

    def model(cfg):
        calls.append(cfg.get("rho"))
        return abs(math.log2(cfg["rho"]) - 18) if "rho" in cfg else 1.0

    at.Tuner(measure=model).search(n=1 << 24, nsrc=1, w_median=1, rules=("rho",))
    sweep = [c for c in calls if c is not None]
    # 2^24, 2^22, 2^20, 2^18 (best), 2^16, 2^14 (second slower: stop), then 2^17 and 2^19.
    assert sweep[:6] == [1 << 24, 1 << 22, 1 << 20, 1 << 18, 1 << 16, 1 << 14]
    assert set(sweep[6:8]) == {1 << 17, 1 << 19}


def test_sweep_crosses_a_flat_stretch():
    # Every rho above 2^16 behaves alike (noise within 2%); the optimum is at 2^10.
    def model(cfg):
        if "rho" not in cfg:
            return 1.0
        lg = math.log2(cfg["rho"])
        noise = 0.02 * ((int(lg) * 7919) % 3 - 1)
        return 100.0 * (1 + noise) if lg > 16 else 10 + (lg - 10) ** 2

    cfg = at.Tuner(measure=model).search(n=1 << 24, nsrc=1, w_median=1, rules=("rho",))
    assert cfg["rho"] == 1 << 10


def test_search_single_source_has_no_teams_and_obeys_budget():
    tu = at.Tuner(measure=cost_model, budget_s=60)
    cfg = tu.search(n=1 << 16, nsrc=1, w_median=1 << 12, rules=("delta",))
    assert cfg["rule"] == "delta" and cfg["delta"] == 1 << 12
    assert all("teams" not in c.get("tuning", {}) for c, _ in tu.history)
    tu0 = at.Tuner(measure=cost_model, budget_s=0)
    cfg0 = tu0.search(n=1 << 16, nsrc=1, w_median=100)
    assert len(tu0.history) == 1 and cfg0["ms"] == tu0.history[0][1]


def local_model(cfg):
    """Delta*-stepping on a graph that relaxes locally: Delta = 2^lg needs a
    local budget of 4096 * 2^(lg - 12); below it the steps multiply (cost
    100). With enough budget, larger Delta is cheaper (fewer steps)."""
    if cfg["rule"] != "delta":
        return 1000.0
    lg = math.log2(cfg["delta"])
    lb = cfg.get("tuning", {}).get("local_budget", at.DEFAULT_LOCAL_BUDGET)
    need = at.DEFAULT_LOCAL_BUDGET * 2 ** max(0.0, lg - 12)
    if lg < 12:
        return 12 + (12 - lg) ** 2
    if lb < need:
        return 100.0
    return 12 - 0.3 * (lg - 12) + 0.1 * math.log2(lb / need)


def test_local_budget_searched_with_delta():
    assert at.local_candidates(1 << 12) == [(1 << 12, 8192), (1 << 13, 8192), (1 << 13, 16384),
                                            (1 << 14, 16384), (1 << 14, 32768)]
    assert at.relaxes_locally(1000, 3600) and not at.relaxes_locally(1000, 10000)
    tu = at.Tuner(measure=local_model)
    cfg = tu.search(n=1 << 20, nsrc=1, w_median=1 << 12, rules=("delta",), local=True)
    # The default budget finds Delta = 2^12; the joint step finds 2^14 with 4x the budget.
    assert cfg["delta"] == 1 << 14 and cfg["tuning"]["local_budget"] == 16384
    assert cfg["ms"] == pytest.approx(11.4)
    # Without local expansion the budget is never tried.
    tu2 = at.Tuner(measure=local_model)
    cfg2 = tu2.search(n=1 << 20, nsrc=1, w_median=1 << 12, rules=("delta",))
    assert cfg2["delta"] == 1 << 12
    assert all("local_budget" not in c.get("tuning", {}) for c, _ in tu2.history)


def defer_model(cfg):
    """rho-stepping on a power-law graph: without deferral the best rho is
    2^14; deferring hubs of degree >= 64 with divisor 300 makes rho = 2^16
    best."""
    if cfg["rule"] != "rho":
        return 1000.0
    lg = math.log2(cfg["rho"])
    t = cfg.get("tuning", {})
    if t.get("hub_defer_degree") == 64 and t.get("hub_defer_div") == 300:
        return 8 + (lg - 16) ** 2
    if t.get("hub_defer_degree"):
        return 9.5 + (lg - 15) ** 2
    return 10 + (lg - 14) ** 2


def test_hub_deferral_searched_with_rho():
    assert at.defer_candidates(1 << 10)[:3] == [(1 << 10, 32, 1000), (1 << 10, 64, 300), (1 << 10, 128, 100)]
    assert len(at.defer_candidates(1 << 10)) == 12 and at.defer_candidates(8)[-1] == (64, 128, 100)
    assert at.has_hubs([0, 1, 2, 3, 4, 5]) and not at.has_hubs([9, 9, 9, 9, 9]) and not at.has_hubs(None)
    tu = at.Tuner(measure=defer_model)
    cfg = tu.search(n=1 << 20, nsrc=1, w_median=1, rules=("rho",), hubs=True)
    assert cfg["rho"] == 1 << 16 and cfg["tuning"]["hub_defer_degree"] == 64
    assert cfg["tuning"]["hub_defer_div"] == 300 and cfg["ms"] == pytest.approx(8.0)
    tu2 = at.Tuner(measure=defer_model)
    cfg2 = tu2.search(n=1 << 20, nsrc=1, w_median=1, rules=("rho",))
    assert cfg2["rho"] == 1 << 14
    assert all("hub_defer_degree" not in c.get("tuning", {}) for c, _ in tu2.history)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    tu = at.Tuner(cache_path=path, measure=cost_model)

    class FakeGraph:
        n = 1 << 12
        fingerprint = "abc"
        summary = {"weight_q10_50_90": [1, 4096, 9]}

    cfg = tu.tune(FakeGraph(), list(range(10)))
    again = at.Tuner(cache_path=path, measure=lambda c: pytest.fail("cache miss"))
    assert again.tune(FakeGraph(), list(range(12))) == cfg  # same batch class (16)
    assert again.lookup("abc", 1) is None


@pytest.mark.gpu
def test_tuned_solves_match_oracle(torch_cuda, tmp_path):
    import graphgen
    import oracle
    import paper_2105_06145_amd as sp
    g = graphgen.rmat(12, 16, seed=31)
    G = sp.Graph.from_csr(g.offsets, g.targets, g.weights)
    tu = at.Tuner(cache_path=str(tmp_path / "t.json"), budget_s=20)
    srcs = [int(np.argmax(g.degrees())), 5, 77, 1000, 4000, 123, 9, 2048, 17]
    for batch in (srcs[:1], srcs):
        dist, st = at.solve_tuned(G, batch, tu)
        got = sp.to_numpy_u64(dist)
        for i, s in enumerate(batch):
            exp = oracle.dijkstra(g.offsets, g.targets, g.weights, s)
            assert np.array_equal(got[i], exp), (len(batch), i)
    assert tu.lookup(G.fingerprint, 1) is not None and tu.lookup(G.fingerprint, len(srcs)) is not None
    G.close()
