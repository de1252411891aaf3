"""Host logic of the benchmark (CPU): the algorithmic byte count the
roofline prices, the configuration keys of the committed traffic counters,
and that counters taken on other kernel sources are not used."""

import json
import os
import sys

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, REPO)

import bench  # noqa: E402


def test_algorithmic_bytes_terms():
    st = {"dense_steps": 3, "queue_dense": 1000, "extracted": 500, "edges_relaxed": 7000,
          "writemin_success": 40, "list_appends": 30}
    n = 1 << 20
    # S0: 8 n + n / 8; dense steps: 3 n / 8 + 8 * 1000; extracted: (2 * 8 + 16) * 500;
    # arcs: 16 * 7000; successes: 12 * 40; list entries: 4 * 30.
    exp = (8 * n + n // 8) + (3 * (n // 8) + 8 * 1000) + 32 * 500 + 16 * 7000 + 12 * 40 + 4 * 30
    assert bench.algorithmic_bytes(n, st, 1) == exp
    # Two sources double the per-source S0 term only.
    assert bench.algorithmic_bytes(n, st, 2) == exp + 8 * n + n // 8
    # int32 offsets read 2 * 4 bytes per extracted vertex.
    assert bench.algorithmic_bytes(n, st, 1, offset_bytes=4) == exp - 8 * 500
    st2 = dict(st, queue_list=10)
    assert bench.implementation_bytes(n, st2, 1) == exp + 20 * n + 12 * 10 + 4 * 40


def test_traffic_keys():
    assert bench.traffic_key(524288, None) == "524288"
    assert bench.traffic_key(2097152, {"hub_defer_degree": 64, "hub_defer_div": 300}) == "2097152:defer64/300"
    assert bench.traffic_key(2097152, {"hub_defer_degree": 32, "hub_defer_div": 1000, "list_divisor": 256}) == \
        "2097152:defer32/1000:list256"
    assert bench.traffic_key(2097152, {"hub_defer_degree": 32, "hub_defer_div": 1000, "list_divisor": 64}) == \
        "2097152:defer32/1000"


def test_committed_traffic_matches_sources_and_is_refused_otherwise(tmp_path, monkeypatch):
    d = json.load(open(bench.TRAFFIC_FILE))
    current = d["kernel_sha"] == bench.kernel_sha()
    for key, rec in d["by_rho"].items():
        # Used only while the kernel sources are the ones the counters were
        # taken on (or sources whose device code is identical, as noted).
        got = bench.load_traffic("rmat24", key)
        assert got == (rec["traffic_bytes_per_launch"] if current else None)
        assert rec["traffic_bytes_per_launch"] > rec["algorithmic_bytes_per_launch"] > 0
    assert bench.load_traffic("rmat24", "1:defer1/1") is None
    assert bench.load_traffic("road5000", next(iter(d["by_rho"]))) is None
    # Counters of other sources are not used.
    stale = dict(d, kernel_sha="0" * 16)
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("rmat24", next(iter(d["by_rho"]))) is None
