"""Autotuner host logic (CPU) and its use on the GPU."""
import json

import pytest

from paper_2105_01533_amd import autotune as A


def test_bucket_keys():
    assert A.bucket_key(24, 1 << 16) == "narrow_lg16"
    assert A.bucket_key(100, (1 << 20) + 1) == "wide_lg21"
    assert A.bucket_key(64, 2) == "narrow_lg1"


def test_greedy_search_finds_separable_optimum():
    target = {"fuse_max": 256, "bs_min_gates": 64, "mono_mode": 1, "block": 128, "load_factor": 0.7}
    cost = lambda k: sum(abs(A.SPACE[n].index(k[n]) - A.SPACE[n].index(target[n])) for n in A.SPACE) + 1.0
    best, t, trials = A.greedy_search(cost)
    assert {k: best[k] for k in A.SPACE} == target and t == 1.0
    assert len(trials) == 1 + sum(len(v) - 1 for v in A.SPACE.values())


def test_lookup_nearest_bucket_and_defaults(tmp_path):
    table = {"narrow_lg12": {"knobs": {**A.DEFAULTS, "fuse_max": 16}, "log2_capacity": 12},
             "narrow_lg20": {"knobs": {**A.DEFAULTS, "fuse_max": 4096}, "log2_capacity": 20}}
    assert A.lookup(table, 24, 1 << 13)["fuse_max"] == 16
    assert A.lookup(table, 24, 1 << 19)["fuse_max"] == 4096
    assert A.lookup(table, 100, 1 << 19) == A.DEFAULTS
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    assert A.load(str(p)) == table
    assert A.load(str(tmp_path / "missing.json")) == {}


@pytest.mark.gpu
def test_tuned_knobs_keep_results(tmp_path):
    """A small tuning run writes a table, and the chosen knobs give the same
    labels and amplitudes within 1e-12 as the defaults."""
    from helpers import assert_same_state
    from paper_2105_01533_amd import sim as S, workloads as W
    table = A.tune(buckets=((24, 10), (100, 12)), gates=600, repeats=1, cache=str(tmp_path / "t.json"), server=False)
    assert set(table) == {"narrow_lg10", "wide_lg12"}
    for nq, lg in ((24, 10), (100, 12)):
        w = A.representative(W, nq, lg, 800, seed=5)
        ref, o1, _ = S.run_workload(w, tuned=False)
        knobs = A.lookup(table, nq, w.capacity)
        tuned, o2, _ = S.run_workload(w, tuned=False, **knobs)
        assert list(o1) == list(o2)
        assert_same_state(ref.export(), tuned.export(), what=str(knobs))
        ref.close()
        tuned.close()


def test_state_and_server_knobs_follow_table_and_overrides(monkeypatch):
    """Unset knobs come from the committed table (nearest bucket), given ones
    win, and SPARSESIM_TUNING=off gives the defaults."""
    t = A.table()
    k = A.state_knobs(100, 1 << 20, {})
    assert set(k) == set(A.DEFAULTS)
    if any(key.startswith("wide") for key in t):
        assert k == A.lookup(t, 100, 1 << 20)
    assert A.state_knobs(100, 1 << 20, {"fuse_max": 7})["fuse_max"] == 7
    sk = A.server_knobs({"grid": 512})
    assert sk["grid"] == 512 and set(sk) == set(A.SERVER_DEFAULTS)
    if "server" in t:
        assert sk["tick_updates"] == t["server"]["knobs"]["tick_updates"]
        assert sk["lane_capacity"] == 0   # the lane is never switched on by the table
    monkeypatch.setenv("SPARSESIM_TUNING", "off")
    assert A.state_knobs(100, 1 << 20, {}) == A.DEFAULTS
    assert A.server_knobs() == A.SERVER_DEFAULTS


def test_greedy_search_ignores_noise():
    """A value within min_gain of the held one does not replace it."""
    space = {"fuse_max": [4096, 65536]}
    t = {4096: 0.990, 65536: 1.0}
    best, bt, _ = A.greedy_search(lambda k: t[k["fuse_max"]], space=space, start={"fuse_max": 65536}, min_gain=0.02)
    assert best["fuse_max"] == 65536 and bt == 1.0
    best, bt, _ = A.greedy_search(lambda k: t[k["fuse_max"]], space=space, start={"fuse_max": 65536}, min_gain=0.0)
    assert best["fuse_max"] == 4096
