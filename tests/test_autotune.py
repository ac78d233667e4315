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
    assert best == target and t == 1.0
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
    table = A.tune(buckets=((24, 10), (100, 12)), gates=600, repeats=1, cache=str(tmp_path / "t.json"))
    assert set(table) == {"narrow_lg10", "wide_lg12"}
    for nq, lg in ((24, 10), (100, 12)):
        w = A.representative(W, nq, lg, 800, seed=5)
        ref, o1, _ = S.run_workload(w)
        knobs = A.lookup(table, nq, w.capacity)
        tuned, o2, _ = S.run_workload(w, **knobs)
        assert list(o1) == list(o2)
        assert_same_state(ref.export(), tuned.export(), what=str(knobs))
        ref.close()
        tuned.close()
