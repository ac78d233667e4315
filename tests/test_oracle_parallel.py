"""The oracle's multithreaded queue (Sec. 5: queues of more than 64 gates on
more than 4096 entries are applied by several threads) must give bitwise the
serial oracle's state, outcomes and counters."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2105_01533_amd import workloads as W


def run(w, threads, state=None):
    o = Oracle(w.n_qubits, w.eps)
    o.set_threads(threads)
    if state is None:
        o.set_basis(*w.basis)
    else:
        o.import_state(*state)
    out, _ = o.run(w.ops)
    return o, out


def assert_bitwise(a, b):
    for x, y in zip(a.export(), b.export()):
        assert x.tobytes() == y.tobytes()


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_c2_family_bitwise(threads):
    w = W.config2(8, n=100, h_qubits=14, gates=6000, round_gates=1500, meas_per_round=3)
    a, oa = run(w, 1)
    b, ob = run(w, threads)
    assert b.totals()["parallel_runs"] > 0 and a.totals()["parallel_runs"] == 0
    assert oa.tolist() == ob.tolist()
    assert_bitwise(a, b)
    ta, tb = a.totals(), b.totals()
    for k in ("updates", "u2_applied", "u2_skipped", "measures", "peak_nnz", "pruned"):
        assert ta[k] == tb[k], k


def test_imported_wide_state_long_runs():
    n = 128
    lo, hi, amp = W.random_state(5, 20000, n)
    w = W.random_circuit(6, n=n, gates=600, h_frac=0.01, ctrl_max=3, measure_frac=0.002)
    a, oa = run(w, 1, (lo, hi, amp))
    b, ob = run(w, 5, (lo, hi, amp))
    assert b.totals()["parallel_runs"] > 0
    assert oa.tolist() == ob.tolist()
    assert_bitwise(a, b)


def test_short_queues_stay_serial():
    """A 64-gate queue, or a state of 4096 entries, is not parallelized."""
    c = W.Circuit()
    for q in range(13):
        c.h(q)
    for k in range(64):
        c.x(20 + k % 10, (k % 13,))
    w = W.Workload("q64", 40, 0.0, c.array(), capacity=1 << 13)
    o, _ = run(w, 4)
    assert o.totals()["parallel_runs"] == 0
    c.x(39)
    w = W.Workload("q65_4096", 40, 0.0, c.array()[1:], capacity=1 << 13)   # 12 H gates: 4096 entries
    o, _ = run(w, 4)
    assert o.totals()["parallel_runs"] == 0
