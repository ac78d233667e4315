"""The library's gate-commuting rewrite (sim_commute_ops, host only) against
the oracle's commuting runner: the same ops reach the state, in the same
order, bit for bit (the oracle's runner is pinned in test_commute_oracle.py).
No GPU needed."""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_2105_01533_amd import sim as S
from paper_2105_01533_amd import workloads as W
from test_commute_oracle import fig1_circuit


def oracle_log(n, ops, eps=0.0):
    o = Oracle(n, eps)
    o.set_basis(0, 0)
    _, log = o.run_commuting(ops)
    return log


def same_ops(a, b):
    assert len(a) == len(b)
    for f in ("kind", "target", "ctrl_lo", "ctrl_hi", "cap", "forced"):
        assert np.array_equal(a[f], b[f]), f
    assert a["param"].tobytes() == b["param"].tobytes()


def test_fig1_sequence():
    ops = fig1_circuit().array()
    same_ops(S.sim_commute_ops(ops, 8), oracle_log(8, ops))


@pytest.mark.parametrize("seed", range(8))
def test_random_circuits(seed):
    n = (5, 9, 64, 100)[seed % 4]
    wide = n > 16     # keep the oracle's states small: fewer gates and H's on wide registers
    w = W.random_circuit(500 + seed, n=n, gates=150 if wide else 600, h_frac=0.2 if wide else 0.45, ctrl_max=3,
                         measure_frac=0.02)
    same_ops(S.sim_commute_ops(w.ops, n), oracle_log(n, w.ops))


def test_configs():
    # (Skip caps are decided where a gate is applied, so commuting suits
    # circuits without them.  On the Trotter-like circuit the postponed
    # basis-change H's keep transient states large, so few terms here.)
    for w in (W.config3(terms=15), W.config1(3, w=6, adds=4, n=24)):
        same_ops(S.sim_commute_ops(w.ops, w.n_qubits), oracle_log(w.n_qubits, w.ops, eps=w.eps))


def test_invalid_and_buffer():
    c = W.Circuit()
    c.h(0)
    c.x(1, (0,))
    ops = c.array()
    bad = ops.copy()
    bad["target"][1] = 7
    with pytest.raises(S.SimError):
        S.sim_commute_ops(bad, 4)
    assert len(S.sim_commute_ops(ops, 4)) == 2
    assert len(S.sim_commute_ops(ops[:0], 4)) == 0
