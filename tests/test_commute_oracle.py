"""Pins for the oracle's gate-commuting runner (Sec. 3.3, Fig. 1).

The runner keeps per-qubit H, Rx and Ry queues behind the phase/permutation
queue.  It is pinned by:
  * the figure's worked sequence (a)-(e): which gates reach the state, in
    which order;
  * closed-form gate identities (H H = I, H Ry(a) H = Ry(-a), X H = H Z,
    Rx(a) Rx(-a) = I);
  * equivalence with the plain runner and with the dense simulator when no
    amplitude is pruned (eps = 0, no skip caps).
"""
import math

import numpy as np
import pytest

from dense_ref import Dense
from oracle import Oracle
from paper_2105_01533_amd import workloads as W

K = W


def log_list(log):
    return [(int(r["kind"]), int(r["target"]), int(r["ctrl_lo"]), round(float(r["param"]), 12)) for r in log]


def commuting(n, ops, eps=0.0, basis=0):
    o = Oracle(n, eps)
    o.set_basis(basis, 0)
    out, log = o.run_commuting(ops)
    return o, out, log


def state_dict(o):
    lo, hi, amp = o.export()
    return {int(a) | (int(b) << 64): complex(c) for a, b, c in zip(lo, hi, amp)}


def assert_close_states(d1, d2, tol=1e-12):
    for k in set(d1) | set(d2):
        assert abs(d1.get(k, 0) - d2.get(k, 0)) <= tol, (k, d1.get(k), d2.get(k))


def fig1_circuit():
    """Fig. 1 on 8 qubits: first the gates that leave the figure's starting
    queues (Q = CNOT(0->3), Z2, CZ(1,4); H pending on qubits 1-4; Ry(0.6) on
    qubit 1; Rx(0.75) on qubit 4), then steps (a)-(e)."""
    c = W.Circuit()
    c.x(3, (0,))
    c.gate(K.K_Z, 2)
    c.gate(K.K_Z, 4, (1,))
    for q in (1, 2, 3, 4):
        c.h(q)
    c.gate(K.K_RY, 1, (), param=0.6)
    c.gate(K.K_RX, 4, (), param=0.75)
    c.h(0)                                   # (a) H queued on qubit 0
    c.h(1)                                   # (b) Ry(0.6) -> Ry(-0.6), H H = I on qubit 1
    c.x(2)                                   # (c) X H = H Z: Z2 joins the queue
    c.x(5, (3, 4))                           # (d) CCNOT: queue, H3, H4, Rx4(0.75) executed
    c.gate(K.K_RX, 6, (), param=-math.pi / 4)  # (e) Rx queued, not applied
    return c


def test_fig1_worked_sequence():
    c = fig1_circuit()
    o, _, log = commuting(8, c.array())
    expect = [
        (K.K_X, 3, 1 << 0, 0.0), (K.K_Z, 2, 0, 0.0), (K.K_Z, 4, 1 << 1, 0.0),   # the queue before (d) ...
        (K.K_Z, 2, 0, 0.0),                                                    # ... with (c)'s Z2
        (K.K_H, 3, 0, 0.0), (K.K_H, 4, 0, 0.0), (K.K_RX, 4, 0, 0.75),          # (d): qubits 3 and 4
        (K.K_X, 5, (1 << 3) | (1 << 4), 0.0),                                 # end: the queue (CCNOT) ...
        (K.K_H, 0, 0, 0.0), (K.K_RY, 1, 0, -0.6), (K.K_H, 2, 0, 0.0),          # ... qubits 0, 1, 2
        (K.K_RX, 6, 0, round(-math.pi / 4, 12)),                               # ... and 6 from (e)
    ]
    assert log_list(log) == expect
    d = Dense(8)
    d.run(c.array())
    assert_close_states(state_dict(o), d.as_dict(1e-15))


def test_figure_step_d_executes_only_involved_qubits():
    """(d) executes the queue and the queues of the CCNOT's qubits (3, 4)
    before the CCNOT; qubits 0-2 stay queued until the end."""
    c = fig1_circuit()
    ops = c.array()
    o, _, log = commuting(8, ops[:-1])            # up to (d)
    lst = log_list(log)
    assert lst[7] == (K.K_X, 5, (1 << 3) | (1 << 4), 0.0)
    assert lst[:7] == [(K.K_X, 3, 1, 0.0), (K.K_Z, 2, 0, 0.0), (K.K_Z, 4, 2, 0.0), (K.K_Z, 2, 0, 0.0),
                       (K.K_H, 3, 0, 0.0), (K.K_H, 4, 0, 0.0), (K.K_RX, 4, 0, 0.75)]


@pytest.mark.parametrize("a", [0.3, -1.1, 2.5])
def test_closed_form_identities(a):
    def run(build):
        c = W.Circuit()
        build(c)
        return log_list(commuting(4, c.array())[2])

    assert run(lambda c: (c.h(1), c.h(1))) == []                                      # H H = I
    assert run(lambda c: (c.h(1), c.gate(K.K_RY, 1, (), param=a), c.h(1))) == [(K.K_RY, 1, 0, round(-a, 12))]
    assert run(lambda c: (c.h(2), c.x(2))) == [(K.K_Z, 2, 0, 0.0), (K.K_H, 2, 0, 0.0)]   # X H = H Z
    assert run(lambda c: (c.h(2), c.gate(K.K_Z, 2))) == [(K.K_X, 2, 0, 0.0), (K.K_H, 2, 0, 0.0)]
    assert run(lambda c: (c.h(2), c.x(2, (0,)))) == [(K.K_Z, 2, 1, 0.0), (K.K_H, 2, 0, 0.0)]   # CNOT -> CZ
    assert run(lambda c: (c.gate(K.K_RX, 0, (), param=a), c.gate(K.K_RX, 0, (), param=-a))) == []
    assert run(lambda c: (c.gate(K.K_RX, 0, (), param=a), c.h(0))) == [(K.K_RX, 0, 0, round(a, 12)),
                                                                      (K.K_H, 0, 0, 0.0)]
    assert run(lambda c: (c.gate(K.K_RY, 0, (), param=a), c.gate(K.K_RX, 0, (), param=0.5))) == [
        (K.K_RY, 0, 0, round(a, 12)), (K.K_RX, 0, 0, 0.5)]
    # a control with H pending, and S on an H-pending target, are executed first
    assert run(lambda c: (c.h(0), c.x(1, (0,)))) == [(K.K_H, 0, 0, 0.0), (K.K_X, 1, 1, 0.0)]
    assert run(lambda c: (c.h(0), c.gate(K.K_S, 0))) == [(K.K_H, 0, 0, 0.0), (K.K_S, 0, 0, 0.0)]


def test_measurement_executes_queue_and_qubit():
    c = W.Circuit()
    c.h(0)
    c.h(1)
    c.x(2, (3,))
    c.measure(0, 0.3)
    o, out, log = commuting(4, c.array())
    assert log_list(log) == [(K.K_X, 2, 8, 0.0), (K.K_H, 0, 0, 0.0), (K.K_MEASURE, 0, 0, 0.3),
                             (K.K_H, 1, 0, 0.0)]
    assert out.tolist() == [0]


def test_capped_gate_decides_where_applied():
    """A capped H is sent to the state at its place, after executing only its
    own qubit: here the H on qubit 0 is still queued, so nnz is 1 and the
    capped gate is applied (a plain run would have skipped it)."""
    c = W.Circuit()
    c.h(0)
    c.h(1, cap=2)
    o, _, log = commuting(4, c.array(), eps=1e-20)
    assert log_list(log) == [(K.K_H, 1, 0, 0.0), (K.K_H, 0, 0, 0.0)]
    assert o.nnz == 4
    p = Oracle(4, 1e-20)
    p.set_basis(0, 0)
    p.run(c.array())
    assert p.nnz == 2


def _circuit(seed, n, gates):
    return W.random_circuit(seed, n=n, gates=gates, h_frac=0.45, ctrl_max=2, measure_frac=0.03)


@pytest.mark.parametrize("seed", range(6))
def test_equivalent_to_plain_runner(seed):
    """With nothing pruned or skipped, commuting only reorders exactly
    commuting gates: same state (to rounding) and the same outcomes."""
    w = _circuit(300 + seed, 9, 300)
    o1, out1, log = commuting(9, w.ops)
    o2 = Oracle(9, 0.0)
    o2.set_basis(0, 0)
    out2, _ = o2.run(w.ops)
    assert out1.tolist() == out2.tolist()
    assert_close_states(state_dict(o1), state_dict(o2))
    assert len(log) <= len(w.ops)


@pytest.mark.parametrize("seed", range(4))
def test_vs_dense(seed):
    w = _circuit(400 + seed, 8, 250)
    o, out, _ = commuting(8, w.ops)
    d = Dense(8)
    outs = d.run(w.ops)
    assert out.tolist() == outs
    assert_close_states(state_dict(o), d.as_dict(1e-15))


def test_commuting_saves_branching_passes():
    """H H pairs and H-conjugated rotations never reach the state."""
    c = W.Circuit()
    for q in range(6):
        c.h(q)
        c.gate(K.K_RY, q, (), param=0.1 * (q + 1))
        c.h(q)
        c.h(q)
    o, _, log = commuting(6, c.array())
    kinds = [k for k, *_ in log_list(log)]
    assert kinds.count(K.K_H) == 6 and kinds.count(K.K_RY) == 6
