"""Host side of the library's Pauli exponentials (CPU, no GPU calls).

sim_gates_from_pauli turns exp(-i theta P) terms into sim_gate ops.  These
tests interpret the ops it writes with a small dense model of the sim_gate
semantics the header documents (phase/permutation ops; branching ops with
partner label ^ x, pivot bit, off-diagonal sign (-1)^popcount(b0 & z)), and
compare the result with the oracle's Pauli runner, which works from the
closed form cos(theta) I - i sin(theta) P instead.  That checks the
conversion and the documented op semantics the kernels implement.
"""
import ctypes

import numpy as np
import pytest

from oracle import Oracle
from paper_2105_01533_amd import workloads as W

S = pytest.importorskip("paper_2105_01533_amd.sim")


def masks(g, f):
    return int(g[f + "_lo"]) | (int(g[f + "_hi"]) << 64)


def interpret(gates, psi, n):
    """Apply sim_gate records to a dense state, as the header defines them."""
    psi = psi.copy()
    idx = np.arange(1 << n)
    for g in gates:
        ctrl = masks(g, "ctrl")
        on = (idx & ctrl) == ctrl
        t = int(g["target"])
        m = g["m"]
        if g["op"] == S.SIM_OP_MONO:
            v = (idx >> t) & 1
            amp = np.where(on, psi * np.where(v == 1, m[1], m[0]), psi)
            dest = np.where(on & bool(g["flip"]), idx ^ (1 << t), idx)
            out = np.zeros_like(psi)
            out[dest] = amp
            psi = out
        else:
            assert g["op"] == S.SIM_OP_U2
            x = masks(g, "x") or (1 << t)
            z = masks(g, "z")
            assert (x >> t) & 1
            out = psi.copy()
            for b in idx[on & (((idx >> t) & 1) == 0)]:
                b1 = int(b) ^ x
                s = -1.0 if bin(int(b) & z).count("1") % 2 else 1.0
                out[b] = m[0] * psi[b] + s * m[1] * psi[b1]
                out[b1] = s * m[2] * psi[b] + m[3] * psi[b1]
            psi = out
    return psi


def oracle_dense(terms, psi, n):
    o = Oracle(n, 0.0)
    idx = np.arange(1 << n, dtype=np.uint64)
    o.import_state(idx, np.zeros_like(idx), psi)
    o.run_pauli(terms)
    lo, _, amp = o.export()
    out = np.zeros(1 << n, complex)
    out[lo.astype(np.int64)] = amp
    return out


@pytest.mark.parametrize("seed", range(5))
def test_conversion_matches_oracle(seed):
    n = 7
    terms = W.random_pauli_terms(1200 + seed, n, 30, max_weight=5, ctrl_max=2, diag_frac=0.25, ident_frac=0.1)
    psi = W.random_amplitudes(40 + seed, 1 << n)
    gates = S.sim_gates_from_pauli(terms, n)
    got = interpret(gates, psi, n)
    ref = oracle_dense(terms, psi, n)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_op_counts_and_fields():
    n = 100
    terms = np.array([
        W.pauli_term([3, 70, 80], ["Y", "X", "Z"], 0.2, ctrls=(5, 99), cap=64),
        W.pauli_term([1, 64, 90], ["Z", "Z", "Z"], 0.3),
        W.pauli_term([], [], 0.4),
        W.pauli_term([], [], 0.5, ctrls=(66, 7)),
        W.pauli_term([65], ["Y"], 0.6),
    ], dtype=W.PAULI_DTYPE)
    g = S.sim_gates_from_pauli(terms, n)
    assert len(g) == 1 + 5 + 1 + 1 + 1
    u = g[0]
    assert u["op"] == S.SIM_OP_U2 and u["target"] == 3 and u["cap"] == 64
    assert masks(u, "x") == (1 << 3) | (1 << 70) and masks(u, "z") == (1 << 3) | (1 << 80)
    assert masks(u, "ctrl") == (1 << 5) | (1 << 99)
    # one Y: u10 = -i sin * i = sin, u01 = -u10
    assert u["m"][2] == complex(np.sin(0.2), 0.0) and u["m"][1] == -u["m"][2]
    assert u["m"][0] == u["m"][3] == complex(np.cos(0.2), 0.0)
    diag = g[1:6]
    assert [int(x["target"]) for x in diag] == [1] * 5
    assert [masks(x, "ctrl") for x in diag] == [1 << 64, 1 << 90, 0, 1 << 90, 1 << 64]
    assert all(bool(x["flip"]) for x in diag[[0, 1, 3, 4]]) and not diag[2]["flip"]
    assert diag[2]["m"][0] == complex(np.cos(0.3), -np.sin(0.3)) and diag[2]["m"][1] == complex(np.cos(0.3),
                                                                                              np.sin(0.3))
    glob = g[6]
    assert glob["op"] == S.SIM_OP_MONO and glob["m"][0] == glob["m"][1] == complex(np.cos(0.4), -np.sin(0.4))
    ctl = g[7]
    assert ctl["target"] == 7 and masks(ctl, "ctrl") == 1 << 66 and ctl["m"][0] == 1
    assert g[8]["target"] == 65 and masks(g[8], "x") == masks(g[8], "z") == 1 << 65


def test_errors():
    n = 10
    bad = np.array([W.pauli_term([2], ["X"], 0.1, ctrls=(2,))], dtype=W.PAULI_DTYPE)
    with pytest.raises(S.SimError) as e:
        S.sim_gates_from_pauli(bad, n)
    assert e.value.code == S.SIM_E_ARG
    out_of_range = np.array([W.pauli_term([10], ["Z"], 0.1)], dtype=W.PAULI_DTYPE)
    with pytest.raises(S.SimError):
        S.sim_gates_from_pauli(out_of_range, n)
    nan = np.array([W.pauli_term([1], ["X"], float("nan"))], dtype=W.PAULI_DTYPE)
    with pytest.raises(S.SimError):
        S.sim_gates_from_pauli(nan, n)
    # a too-small buffer reports the count needed
    terms = np.array([W.pauli_term([1, 2, 3], ["Z", "Z", "Z"], 0.1)], dtype=W.PAULI_DTYPE)
    out = np.zeros(2, S.GATE_DTYPE)
    cnt = ctypes.c_size_t(0)
    rc = S._lib.sim_gates_from_pauli(S._ptr(terms), 1, n, S._ptr(out), 2, ctypes.byref(cnt))
    assert rc == S.SIM_E_BUFFER and cnt.value == 5
