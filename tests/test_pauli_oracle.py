"""Pins for the oracle's Pauli-exponential runner, exp(-i theta P) (Sec. 3's
intrinsic operations with at most two nonzeros per row).

The runner applies the closed form cos(theta) I - i sin(theta) P term by term.
It is pinned against things it shares no code with:
  * scipy's expm of the dense Kronecker-product matrix of P (controlled terms
    as |1..1><1..1| on the controls (x) U + the rest), on random dense states;
  * the single-qubit cases exp(-i theta X/Y/Z) = Rx/Ry/Rz(2 theta) of the
    oracle's standard-gate runner;
  * the basis-change / CNOT-ladder / Rz decomposition the Trotter workload
    uses (itself pinned against the closed form in test_oracle_pins);
  * theta = pi/2, where the term is -i P: the standard X, Y, Z gates applied
    one by one;
  * group identities (inverse, angle addition), norm, and the readings on the
    cap and the prune.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from dense_ref import pauli_string_matrix
from oracle import Oracle
from paper_2105_01533_amd import workloads as W

MASK64 = (1 << 64) - 1


def state_dict(o):
    lo, hi, amp = o.export()
    return {int(a) | (int(b) << 64): complex(c) for a, b, c in zip(lo, hi, amp)}


def assert_close(d1, d2, tol):
    for k in set(d1) | set(d2):
        assert abs(d1.get(k, 0) - d2.get(k, 0)) <= tol, (hex(k), d1.get(k), d2.get(k))


def dense_state(seed, n):
    amp = W.random_amplitudes(seed, 1 << n)
    return amp


def load_dense(o, psi):
    idx = np.nonzero(psi)[0].astype(np.uint64)
    o.import_state(idx, np.zeros_like(idx), psi[idx.astype(np.int64)])


def term_parts(rec, n):
    x = int(rec["x_lo"]) | (int(rec["x_hi"]) << 64)
    z = int(rec["z_lo"]) | (int(rec["z_hi"]) << 64)
    qs, ps = [], []
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        if xb or zb:
            qs.append(q)
            ps.append("Y" if xb and zb else ("X" if xb else "Z"))
    ctrl = int(rec["ctrl_lo"]) | (int(rec["ctrl_hi"]) << 64)
    return qs, ps, ctrl


def dense_term(n, rec):
    qs, ps, ctrl = term_parts(rec, n)
    P = pauli_string_matrix(n, qs, ps) if qs else np.eye(1 << n, dtype=complex)
    U = expm(-1j * float(rec["theta"]) * P)
    idx = np.arange(1 << n)
    on = (idx & ctrl) == ctrl
    proj = np.diag(on.astype(complex))
    return proj @ U + np.diag((~on).astype(complex))


@pytest.mark.parametrize("seed", range(4))
def test_vs_expm_dense(seed):
    n = 6
    terms = W.random_pauli_terms(900 + seed, n, 25, max_weight=4, ctrl_max=2)
    psi = dense_state(77 + seed, n)
    o = Oracle(n, 0.0)
    load_dense(o, psi)
    o.run_pauli(terms)
    for rec in terms:
        psi = dense_term(n, rec) @ psi
    ref = {i: psi[i] for i in range(1 << n) if psi[i] != 0}
    assert_close(state_dict(o), ref, 1e-12)


@pytest.mark.parametrize("theta", [0.3, -1.7, 2.9])
def test_single_qubit_reduces_to_rotations(theta):
    n = 5
    psi = dense_state(5, n)
    for p, kind in (("X", W.K_RX), ("Y", W.K_RY), ("Z", W.K_RZ)):
        for ctrls in ((), (0, 4)):
            a = Oracle(n, 0.0)
            load_dense(a, psi)
            a.run_pauli(np.array([W.pauli_term([2], [p], theta, ctrls)], dtype=W.PAULI_DTYPE))
            b = Oracle(n, 0.0)
            load_dense(b, psi)
            c = W.Circuit()
            c.gate(kind, 2, ctrls, param=2.0 * theta)
            b.run(c.array())
            assert_close(state_dict(a), state_dict(b), 1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_matches_trotter_decomposition(seed):
    """config3's terms as native records vs config3's circuit (same draws);
    no pruning so both are exact up to rounding."""
    n, terms = 16, 12
    nat = W.config3_terms(seed=3000 + seed, n=n, set_bits=8, terms=terms)
    dec = W.config3(seed=3000 + seed, n=n, set_bits=8, terms=terms)
    a = Oracle(n, 0.0)
    a.set_basis(*nat.basis)
    a.run_pauli(nat.terms)
    b = Oracle(n, 0.0)
    b.set_basis(*dec.basis)
    b.run(dec.ops)
    assert a.nnz > 100
    assert_close(state_dict(a), state_dict(b), 1e-12)


def test_wide_labels_match_decomposition():
    """Terms straddling the 64-bit word boundary of 128-qubit labels."""
    n = 128
    rng = W.SplitMix64(123)
    circ = W.Circuit()
    recs = []
    for _ in range(10):
        qs = sorted(set(rng.distinct(n, 3)) | {63 + rng.randint(2)})
        ps = ["XYZ"[rng.randint(3)] for _ in qs]
        theta = rng.uniform() - 0.5
        recs.append(W.pauli_term(qs, ps, theta))
        W.pauli_exp(circ, qs, ps, theta)
    basis = (0xF0F0 << 56) | (0xABC << 100)
    a = Oracle(n, 0.0)
    a.set_basis(basis & MASK64, basis >> 64)
    a.run_pauli(np.array(recs, dtype=W.PAULI_DTYPE))
    b = Oracle(n, 0.0)
    b.set_basis(basis & MASK64, basis >> 64)
    b.run(circ.array())
    assert a.nnz > 1
    assert_close(state_dict(a), state_dict(b), 1e-12)


@pytest.mark.parametrize("paulis", ["XYZ", "YYX", "ZXY", "YZZ"])
def test_half_pi_is_minus_i_pauli(paulis):
    """exp(-i pi/2 P) = -i P: the standard X, Y, Z gates applied in turn (the
    cos(pi/2) ~ 6e-17 leftovers fall under eps)."""
    n = 7
    qs = [1, 3, 6]
    psi = dense_state(11, n)
    a = Oracle(n, 1e-20)
    load_dense(a, psi)
    a.run_pauli(np.array([W.pauli_term(qs, list(paulis), math.pi / 2)], dtype=W.PAULI_DTYPE))
    b = Oracle(n, 0.0)
    load_dense(b, psi)
    c = W.Circuit()
    kinds = {"X": W.K_X, "Y": W.K_Y, "Z": W.K_Z}
    for q, p in zip(qs, paulis):
        c.gate(kinds[p], q)
    b.run(c.array())
    ref = {k: -1j * v for k, v in state_dict(b).items()}
    assert a.nnz == 1 << n
    assert_close(state_dict(a), ref, 1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_inverse_and_angle_addition(seed):
    n = 9
    terms = W.random_pauli_terms(950 + seed, n, 8, max_weight=5, ctrl_max=2)
    psi = dense_state(21 + seed, n)
    # exp(-i a P) exp(-i b P) = exp(-i (a + b) P)
    for rec in terms:
        two = np.array([rec, rec], dtype=W.PAULI_DTYPE)
        two["theta"] = [0.4, float(rec["theta"]) - 0.4]
        a = Oracle(n, 0.0)
        load_dense(a, psi)
        a.run_pauli(two)
        b = Oracle(n, 0.0)
        load_dense(b, psi)
        b.run_pauli(np.array([rec], dtype=W.PAULI_DTYPE))
        assert_close(state_dict(a), state_dict(b), 1e-13)
    # the terms followed by their inverses in reverse order give the identity
    inv = terms[::-1].copy()
    inv["theta"] = -inv["theta"]
    a = Oracle(n, 0.0)
    load_dense(a, psi)
    a.run_pauli(np.concatenate([terms, inv]))
    assert_close(state_dict(a), {i: psi[i] for i in range(1 << n)}, 1e-13)


def test_norm_preserved_and_totals():
    n = 10
    terms = W.random_pauli_terms(77, n, 40, max_weight=4, ctrl_max=1, diag_frac=0.3, ident_frac=0.1)
    o = Oracle(n, 0.0)
    tr = o.run_pauli(terms, trace=True)
    _, _, amp = o.export()
    assert abs(float(np.sum(np.abs(amp) ** 2)) - 1.0) < 1e-13
    branching = (terms["x_lo"] != 0) | (terms["x_hi"] != 0)
    t = o.totals()
    assert t["u2_applied"] == int(branching.sum())
    assert t["mono_gates"] == int((~branching).sum())
    assert t["updates"] == int(tr["nnz_in"].sum())


def test_cap_skips_only_branching_terms():
    n = 6
    o = Oracle(n, 1e-20)
    terms = np.array([W.pauli_term([0], ["X"], 0.3),            # 1 -> 2 entries
                      W.pauli_term([1], ["Y"], 0.3, cap=3),     # 2*2 > 3: skipped
                      W.pauli_term([1, 2], ["Z", "Z"], 0.3, cap=1),   # diagonal: cap ignored
                      W.pauli_term([3], ["X"], 0.3, cap=4)],    # 2*2 <= 4: applied
                     dtype=W.PAULI_DTYPE)
    tr = o.run_pauli(terms, trace=True)
    assert tr["applied"].tolist() == [1, 0, 1, 1]
    assert o.nnz == 4
    t = o.totals()
    assert (t["u2_applied"], t["u2_skipped"], t["mono_gates"]) == (2, 1, 1)


def test_diagonal_terms_never_prune():
    """A Z-only term is a phase gate: amplitudes below eps stay."""
    n = 4
    o = Oracle(n, 1e-6)
    o.import_state(np.array([0, 1, 3], np.uint64), np.zeros(3, np.uint64),
                   np.array([1.0, 1e-4, 1e-5j], complex))
    o.run_pauli(np.array([W.pauli_term([0, 1], ["Z", "Z"], 0.7)], dtype=W.PAULI_DTYPE))
    assert o.nnz == 3
    d = state_dict(o)
    assert abs(d[1] - 1e-4 * np.exp(0.7j)) < 1e-18          # parity 1: e^{+i theta}
    assert abs(d[3] - 1e-5j * np.exp(-0.7j)) < 1e-18        # parity 0: e^{-i theta}
    # a branching term prunes: every entry but label 0 (and label 0's new
    # branch, |sin 1e-4|^2 ~ 1e-8) falls under eps
    o.run_pauli(np.array([W.pauli_term([2], ["X"], 1e-4)], dtype=W.PAULI_DTYPE))
    assert set(state_dict(o)) == {0}


def test_controls_leave_other_labels_bitwise():
    n = 6
    psi = dense_state(3, n)
    o = Oracle(n, 0.0)
    load_dense(o, psi)
    o.run_pauli(np.array([W.pauli_term([0, 2], ["Y", "X"], 0.9, ctrls=(4, 5))], dtype=W.PAULI_DTYPE))
    d = state_dict(o)
    for i in range(1 << n):
        if (i >> 4) & 3 != 3:
            assert d[i] == psi[i]


def test_invalid_terms_rejected():
    o = Oracle(6, 0.0)
    from oracle import OracleError
    with pytest.raises(OracleError):
        o.run_pauli(np.array([W.pauli_term([6], ["X"], 0.1)], dtype=W.PAULI_DTYPE))      # out of range
    with pytest.raises(OracleError):
        o.run_pauli(np.array([W.pauli_term([1], ["X"], 0.1, ctrls=(1,))], dtype=W.PAULI_DTYPE))   # ctrl on P
