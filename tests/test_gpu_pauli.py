"""GPU parity of native Pauli exponentials exp(-i theta P) (sim_apply_pauli /
sim_gates_from_pauli + sim_apply_gates) against the oracle's Pauli runner.

Bar: sorted label sets bit-exact, amplitudes within 1e-12, the same skip
decisions.  Covers narrow and wide labels, terms across the 64-bit word
boundary, pairs whose partners both exist, controls, diagonal and identity
terms in both fused-pass kernels, the cap rule, the full-size Trotter step
(golden oracle digest) and the batched server.
"""
import json
import os
import sys

import numpy as np
import pytest

from helpers import assert_same_state, keys_digest
from oracle import Oracle, run_pauli_workload as oracle_pauli
from paper_2105_01533_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MASK64 = (1 << 64) - 1


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S():
    from paper_2105_01533_amd import sim
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sim


def run_both(S, n, terms, eps, capacity, state=None, basis=(0, 0), **kw):
    say(f"[gpu] pauli n={n} terms={len(terms)} eps={eps} cap={capacity} "
        f"entries={len(state[0]) if state else 1} {kw}")
    s = S.Simulator(n, capacity, eps, **kw)
    o = Oracle(n, eps)
    if state is None:
        s.set_basis(*basis)
        o.set_basis(*basis)
    else:
        s.import_state(*state)
        o.import_state(*state)
    _, st = s.apply_pauli(terms)
    g = s.export()
    s.close()
    tr = o.run_pauli(terms, trace=True)
    ref = o.export()
    return g, ref, st, o.totals(), tr


def check(S, n, terms, eps, capacity, **kw):
    g, ref, st, tot, _ = run_both(S, n, terms, eps, capacity, **kw)
    assert_same_state(g, ref, what=f"pauli n={n}")
    assert st["u2_applied"] == tot["u2_applied"] and st["u2_skipped"] == tot["u2_skipped"]
    return g, st


@pytest.mark.parametrize("seed", range(3))
def test_dense_small(S, seed):
    """n = 9 from |0>: the state fills up, so most pairs have both partners."""
    terms = W.random_pauli_terms(500 + seed, 9, 40, max_weight=5, ctrl_max=2, diag_frac=0.2, ident_frac=0.05)
    check(S, 9, terms, 0.0, 1 << 9)


@pytest.mark.parametrize("n,seed", [(40, 1), (64, 2), (70, 3), (128, 4)])
def test_random_state_ragged(S, n, seed):
    """A few thousand entries (several 2048-entry tiles, ragged tail), seven
    terms of weight up to 6 with controls."""
    lo, hi, amp = W.random_state(600 + seed, 2500 + 37 * seed, n)
    terms = W.random_pauli_terms(700 + seed, n, 7, max_weight=6, ctrl_max=2, diag_frac=0.2, ident_frac=0.1,
                                 theta_scale=1.0)
    check(S, n, terms, 1e-14, 1 << 20, state=(lo, hi, amp))


def test_partners_both_present_wide(S):
    """The state is closed under b -> b ^ x of the first term (x straddles the
    64-bit words), so every pair meets both partners and only the pivot-set
    label emits."""
    n = 128
    t0 = W.pauli_term([5, 63, 64, 100], ["Y", "X", "Y", "Z"], 0.37, ctrls=(7,))
    x = (int(t0[0]) | (int(t0[1]) << 64))
    lo, hi, amp = W.random_state(61, 1500, n)
    keys = [int(a) | (int(b) << 64) | (1 << 7) for a, b in zip(lo, hi)]
    keys = sorted(set(keys) | {k ^ x for k in keys})
    amps = W.random_amplitudes(62, len(keys))
    state = (np.array([k & MASK64 for k in keys], np.uint64), np.array([k >> 64 for k in keys], np.uint64), amps)
    terms = np.array([t0, W.pauli_term([0, 64], ["X", "X"], -0.8)], dtype=W.PAULI_DTYPE)
    g, st = check(S, n, terms, 0.0, 1 << 16, state=state)
    assert st["u2_applied"] == 2


@pytest.mark.parametrize("mode", ["direct", "bitslice"])
def test_diagonal_terms_both_fused_kernels(S, mode):
    """Z-only and identity terms run as CNOT-gathered parity phases inside a
    fused run, in either fused-pass kernel."""
    n = 80
    lo, hi, amp = W.random_state(81, 5000, n)
    terms = W.random_pauli_terms(82, n, 60, max_weight=6, ctrl_max=3, diag_frac=0.9, ident_frac=0.1)
    terms = terms[(terms["x_lo"] == 0) & (terms["x_hi"] == 0)]
    assert len(terms) > 40
    kw = {"mono_mode": 1} if mode == "direct" else {"mono_mode": 2, "bs_min_gates": 1}
    g, st = check(S, n, terms, 0.0, 1 << 13, state=(lo, hi, amp), **kw)
    assert st["u2_applied"] == 0
    if mode == "bitslice":
        assert st["bitslice_passes"] >= 1


def test_cap_rule(S):
    n = 30
    terms = W.random_pauli_terms(91, n, 20, max_weight=3, ctrl_max=0, diag_frac=0.2, cap=1 << 6)
    g, ref, st, tot, tr = run_both(S, n, terms, 1e-20, 1 << 8)
    assert_same_state(g, ref, what="cap")
    assert tot["u2_skipped"] > 0
    assert st["u2_skipped"] == tot["u2_skipped"] and st["u2_applied"] == tot["u2_applied"]


def test_trotter_scaled(S):
    w = W.config3_terms(seed=3007, terms=120)
    g, ref, st, tot, _ = run_both(S, w.n_qubits, w.terms, w.eps, w.capacity, basis=w.basis)
    assert_same_state(g, ref, what=w.name)
    assert st["u2_applied"] == tot["u2_applied"] and st["peak_nnz"] == tot["peak_nnz"]


def test_trotter_full_golden(S):
    """The 500-term Trotter step of 40 qubits as native terms, against the
    oracle's digest (tests/golden/make_golden.py)."""
    with open(os.path.join(GOLDEN, "config3_native_full.json")) as f:
        doc = json.load(f)
    w = W.config3_terms()
    say(f"[gpu] {w.name} terms={len(w.terms)}")
    s, st = S.run_pauli_workload(w)
    lo, hi, amp = s.export()
    s.close()
    assert len(lo) == doc["nnz"] and keys_digest(lo, hi) == doc["keys_sha256"]
    assert st["u2_applied"] == doc["u2_applied"] and st["u2_skipped"] == doc["u2_skipped"]
    assert st["peak_nnz"] == doc["peak_nnz"]
    err = 0.0
    for k, (slo, shi, re_, im_) in enumerate(doc["samples"]):
        i = k * doc["stride"]
        assert int(lo[i]) == slo and int(hi[i]) == shi
        err = max(err, abs(amp[i] - complex(float.fromhex(re_), float.fromhex(im_))))
    assert err <= 1e-12, err


def test_native_beats_decomposition_on_transients(S):
    """The native terms never hold more than the final state's worth of
    entries per step, while the basis-change decomposition of the same terms
    branches through 2^(number of X/Y) transients."""
    nat = W.config3_terms(seed=3011, terms=60)
    dec = W.config3(seed=3011, terms=60)
    s, st_n = S.run_pauli_workload(nat)
    s.close()
    s2, _, st_d = S.run_workload(dec)
    s2.close()
    assert st_n["peak_nnz"] < st_d["peak_nnz"]
    assert st_n["u2_applied"] < st_d["u2_applied"]


def test_server_runs_pauli_gates(S):
    """Converted Pauli terms submitted to the batched server, mixed with a
    standard-gate request: each result matches the oracle."""
    w = W.config3_terms(seed=3013, terms=80)
    gates = S.sim_gates_from_pauli(w.terms, w.n_qubits)
    small = W.random_pauli_terms(95, 70, 25, max_weight=4, ctrl_max=2)
    other = W.random_circuit(96, n=12, gates=200, h_frac=0.2, ctrl_max=2)
    other.capacity = 1 << 12
    srv = S.Server(1 << 28, max_slots=8, lane_capacity=S.SRV_LANE_OFF)   # the batched kernels
    ids = [srv.submit(S.sim_config(n_qubits=w.n_qubits, capacity=1 << 14, eps=w.eps), gates, w.basis),
           srv.submit(S.sim_config(n_qubits=70, capacity=1 << 16, eps=0.0), S.sim_gates_from_pauli(small, 70)),
           srv.submit_workload(other)]
    srv.run()
    res = []
    for rid in ids:
        st, err = srv.poll(rid)
        assert st == S.SRV_DONE, (st, err)
        res.append(srv.result(rid))
    srv.close()
    o, _ = oracle_pauli(w)
    assert_same_state(res[0][:3], o.export(), what="server trotter")
    o2 = Oracle(70, 0.0)
    o2.run_pauli(small)
    assert_same_state(res[1][:3], o2.export(), what="server random terms")
