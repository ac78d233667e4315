"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them re-types the oracle's formulas:
worked states have closed forms, gate identities hold for the matrices of
Sec. 2.1, the dense Schrodinger simulator (Sec. 2.2) is a different algorithm
built on scipy's matrix exponential, and the adder is checked against integer
arithmetic.
"""
import math

import numpy as np
import pytest

from oracle import Oracle, monomial_samples, run_workload
from paper_2105_01533_amd import workloads as W
from dense_ref import Dense, pauli_string_matrix
from scipy.linalg import expm

S = math.sqrt(0.5)
ALL = (1 << 64) - 1


def state_dict(o: Oracle) -> dict:
    lo, hi, amp = o.export()
    return {int(l) | (int(h) << 64): complex(a) for l, h, a in zip(lo, hi, amp)}


def run_ops(n, c: W.Circuit, eps=0.0, basis=0, queued=True):
    o = Oracle(n, eps)
    o.set_basis(basis & ALL, basis >> 64)
    out, _ = o.run(c.array(), queued=queued)
    return o, out


# --- worked states ------------------------------------------------------------
def test_bell_state():
    c = W.Circuit()
    c.h(0)
    c.x(1, (0,))
    o, _ = run_ops(2, c)
    d = state_dict(o)
    assert set(d) == {0b00, 0b11}
    assert d[0] == S and d[3] == S


@pytest.mark.parametrize("n", [3, 64, 65, 128])
def test_ghz(n):
    c = W.Circuit()
    c.h(0)
    for q in range(1, n):
        c.x(q, (q - 1,))
    o, _ = run_ops(n, c)
    d = state_dict(o)
    assert set(d) == {0, (1 << n) - 1}
    assert d[0] == S and d[(1 << n) - 1] == S


def test_hh_is_identity_keys_exact():
    c = W.Circuit()
    c.h(5)
    c.h(5)
    o, _ = run_ops(8, c, eps=1e-20)
    d = state_dict(o)
    assert set(d) == {0}                       # |1> cancels exactly and is dropped
    assert abs(d[0] - 1.0) <= 4.5e-16          # 2 * fl(sqrt(.5))^2


def test_h_layer_10():
    c = W.Circuit()
    for q in range(10):
        c.h(q)
    o, _ = run_ops(24, c, eps=1e-20)
    d = state_dict(o)
    assert set(d) == set(range(1024))
    assert all(abs(a - 2.0 ** -5) < 1e-15 for a in d.values())


def test_x_layer_128_all_ones():
    c = W.Circuit()
    for q in range(128):
        c.x(q)
    o, _ = run_ops(128, c)
    lo, hi, amp = o.export()
    assert lo.tolist() == [ALL] and hi.tolist() == [ALL] and amp[0] == 1.0


# --- gate identities ------------------------------------------------------------
def _superposed(n, c):
    for q in range(n):
        c.h(q)
    c.gate(W.K_RY, 0, (), param=0.7)
    c.gate(W.K_RX, 1, (), param=-1.3)


@pytest.mark.parametrize("a,b,times", [
    (W.K_S, W.K_Z, 2), (W.K_T, W.K_S, 2), (W.K_SDG, W.K_S, 3), (W.K_TDG, W.K_T, 7)])
def test_power_identities(a, b, times):
    """S^2 = Z, T^2 = S, (S^dagger)^3 = S, (T^dagger)^7 = T, controlled too."""
    for ctrls in [(), (2,)]:
        c1, c2 = W.Circuit(), W.Circuit()
        _superposed(3, c1)
        _superposed(3, c2)
        for _ in range(times):
            c1.gate(a, 1, ctrls)
        c2.gate(b, 1, ctrls)
        d1, d2 = state_dict(run_ops(3, c1)[0]), state_dict(run_ops(3, c2)[0])
        assert set(d1) == set(d2)
        assert max(abs(d1[k] - d2[k]) for k in d1) < 1e-15


def test_rz_2pi_is_minus_identity():
    c1, c2 = W.Circuit(), W.Circuit()
    _superposed(3, c1)
    _superposed(3, c2)
    c1.gate(W.K_RZ, 2, (), param=2 * math.pi)
    d1, d2 = state_dict(run_ops(3, c1)[0]), state_dict(run_ops(3, c2)[0])
    assert max(abs(d1[k] + d2[k]) for k in d1) < 1e-15


def test_hzh_is_x_and_hxh_is_z():
    for inner, outer in [(W.K_Z, W.K_X), (W.K_X, W.K_Z)]:
        c1, c2 = W.Circuit(), W.Circuit()
        for c in (c1, c2):
            _superposed(3, c)
        c1.h(1)
        c1.gate(inner, 1)
        c1.h(1)
        c2.gate(outer, 1)
        d1, d2 = state_dict(run_ops(3, c1, eps=1e-24)[0]), state_dict(run_ops(3, c2, eps=1e-24)[0])
        assert set(d1) == set(d2)
        assert max(abs(d1[k] - d2[k]) for k in d1) < 1e-14


# --- dense Schrodinger simulator on random circuits -----------------------------
def _compare_dense(w, eps_keys=1e-12, tol=1e-12):
    o, outs, tr = run_workload(w, trace=True)
    basis = w.basis[0] | (w.basis[1] << 64)
    d = Dense(w.n_qubits, basis)
    skipped = {i for i, t in enumerate(tr) if t["applied"] == 0}
    douts = d.run(w.ops, skip_cap_nnz=lambda i: i in skipped)
    assert list(outs) == douts
    sp = state_dict(o)
    dd = d.as_dict(tol=eps_keys)
    assert set(dd) <= set(sp)
    for k, a in sp.items():
        assert abs(a - d.psi[k]) < tol, (k, a, d.psi[k])
    return o


@pytest.mark.parametrize("seed", range(6))
def test_random_circuits_vs_dense(seed):
    w = W.random_circuit(seed, n=7, gates=120, h_frac=0.25, ctrl_max=3)
    _compare_dense(w)


@pytest.mark.parametrize("seed", range(4))
def test_random_circuits_with_measurement_vs_dense(seed):
    w = W.random_circuit(100 + seed, n=6, gates=150, h_frac=0.3, ctrl_max=2, measure_frac=0.05)
    _compare_dense(w)


def test_config0_scaled_vs_dense():
    w = W.config0(7, n=12, h_qubits=6, gates=800, cap=1 << 9)
    w.eps = 0.0
    _compare_dense(w)


def test_config2_scaled_vs_dense():
    w = W.config2(11, n=14, h_qubits=7, gates=3000, round_gates=600, meas_per_round=2)
    w.eps = 0.0
    _compare_dense(w)


def test_skip_rule():
    """Branching gate with cap: skipped iff 2*nnz > cap."""
    c = W.Circuit()
    c.h(0, cap=2)      # nnz 1: 2 > 2 false -> applied (nnz 2)
    c.h(1, cap=2)      # nnz 2: 4 > 2 -> skipped
    c.h(1, cap=4)      # 4 > 4 false -> applied (nnz 4)
    o = Oracle(4, 1e-20)
    _, tr = o.run(c.array(), trace=True)
    assert tr["applied"].tolist() == [1, 0, 1]
    assert tr["nnz_in"].tolist() == [1, 2, 2]
    assert o.nnz == 4


# --- Pauli exponentials: closed form exp(-i theta P) = cos I - i sin P ----------
@pytest.mark.parametrize("seed", range(8))
def test_pauli_exponential_closed_form(seed):
    rng = W.SplitMix64(seed + 77)
    n = 6
    qs = sorted(rng.distinct(n, 4))
    ps = ["XYZ"[rng.randint(3)] for _ in qs]
    theta = 0.5 * rng.normal()
    prep = W.Circuit()
    _superposed(n, prep)
    c = W.Circuit()
    c.rows = list(prep.rows)
    W.pauli_exp(c, qs, ps, theta)
    d = Dense(n)
    d.run(prep.array())
    P = pauli_string_matrix(n, qs, ps)
    want = (math.cos(theta) * np.eye(1 << n) - 1j * math.sin(theta) * P) @ d.psi
    want2 = expm(-1j * theta * P) @ d.psi
    assert np.max(np.abs(want - want2)) < 1e-13
    got = state_dict(run_ops(n, c)[0])
    vec = np.zeros(1 << n, complex)
    for k, a in got.items():
        vec[k] = a
    assert np.max(np.abs(vec - want)) < 1e-13


# --- CDKM adder: integer arithmetic -----------------------------------------------
@pytest.mark.parametrize("w", [1, 2, 3, 4])
def test_cdkm_adder_all_inputs(w):
    A, B = list(range(w)), list(range(w, 2 * w))
    c0, z = 2 * w, 2 * w + 1
    add = W.Circuit()
    W.cdkm_add(add, A, B, c0, z)
    ops = add.array()
    n = 2 * w + 2
    for a in range(1 << w):
        for b in range(1 << w):
            for zin in (0, 1):
                key = a | (b << w) | (zin << z)
                lo, hi, amp = monomial_samples(ops, [key], [0], [1.0])
                s = a + b
                want = (s & ((1 << w) - 1)) | (b << w) | ((zin ^ (s >> w)) << z)
                assert int(lo[0]) == want and hi[0] == 0 and amp[0] == 1.0
    assert n <= 10


def test_config1_closed_form():
    """A <- (a + adds*c) mod 2^w, B = c, c0 = 0, z = parity of the carries."""
    w_bits, adds = 6, 9
    wl = W.config1(123, w=w_bits, adds=adds, n=16)
    const = wl.meta["const"]
    kinds = wl.ops["kind"]
    first_h_tail = len(wl.ops) - w_bits
    body = wl.ops[w_bits:first_h_tail]                 # loads, adds, ladder
    assert np.all(np.isin(kinds[w_bits:first_h_tail], W.MONOMIAL_KINDS))
    keys = np.arange(1 << w_bits, dtype=np.uint64)
    lo, hi, amp = monomial_samples(body, keys, np.zeros_like(keys), np.ones(len(keys)))
    mask = (1 << w_bits) - 1
    for a in range(1 << w_bits):
        acc, z = a, 0
        for _ in range(adds):
            s = acc + const
            z ^= s >> w_bits
            acc = s & mask
        want = acc | (const << w_bits) | (z << (2 * w_bits + 1))
        assert int(lo[a]) == want
        # the ladder phase: product over (i, j) with A[i] and A[i+j] set of e^{+-i pi/2^(j+1)}
        ph = 0.0
        for i in range(w_bits):
            for j in range(1, w_bits - i):
                if (acc >> (i + j)) & 1:
                    ph += (math.pi / (1 << j)) / 2 * (1 if (acc >> i) & 1 else -1)
        assert abs(amp[a] - np.exp(1j * ph)) < 1e-14


# --- invariants -------------------------------------------------------------------
def test_queued_equals_gate_by_gate_bitwise():
    for w in [W.config0(5, gates=1500), W.config2(9, n=100, h_qubits=10, gates=4000, round_gates=1000,
                                                   meas_per_round=3),
              W.config3(4, terms=40), W.random_circuit(3, n=9, gates=300, h_frac=0.2)]:
        o1, out1, _ = run_workload(w, queued=True)
        o2, out2, _ = run_workload(w, queued=False)
        a, b = o1.export(), o2.export()
        assert list(out1) == list(out2)
        for x, y in zip(a, b):
            assert x.tobytes() == y.tobytes()


def test_permutations_preserve_nnz_and_amplitudes():
    w = W.config2(21, n=100, h_qubits=12, gates=3000, round_gates=10 ** 9)
    pre = W.Circuit()
    for q in range(12):
        pre.h(q)
    for q in range(3):
        pre.gate(W.K_RY, q, (), param=0.3 + q)
    o = Oracle(100, 1e-20)
    o.run(pre.array())
    lo0, hi0, amp0 = o.export()
    perm = w.ops[np.isin(w.ops["kind"], (W.K_X,))]
    o.run(perm)
    lo1, hi1, amp1 = o.export()
    assert len(lo1) == len(lo0)
    assert sorted(amp0.view(np.uint64).tolist()) == sorted(amp1.view(np.uint64).tolist())


def test_norm_plus_pruned_mass():
    w = W.config3(8, terms=60)
    o, _, _ = run_workload(w)
    lo, hi, amp = o.export()
    t = o.totals()
    assert abs(np.sum(np.abs(amp) ** 2) + t["pruned_mass"] - 1.0) < 1e-9
    assert t["pruned"] > 0


def test_measurement_born_rule_and_collapse():
    c = W.Circuit()
    c.h(0)
    c.x(1, (0,))
    c.gate(W.K_RY, 2, (), param=1.0)
    o = Oracle(3)
    o.run(c.array())
    p0, p1 = o.probabilities(2)
    assert abs(p0 - math.cos(0.5) ** 2) < 1e-15 and abs(p1 - math.sin(0.5) ** 2) < 1e-15
    m = W.Circuit()
    m.measure(0, 0.99)                  # u >= p0 = 1/2 -> outcome 1
    out, _ = o.run(m.array())
    assert out.tolist() == [1]
    d = state_dict(o)
    assert set(d) == {0b011, 0b111}
    assert abs(sum(abs(a) ** 2 for a in d.values()) - 1) < 1e-15
    m2 = W.Circuit()
    m2.measure(2, 0.0, forced=0)
    o.run(m2.array())
    d = state_dict(o)
    assert list(d) == [0b011] and abs(d[0b011] - 1) < 1e-15


def test_circuit_then_inverse_returns_initial_state():
    """A random permutation/phase/H circuit followed by its inverse."""
    rng = W.SplitMix64(99)
    c = W.Circuit()
    for q in range(6):
        c.h(q)
    body = W.Circuit()
    for _ in range(400):
        W._random_mono(rng, body, 40, 0.7, 0.25, 0)
    inv = {W.K_S: W.K_SDG, W.K_T: W.K_TDG}
    c.rows += body.rows
    for r in reversed(body.rows):
        kind, t, lo, hi, th, cap, f, p = r
        if kind == W.K_RZ:
            th = -th
        c.rows.append((inv.get(kind, kind), t, lo, hi, th, cap, f, p))
    o, _ = run_ops(40, c, eps=1e-20)
    d = state_dict(o)
    assert set(d) == set(range(64))
    assert max(abs(a - 0.125) for a in d.values()) < 1e-13


def test_eps_boundary_is_strict():
    """T_eps drops an entry iff re*re + im*im < eps (the reading of the
    paper's 'only nonzero amplitudes are stored' with a threshold): after an
    exact identity branching gate (Rx(0): cos 0 = 1, sin 0 = 0, Eq. 2 with
    U = I), an amplitude whose |a|^2 is exactly eps survives, in the real and
    in the imaginary part, and the next double below it is dropped; the
    absent partners' exact zeros are dropped too."""
    x = 3.0e-11
    eps = x * x
    below, above = np.nextafter(x, 0.0), np.nextafter(x, 1.0)
    assert below * below < eps < above * above
    lo = np.array([0b0001, 0b0011, 0b0101, 0b0111, 0b1001, 0b1011], np.uint64)
    amp = np.array([x, below, above, 1j * x, 1j * below, 0.5], np.complex128)
    c = W.Circuit()
    c.gate(W.K_RX, 6, param=0.0)
    o = Oracle(8, eps)
    o.import_state(lo, np.zeros(6, np.uint64), amp)
    o.run(c.array())
    glo, _, gamp = o.export()
    assert [int(v) for v in glo] == [0b0001, 0b0101, 0b0111, 0b1011]
    assert list(gamp) == [x, above, 1j * x, 0.5]          # passed through exactly
    t = o.totals()
    assert t["pruned"] == 6 + 2
    assert t["pruned_mass"] == below * below + below * below


def test_prune_margin_closed_form():
    """The oracle's decision margin min | |a|^2 - eps | / eps (a diagnostic;
    the state is untouched): H on |0> gives |a|^2 = 1/2 twice, so with
    eps = 0.4 the margin is (0.5 - 0.4) / 0.4 = 0.25; in the T_eps test state
    above (|a|^2 = eps exactly) it is 0; with eps = 0 nothing is examined
    (+inf); phase/permutation gates never change it."""
    c = W.Circuit()
    c.h(0)
    o = Oracle(4, 0.4)
    o.run(c.array())
    assert o.totals()["min_margin"] == pytest.approx((0.5 - 0.4) / 0.4, rel=1e-15)
    lo, _, amp = o.export()
    assert len(lo) == 2 and np.allclose(np.abs(amp) ** 2, 0.5)
    x = 3.0e-11
    o = Oracle(8, x * x)
    o.import_state(np.array([1], np.uint64), np.zeros(1, np.uint64), np.array([x], np.complex128))
    c = W.Circuit()
    c.gate(W.K_RX, 6, param=0.0)
    o.run(c.array())
    assert o.totals()["min_margin"] == 0.0
    o = Oracle(4, 0.0)
    c = W.Circuit()
    c.h(0)
    c.x(1)
    o.run(c.array())
    assert o.totals()["min_margin"] == math.inf
    o = Oracle(4, 0.4)
    c = W.Circuit()
    c.x(1)
    c.gate(W.K_T, 1)
    o.run(c.array())
    assert o.totals()["min_margin"] == math.inf
