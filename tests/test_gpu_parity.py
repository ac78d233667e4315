"""GPU parity: the HIP library against the CPU oracle, through the C-ABI.

Bar: sorted label sets bit-exact, amplitudes within 1e-12 (complex modulus),
identical measurement outcomes and skip decisions.  Sizes span many blocks
and ragged tails; the full-size workloads are checked against the oracle
where it finishes in seconds, against golden oracle digests where it does not
(tests/golden/make_golden.py), and on oracle-computed samples at the largest
size.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from helpers import assert_same_state, keys_digest, lookup, sorted_unique
from oracle import Oracle, monomial_samples, run_workload as oracle_run
from paper_2105_01533_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sim():
    from paper_2105_01533_amd import sim as S
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return S


def gpu_run(S, w, **kw):
    say(f"[gpu] {w.name} ops={len(w.ops)} n={w.n_qubits} cap={w.capacity} {kw}")
    s, outcomes, stats = S.run_workload(w, **kw)
    out = s.export()
    s.close()
    return out, outcomes, stats


def check_vs_oracle(S, w, tol=1e-12, **kw):
    g, gout, gst = gpu_run(S, w, **kw)
    o, oout, _ = oracle_run(w)
    assert list(gout) == list(oout), "measurement outcomes differ"
    assert_same_state(g, o.export(), tol, w.name)
    t = o.totals()
    assert gst["u2_applied"] == t["u2_applied"] and gst["u2_skipped"] == t["u2_skipped"]
    assert gst["updates"] == t["updates"]
    assert gst["pruned"] == t["pruned"]
    assert abs(gst["pruned_mass"] - t["pruned_mass"]) <= 1e-12, (gst["pruned_mass"], t["pruned_mass"])
    return g, gst


# --- worked states ------------------------------------------------------------
def test_bell_ghz_x128(sim):
    for n in (2, 64, 65, 128):
        c = W.Circuit()
        c.h(0)
        for q in range(1, n):
            c.x(q, (q - 1,))
        w = W.Workload(f"ghz{n}", n, 0.0, c.array(), capacity=4)
        g, _ = check_vs_oracle(sim, w)
        assert len(g[0]) == 2 and g[2][0] == math.sqrt(0.5)
    c = W.Circuit()
    for q in range(128):
        c.x(q)
    g, _ = check_vs_oracle(sim, W.Workload("x128", 128, 0.0, c.array(), capacity=2))
    assert g[0].tolist() == [2 ** 64 - 1] and g[1].tolist() == [2 ** 64 - 1] and g[2][0] == 1.0


def _eps_boundary_case():
    """A state whose pass through an exact identity branching gate (Rx(0):
    cos 0 = 1, sin 0 = 0) leaves one amplitude with |a|^2 exactly eps, one
    just below and one just above, in the real and in the imaginary part."""
    x = 3.0e-11
    eps = x * x                                  # |(x, 0)|^2 = re*re + 0 exactly
    below, above = np.nextafter(x, 0.0), np.nextafter(x, 1.0)
    assert below * below < eps < above * above
    lo = np.array([0b0001, 0b0011, 0b0101, 0b0111, 0b1001, 0b1011], np.uint64)
    hi = np.zeros(6, np.uint64)
    amp = np.array([x, below, above, 1j * x, 1j * below, 0.5], np.complex128)
    c = W.Circuit()
    c.gate(W.K_RX, 6, param=0.0)                 # qubit 6 is clear in every label: partners are absent
    return 8, eps, lo, hi, amp, c.array(), {0b0001, 0b0101, 0b0111, 0b1011}


def test_eps_boundary(sim):
    """T_eps drops iff |a|^2 < eps: an entry exactly at eps survives, on the
    single-state path (both fused-pass forms do not prune; the branching
    kernels do) and in the batched server."""
    nq, eps, lo, hi, amp, ops, keep = _eps_boundary_case()
    from paper_2105_01533_amd.sim import Server, Simulator, sim_config, sim_gates_from_ops
    for flags in (0, sim.SIM_FLAG_U2_TWO_PASS):
        s = Simulator(nq, 64, eps, flags=flags)
        s.import_state(lo, hi, amp)
        _, _, st = s.apply_ops(ops)
        glo, ghi, gamp = s.export()
        s.close()
        assert set(int(v) for v in glo) == keep, (flags, glo)
        assert st["pruned"] == 6 + 2                # six absent partners (exact zeros) + two below eps
        ref = {int(k): a for k, a in zip(lo, amp)}
        assert all(gamp[i] == ref[int(glo[i])] for i in range(len(glo)))
    o = Oracle(nq, eps)
    o.import_state(lo, hi, amp)
    o.run(ops)
    assert set(int(v) for v in o.export()[0]) == keep
    # The server starts from basis states: one H makes two amplitudes
    # (1/sqrt 2, 0) whose |a|^2 is the rounded h * h; with eps exactly that
    # both survive, with the next double above it both are dropped.
    h = 0.70710678118654752440
    c = W.Circuit()
    c.h(0)
    c.gate(W.K_RX, 3, param=0.0)
    gates = sim_gates_from_ops(c.array())
    for e2, want in ((h * h, [0, 1]), (np.nextafter(h * h, 1.0), [])):
        srv = Server(1 << 26, max_slots=4)
        rid = srv.submit(sim_config(n_qubits=4, capacity=16, eps=e2), gates)
        srv.run()
        r = srv.result(rid)
        srv.close()
        s = Simulator(4, 16, e2)
        s.apply_ops(c.array())
        g = s.export()
        s.close()
        assert sorted(int(v) for v in r[0]) == sorted(int(v) for v in g[0]) == want


def test_hh_identity_prunes(sim):
    c = W.Circuit()
    c.h(3)
    c.h(3)
    g, st = check_vs_oracle(sim, W.Workload("hh", 8, 1e-20, c.array(), capacity=4))
    assert g[0].tolist() == [0] and st["pruned"] == 1


# --- random circuits, every gate kind, narrow and wide labels ---------------------
@pytest.mark.parametrize("n,seed", [(7, 1), (20, 2), (64, 3), (70, 4), (100, 5), (128, 6)])
def test_random_circuits(sim, n, seed):
    w = W.random_circuit(seed, n=n, gates=400, h_frac=0.12, ctrl_max=3, measure_frac=0.01)
    w.capacity = 1 << 20
    check_vs_oracle(sim, w)


@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_random_circuits_eps(sim, eps):
    w = W.random_circuit(77, n=12, gates=500, h_frac=0.3, ctrl_max=2)
    w.eps = eps
    w.capacity = 1 << 12
    check_vs_oracle(sim, w)


# --- scaled and full configs -------------------------------------------------------
def test_config0_full(sim):
    check_vs_oracle(sim, W.config0())


def test_config1_scaled(sim):
    check_vs_oracle(sim, W.config1(5, w=10, adds=12, n=64))


def test_config2_scaled(sim):
    check_vs_oracle(sim, W.config2(6, n=100, h_qubits=12, gates=20000, round_gates=4000, meas_per_round=4))


def test_config3_scaled(sim):
    check_vs_oracle(sim, W.config3(7, terms=80))


def _golden(name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        return json.load(f)


def _check_digest(g, doc, what=""):
    """Sorted state g against an oracle digest: entry count, SHA-256 of the
    sorted labels, every stride-th entry (labels exact, amplitudes within
    1e-12) and the norm."""
    lo, hi, amp = g
    assert len(lo) == doc["nnz"], f"{what}: nnz {len(lo)} != {doc['nnz']}"
    assert keys_digest(lo, hi) == doc["keys_sha256"], f"{what}: label sets differ"
    err = 0.0
    for k, (slo, shi, re_, im_) in enumerate(doc["samples"]):
        i = k * doc["stride"]
        assert int(lo[i]) == slo and int(hi[i]) == shi
        err = max(err, abs(amp[i] - complex(float.fromhex(re_), float.fromhex(im_))))
    assert err <= 1e-12, f"{what}: max |amp diff| {err:.3e}"
    assert abs(np.sum(np.abs(amp) ** 2) - float.fromhex(doc["norm2"])) < 1e-10
    return err


def _check_golden(S, w, doc):
    g, gout, gst = gpu_run(S, w)
    _check_digest(g, doc, w.name)
    assert list(gout) == doc["outcomes"]
    assert gst["updates"] == doc["updates"] and gst["u2_applied"] == doc["u2_applied"]
    assert gst["u2_skipped"] == doc["u2_skipped"]


def test_config1_full_golden(sim):
    _check_golden(sim, W.config1(), _golden("config1_full"))


def test_config3_full_golden(sim):
    _check_golden(sim, W.config3(), _golden("config3_full"))


def test_config2_full_first_round_samples(sim):
    """100 qubits, 2^24 entries: the first 20,000 gates of the full workload
    (every H is skipped at this size) on a seeded random state, checked on
    65,536 entries computed one at a time by the oracle."""
    w = W.config2()
    body = w.ops[24:24 + 20000]
    assert not np.any(body["kind"] == W.K_MEASURE)
    n = 1 << 24
    lo0 = np.arange(n, dtype=np.uint64)
    hi0 = np.zeros(n, np.uint64)
    amp0 = W.random_amplitudes(2024, n)
    from paper_2105_01533_amd.sim import Simulator
    s = Simulator(100, n, 1e-20)
    s.import_state(lo0, hi0, amp0)
    say("[gpu] c2 first round on 2^24 imported entries")
    _, _, st = s.apply_ops(body)
    assert st["u2_applied"] == 0 and st["u2_skipped"] == int(np.sum(body["kind"] == W.K_H))
    lo, hi, amp = s.export()
    s.close()
    assert len(lo) == n
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(n, 65536, replace=False))
    mono = body[body["kind"] != W.K_H]
    elo, ehi, eamp = monomial_samples(mono, lo0[pick], hi0[pick], amp0[pick])
    idx = lookup(lo, hi, elo, ehi)
    assert np.all(idx >= 0)
    assert np.max(np.abs(amp[idx] - eamp)) <= 1e-12
    assert sorted_unique(lo, hi)          # a permutation image: labels stay distinct


def test_config2_full_rounds_golden(sim):
    """The 100-qubit random circuit at full size against the oracle's digests
    of its first three measurement rounds (tests/golden/config2_rounds.json,
    Sec. 3.1 branching and Sec. 2.1 measurement): after each round's 20,000
    gates the 2^24-entry state (round 1: fused passes only; rounds 2 and 3:
    regrown from ~2^16 entries through single-pass branching gates on up to
    2^23-entry inputs), then after its chain of 8 measurements (the first
    decides over 2,048 blocks), with outcomes and update counters."""
    from paper_2105_01533_amd.sim import Simulator
    doc = _golden("config2_rounds")
    w = W.config2()
    assert doc["seed"] == w.meta["seed"] and doc["n_ops"] == len(w.ops)
    s = Simulator(w.n_qubits, w.capacity, w.eps)
    s.set_basis(*w.basis)
    start, upd, u2a, u2s = 0, 0, 0, 0
    for r, rd in enumerate(doc["rounds"]):
        pre, post = rd["pre_measure"], rd["post_measure"]
        say(f"[gpu] c2 round {r + 1}: ops {start}..{pre['op_end']}")
        _, _, st = s.apply_ops(w.ops[start:pre["op_end"]])
        upd, u2a, u2s = upd + st["updates"], u2a + st["u2_applied"], u2s + st["u2_skipped"]
        assert (upd, u2a, u2s) == (pre["updates"], pre["u2_applied"], pre["u2_skipped"])
        err = _check_digest(s.export(), pre, f"c2 round {r + 1} before measuring")
        say(f"[gpu] c2 round {r + 1}: {pre['nnz']} entries, max |diff| {err:.2e}; measuring")
        _, outs, st = s.apply_ops(w.ops[pre["op_end"]:post["op_end"]])
        upd += st["updates"]
        assert list(outs) == post["outcomes"] and st["measures"] == 8
        assert upd == post["updates"]
        _check_digest(s.export(), post, f"c2 round {r + 1} after measuring")
        start = post["op_end"]
    s.close()


def test_config2_full_properties(sim):
    """Full 200,000-gate workload: the normalisation restored by every
    measurement, nnz within the cap, and bitwise determinism."""
    w = W.config2()
    g1, out1, st1 = gpu_run(sim, w)
    assert len(g1[0]) <= 1 << 24 and st1["measures"] == 80
    assert abs(np.sum(np.abs(g1[2]) ** 2) - 1.0) < 1e-9
    g2, out2, st2 = gpu_run(sim, w)
    m1, m2 = st1.pop("pruned_mass"), st2.pop("pruned_mass")   # summed in no fixed order
    for k in ("index_cas", "index_probes"):                      # depend on the insert order
        st1.pop(k), st2.pop(k)
    assert list(out1) == list(out2) and st1 == st2 and abs(m1 - m2) <= 1e-12 * max(1.0, m1)
    for a, b in zip(g1, g2):
        assert a.tobytes() == b.tobytes()


# --- multi-tile, ragged sizes, imported states -------------------------------------
@pytest.mark.parametrize("n_entries", [1, 63, 64, 65, 255, 2047, 2048, 2049, 100_003, (1 << 20) + 17])
def test_ragged_sizes(sim, n_entries):
    nq = 100 if n_entries % 2 else 40
    lo0, hi0, amp0 = W.random_state(n_entries, n_entries, nq)
    rng = W.SplitMix64(n_entries)
    c = W.Circuit()
    for _ in range(300):
        W._random_mono(rng, c, nq, 0.6, 0.4, 0)
    for q in rng.distinct(nq, 3 if n_entries < 100_000 else 1):
        c.h(q)
    t, ctl = rng.distinct(nq, 2)
    c.gate(W.K_RY, t, (ctl,), param=0.3)
    for _ in range(100):
        W._random_mono(rng, c, nq, 0.6, 0.4, 0)
    c.measure(rng.randint(nq), rng.uniform())
    c.h(5, cap=4 * n_entries)
    ops = c.array()
    from paper_2105_01533_amd.sim import Simulator
    s = Simulator(nq, 16 * n_entries + 64, 1e-24)
    s.import_state(lo0, hi0, amp0)
    say(f"[gpu] ragged n={n_entries} nq={nq}")
    _, gout, gst = s.apply_ops(ops)
    g = s.export()
    s.close()
    o = Oracle(nq, 1e-24)
    o.import_state(lo0, hi0, amp0)
    oout, _ = o.run(ops)
    assert list(gout) == list(oout)
    assert_same_state(g, o.export(), what=f"ragged {n_entries}")


# --- bit-sliced fused pass ---------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(5, 11), (31, 12), (33, 13), (64, 14), (65, 15), (100, 16), (128, 17)])
def test_bitslice_random_circuits(sim, n, seed):
    """Every phase/permutation kind with up to 3 controls through the
    bit-sliced pass (forced), narrow and wide labels."""
    w = W.random_circuit(seed, n=n, gates=600, h_frac=0.02, ctrl_max=3, measure_frac=0.005)
    w.capacity = 1 << 16
    _, st = check_vs_oracle(sim, w, mono_mode=sim.SIM_MONO_BITSLICE)
    assert st["bitslice_passes"] > 0


def _x_heavy_circuit(seed, n, gates, superposed):
    """H on a few qubits, then gates dominated by uncontrolled X, mixed with
    CNOTs, Toffolis, uncontrolled and controlled phases (Z/S/T/Rz/PHASE) on
    few qubits, so X gates often meet the controls and targets of later ops."""
    rng = W.SplitMix64(seed)
    c = W.Circuit()
    for q in range(superposed):
        c.h(q)
    qs = list(range(min(n, 12)))
    for _ in range(gates):
        u = rng.uniform()
        if u < 0.45:
            c.x(qs[rng.randint(len(qs))])
        elif u < 0.65:
            a, b = rng.distinct(len(qs), 2)
            c.x(qs[b], (qs[a],))
        elif u < 0.75:
            a, b, t = rng.distinct(len(qs), 3)
            c.x(qs[t], (qs[a], qs[b]))
        else:
            kind = (W.K_Z, W.K_S, W.K_T, W.K_SDG, W.K_RZ, W.K_PHASE, W.K_Y)[rng.randint(7)]
            nc = rng.randint(3) if u > 0.9 else 0
            pick = rng.distinct(len(qs), nc + 1)
            c.gate(kind, qs[pick[-1]], tuple(qs[k] for k in pick[:-1]), param=rng.uniform() * 6.0)
    return W.Workload(f"xheavy_{n}q", n, 0.0, c.array(), capacity=1 << superposed)


@pytest.mark.parametrize("n,seed", [(12, 21), (70, 22), (128, 23)])
def test_bitslice_pending_x(sim, n, seed):
    """The run compiler carries uncontrolled X gates to the end of each
    bit-sliced run (CNOT controls toggle the target's pending X, target-bit
    phases are negated into the run constant, Toffoli and controlled-phase
    controls apply them first): long runs dense in such meetings, with the
    labels spread over both words when n > 64."""
    w = _x_heavy_circuit(seed, n, 3000, 10)
    if n > 12:   # move the register to the top qubits (across the word boundary for n = 70)
        ops = w.ops.copy()
        shift = n - 12
        ops["target"] += shift
        for r in ops:
            m = (int(r["ctrl_lo"]) | (int(r["ctrl_hi"]) << 64)) << shift
            r["ctrl_lo"], r["ctrl_hi"] = m & ((1 << 64) - 1), m >> 64
        w = W.Workload(w.name, n, w.eps, ops, w.capacity)
    g, st = check_vs_oracle(sim, w, mono_mode=sim.SIM_MONO_BITSLICE, bs_min_gates=1)
    assert st["bitslice_passes"] > 0


@pytest.mark.parametrize("n_entries", [1, 2047, 2048, 2049, 6145, 100_003])
def test_bitslice_ragged_tiles(sim, n_entries):
    nq = 100 if n_entries % 2 else 50
    lo0, hi0, amp0 = W.random_state(7 * n_entries, n_entries, nq)
    rng = W.SplitMix64(n_entries + 5)
    c = W.Circuit()
    for _ in range(400):
        W._random_mono(rng, c, nq, 0.7, 0.3, 0)
    c.gate(W.K_Y, 3, (7,))
    c.gate(W.K_PHASE, nq - 2, (2, 9), param=0.77)
    c.gate(W.K_RZ, nq - 1, (0, 1, 4), param=-2.5)
    c.gate(W.K_T, nq - 3, (0, 2, 5))
    ops = c.array()
    from paper_2105_01533_amd.sim import Simulator, SIM_MONO_BITSLICE
    s = Simulator(nq, n_entries, 0.0, mono_mode=SIM_MONO_BITSLICE)
    s.import_state(lo0, hi0, amp0)
    say(f"[gpu] bitslice ragged n={n_entries}")
    _, _, st = s.apply_ops(ops)
    g = s.export()
    s.close()
    assert st["bitslice_passes"] == 1
    o = Oracle(nq, 0.0)
    o.import_state(lo0, hi0, amp0)
    o.run(ops)
    assert_same_state(g, o.export(), what=f"bitslice ragged {n_entries}")


def test_bitslice_full_configs(sim):
    check_vs_oracle(sim, W.config0(), mono_mode=sim.SIM_MONO_BITSLICE)
    check_vs_oracle(sim, W.config1(5, w=10, adds=12, n=64), mono_mode=sim.SIM_MONO_BITSLICE)
    check_vs_oracle(sim, W.config2(6, n=100, h_qubits=12, gates=20000, round_gates=4000, meas_per_round=4),
                    mono_mode=sim.SIM_MONO_BITSLICE)
    check_vs_oracle(sim, W.config3(7, terms=80), mono_mode=sim.SIM_MONO_BITSLICE)


def test_direct_mode_full_configs(sim):
    check_vs_oracle(sim, W.config0(), mono_mode=sim.SIM_MONO_DIRECT)
    check_vs_oracle(sim, W.config2(6, n=100, h_qubits=12, gates=20000, round_gates=4000, meas_per_round=4),
                    mono_mode=sim.SIM_MONO_DIRECT)


# --- launch-shape independence and determinism --------------------------------------
def test_tuning_knobs_do_not_change_results(sim):
    """Launch shapes and index load factor leave results bitwise unchanged for
    a given fused-pass kernel; switching kernels changes rounding only."""
    w = W.config2(31, n=100, h_qubits=11, gates=6000, round_gates=2000, meas_per_round=3)
    for mode in (sim.SIM_MONO_DIRECT, sim.SIM_MONO_BITSLICE):
        ref, _, _ = gpu_run(sim, w, mono_mode=mode)
        knobs = [dict(block=64), dict(block=128), dict(load_factor=0.25), dict(load_factor=0.9)]
        if mode == sim.SIM_MONO_DIRECT:
            knobs.append(dict(fuse_max=7))       # per-entry products: run boundaries do not matter
        for kw in knobs:
            g, _, _ = gpu_run(sim, w, mono_mode=mode, **kw)
            for a, b in zip(ref, g):
                assert a.tobytes() == b.tobytes(), (mode, kw)
    d, _, _ = gpu_run(sim, w, mono_mode=sim.SIM_MONO_DIRECT, fuse_max=1)
    b, _, _ = gpu_run(sim, w, mono_mode=sim.SIM_MONO_BITSLICE)
    assert_same_state(d, b, what="direct vs bit-sliced")


def test_profiling_modes(sim):
    """SIM_PROFILE_MONO times the fused passes only, SIM_PROFILE_ALL every
    kernel class; host classes are always timed; other modes are rejected."""
    w = W.config2(32, n=100, h_qubits=10, gates=3000, round_gates=1000, meas_per_round=2)
    s = sim.Simulator(w.n_qubits, w.capacity, w.eps)
    g = sim.sim_gates_from_ops(w.ops)
    try:
        for mode, timed in ((sim.SIM_PROFILE_MONO, {"mono_pass"}), (sim.SIM_PROFILE_ALL, None)):
            sim.sim_set_profiling(s.h, mode)
            sim.sim_kernel_stats_reset(s.h)
            s.set_basis(*w.basis)
            s.apply_gates(g)
            ks = sim.sim_kernel_stats(s.h)
            for k, v in ks.items():
                if k.startswith("host_") or v["launches"] == 0:
                    continue
                if timed is None or k in timed:
                    assert v["total_ms"] > 0, (mode, k)
                else:
                    assert v["total_ms"] == 0, (mode, k)
            assert ks["host_prepare"]["launches"] >= 1 and ks["host_prepare"]["total_ms"] > 0
        with pytest.raises(sim.SimError):
            sim.sim_set_profiling(s.h, 3)
    finally:
        s.close()


@pytest.mark.parametrize("which", ["c0", "c2_small", "c2_wide_ctrl"])
def test_u2_single_pass_matches_two_pass(sim, which):
    """Branching gates whose outputs fit run as one pass (evaluation, chained
    scan over 2048-entry tiles, ordered write), or, on states of at most 8192
    entries, as one block with the partner index in LDS; the state is bitwise
    the one the separate count, scan and write passes produce, in the same
    order, and the one the global index gives for every size."""
    if which == "c0":
        w = W.config0(seed=W.seed_for(0, 3))
    elif which == "c2_small":
        w = W.config2(41, n=100, h_qubits=14, gates=8000, round_gates=2000, meas_per_round=3)
    else:
        w = W.config2(43, n=128, h_qubits=12, gates=6000, round_gates=3000, meas_per_round=2)
    out = []
    for flags in (0, sim.SIM_FLAG_U2_TWO_PASS, sim.SIM_FLAG_U2_GLOBAL_INDEX):
        s = sim.Simulator(w.n_qubits, w.capacity, w.eps, flags=flags)
        try:
            s.set_basis(*w.basis)
            sim.sim_kernel_stats_reset(s.h)
            _, outs, st = s.apply_ops(w.ops)
            ks = sim.sim_kernel_stats(s.h)
            out.append((s.export(sort=False), list(outs), st, ks))
        finally:
            s.close()
    (a, oa, sa, ka), (b, ob, sb, kb), (c, oc, sc, kc) = out
    for other, oo, so in ((b, ob, sb), (c, oc, sc)):
        for x, y in zip(a, other):
            assert x.tobytes() == y.tobytes()
        assert oa == oo
        for k in ("u2_applied", "u2_skipped", "pruned", "peak_nnz", "updates"):
            assert sa[k] == so[k], k
    # default: small states in the one-block LDS-index kernel, the rest in
    # the single pass; global index: every gate in the single pass
    assert ka["u2_lds"]["launches"] > 0 and kb["u2_lds"]["launches"] == kc["u2_lds"]["launches"] == 0
    assert ka["u2_write"]["launches"] + ka["u2_lds"]["launches"] == sa["u2_applied"]
    assert kb["u2_write"]["launches"] == kc["u2_write"]["launches"] == sa["u2_applied"]
    assert kb["u2_count"]["launches"] == sa["u2_applied"]
    assert ka["u2_count"]["launches"] < sa["u2_applied"]       # most ran as one pass
    assert kc["u2_count"]["launches"] < sa["u2_applied"]
    assert ka["u2_write"]["alg_bytes"] + ka["u2_lds"]["alg_bytes"] == kb["u2_write"]["alg_bytes"]
    assert kc["u2_write"]["alg_bytes"] == kb["u2_write"]["alg_bytes"]


def test_index_reuse_across_forms_and_sizes(sim):
    """The hash index is emptied by the single-pass kernel for the next gate
    and by a clearing launch only where that cannot be known (after the
    two-pass form, or beyond what the last gate used).  Alternating forms and
    state sizes on one handle, every result matches the oracle."""
    n = 80
    s = sim.Simulator(n, 1 << 21, 0.0)
    try:
        for step, (entries, two_pass) in enumerate([(60_000, True), (3_000, False), (50_000, False),
                                                     (500, True), (40_000, False), (70_000, False)]):
            lo, hi, amp = W.random_state(1500 + step, entries, n)
            c = W.Circuit()
            for q in (3, 40, 70, 5):
                c.h(q, ctrls=(11,) if q == 40 else ())
            sim.sim_set_tuning(s.h, flags=sim.SIM_FLAG_U2_TWO_PASS if two_pass else 0)
            s.import_state(lo, hi, amp)
            s.apply_ops(c.array())
            o = Oracle(n, 0.0)
            o.import_state(lo, hi, amp)
            o.run(c.array())
            assert_same_state(s.export(), o.export(), what=f"step {step}")
    finally:
        s.close()


@pytest.mark.parametrize("n,two_pass", [(20, False), (70, False), (70, True)])
def test_pass_byte_counters(sim, n, two_pass):
    """Algorithmic bytes per pass class on a circuit whose entry counts are
    known: three Hadamards take 1 -> 2 -> 4 -> 8 entries, then a measurement
    with a forced outcome keeps 4 of 8.  The count pass exists only in the
    two-pass form of branching gates."""
    c = W.Circuit()
    for q in (0, 1, n - 1):
        c.h(q)
    c.measure(1, 0.5, forced=0)
    s = sim.Simulator(n, 1 << 10, 0.0, flags=sim.SIM_FLAG_U2_TWO_PASS if two_pass else 0)
    try:
        sim.sim_kernel_stats_reset(s.h)
        s.apply_ops(c.array())
        ks = sim.sim_kernel_stats(s.h)
    finally:
        s.close()
    eb = 32 if n > 64 else 24
    assert ks["u2_count"]["alg_bytes"] == ((1 + 2 + 4) * eb if two_pass else 0)
    # small states: the one-block LDS-index kernel unless in the two-pass form
    u2 = ((1 + 2) + (2 + 4) + (4 + 8)) * eb
    assert ks["u2_write"]["alg_bytes"] == (u2 if two_pass else 0)
    assert ks["u2_lds"]["alg_bytes"] == (0 if two_pass else u2)
    assert ks["measure_reduce"]["alg_bytes"] == 8 * 24
    assert ks["measure_write"]["alg_bytes"] == 8 * 8 + 4 * (2 * eb - 8)
    assert ks["block_scan"]["alg_bytes"] == 0 and ks["index_build"]["alg_bytes"] == 0


@pytest.mark.parametrize("n,qs", [(20, [3, 0, 19, 7, 11, 5, 16, 2]),
                                  (100, [3, 70, 64, 63, 99, 10, 80, 0])])
def test_measurement_chain(sim, n, qs):
    """Consecutive measurements: after the first, each takes its sums from the
    previous measurement's write (one reduce pass per chain).  Outcomes and
    the state match the oracle, and match the same measurements made one at a
    time; the chain crosses the 64-bit word boundary and holds a forced
    outcome."""
    lo, hi, amp = W.random_state(1201 + n, 50_000, n)
    rng = W.SplitMix64(1301 + n)
    c = W.Circuit()
    for k, q in enumerate(qs):
        c.measure(q, rng.uniform(), forced=1 if k == 4 else -1)
    ops = c.array()
    s = sim.Simulator(n, 1 << 17, 0.0)
    try:
        s.import_state(lo, hi, amp)
        sim.sim_kernel_stats_reset(s.h)
        _, outs, st = s.apply_ops(ops)
        ks = sim.sim_kernel_stats(s.h)
        g = s.export()
        s.import_state(lo, hi, amp)
        one = [s.measure(int(r["target"]), float(r["param"]), int(r["forced"]))[0] for r in ops]
        g1 = s.export()
    finally:
        s.close()
    assert ks["measure_reduce"]["launches"] == 1 and ks["measure_write"]["launches"] == len(qs)
    o = Oracle(n, 0.0)
    o.import_state(lo, hi, amp)
    oouts, _ = o.run(ops)
    assert list(outs) == list(oouts) == one
    assert_same_state(g, o.export(), what=f"chain n={n}")
    assert_same_state(g, g1, 1e-14, what="chained vs one at a time")
    assert st["measures"] == len(qs)


def test_measurement_chain_zero_probability(sim):
    """A forced outcome of probability zero inside a chain stops the list
    there; the state is the one after the measurements before it."""
    n = 100
    lo, hi, amp = W.random_state(1401, 20_000, n)
    c = W.Circuit()
    c.measure(3, 0.5, forced=0)
    c.measure(70, 0.25)
    c.measure(3, 0.5, forced=1)
    c.measure(5, 0.5)
    s = sim.Simulator(n, 1 << 16, 0.0)
    try:
        s.import_state(lo, hi, amp)
        rc, outs, st = s.apply_ops(c.array(), raise_on_error=False)
        g = s.export()
        # the failed outcome leaves no error behind for the next call
        c2 = W.Circuit()
        c2.measure(5, 0.5)
        rc2, _, _ = s.apply_ops(c2.array(), raise_on_error=False)
    finally:
        s.close()
    assert rc == sim.SIM_E_STATE and st["measures"] == 2 and rc2 == sim.SIM_OK
    o = Oracle(n, 0.0)
    o.import_state(lo, hi, amp)
    oouts, _ = o.run(c.array()[:2])
    assert list(outs[:2]) == list(oouts)
    assert_same_state(g, o.export(), what="chain stopped")


# --- gate commuting (Sec. 3.3) ---------------------------------------------------------
def check_commuting(S, w, tol=1e-12, **kw):
    """GPU run of sim_commute_ops' output vs the oracle's commuting runner."""
    g, gout, gst = gpu_run(S, w, commute=True, **kw)
    o = Oracle(w.n_qubits, w.eps)
    o.set_basis(*w.basis)
    oout, _ = o.run_commuting(w.ops)
    assert list(gout) == list(oout), "measurement outcomes differ"
    assert_same_state(g, o.export(), tol, w.name + " (commuting)")
    t = o.totals()
    assert gst["u2_applied"] == t["u2_applied"] and gst["u2_skipped"] == t["u2_skipped"]
    return g, gst


def test_commuting_fig1(sim):
    from test_commute_oracle import fig1_circuit
    check_commuting(sim, W.Workload("fig1", 8, 0.0, fig1_circuit().array(), capacity=1 << 8))


@pytest.mark.parametrize("n,seed", [(9, 0), (9, 1), (40, 2), (100, 3), (128, 4)])
def test_commuting_random(sim, n, seed):
    wide = n > 16
    w = W.random_circuit(700 + seed, n=n, gates=250 if wide else 800, h_frac=0.2 if wide else 0.45, ctrl_max=3,
                         measure_frac=0.02)
    w.eps = 1e-14
    w.capacity = 1 << 20
    check_commuting(sim, w)
    check_commuting(sim, w, mono_mode=sim.SIM_MONO_DIRECT)


def test_commuting_phase_oracle_blocks(sim):
    w = W.phase_oracle_blocks(7, n=100, superposed=10, blocks=400)
    check_vs_oracle(sim, w)
    g, st = check_commuting(sim, w)
    assert st["u2_applied"] <= 10 + 2   # the blocks' H pairs never reach the state


def test_commuting_trotter_and_adder(sim):
    for w in (W.config3(9, terms=18), W.config1(4, w=8, adds=6, n=32)):
        check_commuting(sim, w)


# --- errors and edge cases ------------------------------------------------------------
def test_capacity_error_leaves_state(sim):
    from paper_2105_01533_amd.sim import Simulator, SIM_E_CAPACITY
    s = Simulator(30, 16, 0.0)
    c = W.Circuit()
    for q in range(4):
        c.h(q)                      # 16 entries: fits
    c.x(9, (1,))
    c.h(5)                          # would need 32
    c.h(6)
    s.apply_ops(c.array()[:5])
    before = s.export()
    rc, _, st = s.apply_ops(c.array()[5:], raise_on_error=False)
    assert rc == SIM_E_CAPACITY and st["gates_applied"] == 0
    # The rejected gate changes no counter: its count pass ran, but the scan
    # commits the staged counters only for outputs that fit.
    assert st["updates"] == 0 and st["pruned"] == 0 and st["peak_nnz"] == 16
    after = s.export()
    for a, b in zip(before, after):
        assert a.tobytes() == b.tobytes()
    s.close()


def test_invalid_ops_apply_nothing(sim):
    from paper_2105_01533_amd.sim import Simulator, SimError, SIM_E_ARG
    s = Simulator(10, 64, 0.0)
    s.apply_ops(W.config0(1, n=10, h_qubits=3, gates=50, cap=64, measured=0).ops)
    before = s.export()
    for bad in [dict(target=10), dict(target=3, ctrl=(3,)), dict(target=1, ctrl=(12,))]:
        c = W.Circuit()
        c.x(0)
        c.gate(W.K_X, bad["target"], bad.get("ctrl", ()))
        with pytest.raises(SimError) as e:
            s.apply_ops(c.array())
        assert e.value.code == SIM_E_ARG
    c = W.Circuit()
    c.measure(2, 1.5)
    with pytest.raises(SimError):
        s.apply_ops(c.array())
    after = s.export()
    for a, b in zip(before, after):
        assert a.tobytes() == b.tobytes()
    s.close()


def test_forced_zero_probability_measurement(sim):
    from paper_2105_01533_amd.sim import Simulator, SimError, SIM_E_STATE
    s = Simulator(5, 8, 0.0)
    c = W.Circuit()
    c.h(0)
    s.apply_ops(c.array())
    m = W.Circuit()
    m.measure(1, 0.0, forced=1)      # qubit 1 is 0 everywhere
    rc, _, _ = s.apply_ops(m.array(), raise_on_error=False)
    assert rc == SIM_E_STATE
    assert s.nnz == 2
    o, p1 = s.measure(0, 0.0, forced=1)
    assert o == 1 and abs(p1 - 0.5) < 1e-15
    lo, hi, amp = s.export()
    assert lo.tolist() == [1] and abs(amp[0] - 1) < 1e-15
    s.close()


def test_everything_pruned_then_measure(sim):
    from paper_2105_01533_amd.sim import Simulator, SIM_E_STATE
    s = Simulator(6, 8, 10.0)        # eps above any |a|^2: a branching gate empties the state
    c = W.Circuit()
    c.h(0)
    s.apply_ops(c.array())
    assert s.nnz == 0
    m = W.Circuit()
    m.measure(0, 0.3)
    rc, _, _ = s.apply_ops(m.array(), raise_on_error=False)
    assert rc == SIM_E_STATE and s.nnz == 0
    s.close()


def test_import_export_roundtrip_and_errors(sim):
    from paper_2105_01533_amd.sim import Simulator, SimError, SIM_E_ARG, SIM_E_CAPACITY
    lo, hi, amp = W.random_state(3, 5000, 128)
    s = Simulator(128, 5000, 0.0)
    s.import_state(lo, hi, amp)
    glo, ghi, gamp = s.export()
    order = np.lexsort((lo, hi))
    assert np.array_equal(glo, lo[order]) and np.array_equal(ghi, hi[order])
    assert gamp.tobytes() == amp[order].tobytes()
    with pytest.raises(SimError) as e:
        s.import_state(np.array([1, 1], np.uint64), np.zeros(2, np.uint64), np.ones(2))
    assert e.value.code == SIM_E_ARG
    with pytest.raises(SimError) as e:
        s.import_state(*W.random_state(4, 5001, 128))
    assert e.value.code == SIM_E_CAPACITY
    s.close()
    s = Simulator(10, 4, 0.0)
    with pytest.raises(SimError) as e:
        s.import_state(np.array([1 << 10], np.uint64), np.zeros(1, np.uint64), np.ones(1))
    assert e.value.code == SIM_E_ARG
    s.close()


def test_empty_and_single_entry(sim):
    from paper_2105_01533_amd.sim import Simulator
    s = Simulator(8, 4, 0.0)
    s.import_state(np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0))
    _, _, st = s.apply_ops(W.config0(2, n=8, h_qubits=0, gates=200, cap=4, measured=0).ops)
    assert s.nnz == 0 and st["updates"] == 0
    s.set_basis(5, 0)
    c = W.Circuit()
    c.x(0)
    c.gate(W.K_S, 2)
    s.apply_ops(c.array())
    lo, hi, amp = s.export()
    assert lo.tolist() == [4] and amp[0] == 1j
    s.close()


# Requests of the 512-request serving trace (seed 4242) whose states reach
# 2^19..2^22 entries on 22, 40 and 51 qubits.
@pytest.mark.parametrize("req", [197, 136, 422])
def test_regplane_reproducible_on_large_states(sim, req):
    """Two register-plane runs and one LDS-plane run of the same circuit give
    the same keys, bit-identical amplitudes and the same outcomes; the
    batched server agrees to 1e-12.  (States of this size and width were not
    reproducible when the register-plane pass ran three waves per SIMD.)"""
    w = W.serving_request(req)
    say(f"[gpu] serving request {req}: n={w.n_qubits} cap={w.capacity} ops={len(w.ops)}")
    gates = sim.sim_gates_from_ops(w.ops)

    def plain(**kw):
        s = sim.Simulator(w.n_qubits, w.capacity, w.eps, tuned=False, **kw)   # register planes unless kw
        s.set_basis(*w.basis)
        _, outs, st = s.apply_gates(gates)
        out = s.export()
        s.close()
        assert st["bitslice_passes"] > 0
        return out, list(outs)

    (a, oa), (b, ob), (c, oc) = plain(), plain(), plain(flags=sim.SIM_FLAG_BS_LDS)
    assert oa == ob == oc
    for x in (b, c):
        assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1]), "keys differ"
        assert a[2].tobytes() == x[2].tobytes(), "amplitudes differ"
    srv = sim.Server(8 << 30, max_slots=2, lane_capacity=sim.SRV_LANE_OFF)   # the batched kernels
    rid = srv.submit(sim.sim_config(n_qubits=w.n_qubits, capacity=w.capacity, eps=w.eps), gates, w.basis)
    srv.run()
    lo, hi, amp, outs, _ = srv.result(rid)
    srv.close()
    assert list(outs) == oa
    assert np.array_equal(lo, a[0]) and np.array_equal(hi, a[1])
    assert float(np.max(np.abs(amp - a[2]))) <= 1e-12


def test_regplane_passes_on_two_streams(sim):
    """Two states of 2^21 entries (adder circuits of the serving trace, their
    controlled-phase ladders in register-plane turn groups) simulated at the
    same time from two host threads, each on its own stream: every result is
    bit-identical to the same circuit run alone."""
    import threading
    import torch

    ws = [W.serving_request(i) for i in (137, 130)]
    gates = [sim.sim_gates_from_ops(w.ops) for w in ws]

    def run(w, g, stream=None):
        with torch.cuda.stream(stream or torch.cuda.current_stream()):
            s = sim.Simulator(w.n_qubits, w.capacity, w.eps, tuned=False)   # register planes
            s.set_basis(*w.basis)
            _, _, st = s.apply_gates(g)
            out = s.export()
            s.close()
        assert st["bitslice_passes"] > 0
        return out

    alone = [run(w, g) for w, g in zip(ws, gates)]
    for rep in range(3):
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        got = [None, None]

        def worker(k):
            got[k] = run(ws[k], gates[k], streams[k])

        ts = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        torch.cuda.synchronize()
        for k in range(2):
            say(f"[gpu] two streams rep {rep} state {k}: {len(got[k][0])} entries")
            assert np.array_equal(got[k][0], alone[k][0]) and np.array_equal(got[k][1], alone[k][1])
            assert got[k][2].tobytes() == alone[k][2].tobytes()


# --- key exactness: how far prune decisions are from flipping ---------------------
@pytest.mark.parametrize("which", ["c0", "c3_80"])
def test_prune_decisions_have_margin(sim, which):
    """The surviving labels are decided by |a|^2 < eps after each branching
    gate.  The fused passes round differently from the oracle's gate-by-gate
    products (the per-entry pass multiplies each gate's factor; the bit-sliced
    passes sum exact turn fractions and take one sincospi), so a decision
    could flip if some |a|^2 came within that rounding of eps.  The oracle
    records the smallest | |a|^2 - eps | / eps over every entry T_eps examined;
    it must exceed, by a factor of 1000, twice the largest relative amplitude
    difference between the per-entry and the register-plane runs (the measured
    rounding gap), and both runs must keep exactly the oracle's labels."""
    w = W.config0() if which == "c0" else W.config3(7, terms=80)
    o, oout, _ = oracle_run(w)
    margin = o.totals()["min_margin"]
    olo, ohi, _ = o.export()
    runs = {}
    for name, kw in (("per_entry", {"mono_mode": sim.SIM_MONO_DIRECT}), ("register_plane", {"mono_mode": 0})):
        s = sim.Simulator(w.n_qubits, w.capacity, w.eps, tuned=False, bs_min_gates=4, **kw)
        s.set_basis(*w.basis)
        _, outs, st = s.apply_ops(w.ops)
        runs[name] = s.export()
        s.close()
        assert list(outs) == list(oout), name
        assert np.array_equal(runs[name][0], olo) and np.array_equal(runs[name][1], ohi), name
    a, b = runs["per_entry"][2], runs["register_plane"][2]
    gap = float(np.max(np.abs(a - b) / np.maximum(np.abs(a), 1e-300)))
    say(f"[gpu] {w.name}: min prune margin {margin:.3e}, kernel rounding gap (relative) {gap:.3e}")
    assert math.isfinite(margin) and margin > 1e3 * 2 * max(gap, 1e-16), (margin, gap)


@pytest.mark.parametrize("n_qubits", [40, 100])
def test_export_records_and_arrays_round_trip(sim, n_qubits):
    """An imported state comes back in storage order, identically, through
    both export calls: records (sim_export_state) and separate arrays
    (sim_export_state_soa).  The size spans three staging chunks and a ragged
    tail for both label widths."""
    import ctypes

    S = sim
    n = 3 * 524_288 + 17
    say(f"[gpu] export round trip: {n_qubits} qubits, {n} entries")
    rng = np.random.default_rng(11 + n_qubits)
    idx = rng.permutation(1 << 21)[:n].astype(np.uint64)          # unique low bits
    if n_qubits <= 64:
        lo = idx | (rng.integers(0, 1 << 19, n, dtype=np.uint64) << np.uint64(21))
        hi = np.zeros(n, np.uint64)
    else:
        lo = idx | (rng.integers(0, 1 << 43, n, dtype=np.uint64) << np.uint64(21))
        hi = rng.integers(0, 1 << (n_qubits - 64), n, dtype=np.uint64)
    amp = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    s = S.Simulator(n_qubits, 1 << 22, 0.0)
    s.import_state(lo, hi, amp)
    a_lo, a_hi, a_amp = s.export(sort=False)
    assert np.array_equal(a_lo, lo) and np.array_equal(a_hi, hi)
    assert a_amp.tobytes() == amp.tobytes()
    keys = np.empty(n, S.KEY_DTYPE)
    amps = np.empty(n, np.complex128)
    got = ctypes.c_uint64()
    assert S._lib.sim_export_state(s.h, S._ptr(keys), S._ptr(amps), n, ctypes.byref(got)) == 0
    assert got.value == n
    assert np.array_equal(keys["lo"], lo) and np.array_equal(keys["hi"], hi)
    assert amps.tobytes() == amp.tobytes()
    # a buffer one entry short is refused, nothing written
    short = np.zeros(n - 1, np.uint64)
    assert S._lib.sim_export_state_soa(s.h, S._ptr(short), None, S._ptr(amps), n - 1, ctypes.byref(got)) == S.SIM_E_BUFFER
    assert got.value == n and not short.any()
    s.close()


def _paired_state(seed, size, n, t):
    """size distinct labels on n qubits where about a third of the entries
    have their partner (label ^ 2^t) present: P pairs and size - 2P singles."""
    rng = np.random.default_rng(seed)
    P = size // 3
    K = size - P
    seen, base = set(), []
    while len(base) < K:
        lo = int(rng.integers(0, 1 << min(n, 63))) | (int(rng.integers(0, 2)) << 63 if n > 63 else 0)
        hi = int(rng.integers(0, 1 << (n - 64))) if n > 64 else 0
        if t < 64:
            lo &= ~(1 << t)
        else:
            hi &= ~(1 << (t - 64))
        if (lo, hi) not in seen:
            seen.add((lo, hi))
            base.append((lo, hi))
    flip = (1 << t) if t < 64 else 0, (1 << (t - 64)) if t >= 64 else 0
    labels = []
    for k, (lo, hi) in enumerate(base):
        if k < P:
            labels += [(lo, hi), (lo ^ flip[0], hi ^ flip[1])]
        elif rng.integers(0, 2):
            labels.append((lo ^ flip[0], hi ^ flip[1]))
        else:
            labels.append((lo, hi))
    order = rng.permutation(len(labels))
    lo = np.array([labels[i][0] for i in order], np.uint64)
    hi = np.array([labels[i][1] for i in order], np.uint64)
    amp = rng.uniform(-1, 1, size) + 1j * rng.uniform(-1, 1, size)
    return lo, hi, amp / np.linalg.norm(amp)


@pytest.mark.parametrize("n", [30, 100])
@pytest.mark.parametrize("size", [1, 3, 4096, 8191, 8192, 8193])
def test_u2_lds_kernel_around_its_limit(sim, n, size):
    """Branching gates on imported states at and around the one-block
    kernel's limit (8192 entries): a controlled Ry, an H on the same target
    and an H on a high qubit (a third of the entries have their partner
    present).  Against the oracle, and bit for bit against the global-index
    path; the one-block kernel runs exactly when the state has at most 8192
    entries."""
    t = 5 if n <= 64 else 70
    lo, hi, amp = _paired_state(9000 + size + n, size, n, t)
    c = W.Circuit()
    c.gate(W.K_RY, t, controls=(n - 2,), param=0.7)
    c.h(t)
    c.h(n - 1)
    ops = c.array()
    res = []
    for flags in (0, sim.SIM_FLAG_U2_GLOBAL_INDEX):
        s = sim.Simulator(n, 1 << 16, 1e-30, flags=flags)
        try:
            s.import_state(lo, hi, amp)
            sim.sim_kernel_stats_reset(s.h)
            _, _, st = s.apply_ops(ops)
            ks = sim.sim_kernel_stats(s.h)
            res.append((s.export(sort=False), st, ks))
        finally:
            s.close()
    (a, sa, ka), (b, sb, kb) = res
    for x, y in zip(a, b):
        assert x.tobytes() == y.tobytes()
    for k in ("u2_applied", "pruned", "peak_nnz", "updates"):
        assert sa[k] == sb[k], k
    # The engine's bound on the entry count before the three gates is size,
    # 2 size and 4 size (the import's count is exact; a branching gate at
    # most doubles it); the one-block kernel runs where that bound is <= 8192.
    assert sa["u2_applied"] == 3
    assert ka["u2_lds"]["launches"] == sum(ub <= 8192 for ub in (size, 2 * size, 4 * size))
    assert kb["u2_lds"]["launches"] == 0
    o = Oracle(n, 1e-30)
    o.import_state(lo, hi, amp)
    o.run(ops)
    order = np.lexsort((a[0], a[1]))
    assert_same_state(tuple(x[order] for x in a), o.export(), 1e-12, f"lds {n} {size}")
    t_ = o.totals()
    assert sa["updates"] == t_["updates"] and sa["pruned"] == t_["pruned"]


@pytest.mark.parametrize("n", [30, 100])
@pytest.mark.parametrize("size", [3000, 50_000])
def test_index_counters(sim, n, size):
    """Partner-index counters (SIM_FLAG_COUNT_INDEX) of one controlled
    branching gate on an imported state: inserts are the entries under the
    control with the pivot bit clear
    and look-ups those with it set (exact, for the one-block LDS index at 3000
    entries and the global index at 50,000); CAS attempts and probes are at
    least one per insert and per look-up, and at load factor <= 1/2 stay
    close to one."""
    t, ctl = (5, n - 2)
    lo, hi, amp = _paired_state(7000 + size + n, size, n, t)
    c = W.Circuit()
    c.gate(W.K_RY, t, controls=(ctl,), param=0.4)
    for flags in (sim.SIM_FLAG_COUNT_INDEX, sim.SIM_FLAG_U2_GLOBAL_INDEX | sim.SIM_FLAG_COUNT_INDEX):
        s = sim.Simulator(n, 1 << 17, 0.0, flags=flags)
        try:
            s.import_state(lo, hi, amp)
            _, _, st = s.apply_ops(c.array())
        finally:
            s.close()
        cw = hi if ctl >= 64 else lo
        under = ((cw >> np.uint64(ctl & 63)) & np.uint64(1)).astype(bool)
        piv = ((lo >> np.uint64(t)) & np.uint64(1)).astype(bool)
        assert st["index_inserts"] == int(np.sum(under & ~piv)), flags
        assert st["index_lookups"] == int(np.sum(under & piv)), flags
        assert st["index_inserts"] <= st["index_cas"] <= 2 * st["index_inserts"] + 64
        assert st["index_lookups"] <= st["index_probes"] <= 3 * st["index_lookups"] + 64
        say(f"[gpu] index counters n={n} size={size} flags={flags}: {st['index_cas'] / max(st['index_inserts'], 1):.3f} "
            f"CAS/insert, {st['index_probes'] / max(st['index_lookups'], 1):.3f} probes/look-up")


def test_index_counting_is_opt_in_for_the_global_index(sim):
    """Without SIM_FLAG_COUNT_INDEX the global index counts nothing (its
    kernels do no counter atomics); the result is the same either way."""
    lo, hi, amp = _paired_state(7777, 50_000, 40, 5)
    c = W.Circuit()
    c.h(5)
    out = []
    for flags in (0, sim.SIM_FLAG_COUNT_INDEX):
        s = sim.Simulator(40, 1 << 17, 0.0, flags=flags)
        try:
            s.import_state(lo, hi, amp)
            _, _, st = s.apply_ops(c.array())
            out.append((s.export(sort=False), st))
        finally:
            s.close()
    (a, sa), (b, sb) = out
    for x, y in zip(a, b):
        assert x.tobytes() == y.tobytes()
    assert sa["index_inserts"] == sa["index_lookups"] == sa["index_cas"] == sa["index_probes"] == 0
    assert sb["index_inserts"] > 0 and sb["index_lookups"] > 0


@pytest.mark.parametrize("size", [300_001, 2_000_003, 8_388_700])
def test_u2_single_pass_tile_sizes(sim, size):
    """The single-pass branching kernel takes 512-, 1024- or 2048-entry tiles
    by state size (these three sizes select one each); a controlled H and an
    H on imported states give bitwise the two-pass form's state, in the same
    order (the two-pass form is compared with the oracle elsewhere)."""
    n = 100
    k = np.arange(size, dtype=np.uint64)
    lo = k * np.uint64(0x9E3779B97F4A7C15)            # distinct (odd multiplier)
    rng = np.random.default_rng(size)
    hi = rng.integers(0, 1 << 36, size, dtype=np.uint64)
    amp = rng.uniform(-1, 1, size) + 1j * rng.uniform(-1, 1, size)
    amp /= np.linalg.norm(amp)
    c = W.Circuit()
    c.h(7, ctrls=(80,))
    c.h(70)
    say(f"[gpu] single-pass tiles: {size} entries")
    out = []
    for flags in (0, sim.SIM_FLAG_U2_TWO_PASS):
        s = sim.Simulator(n, 1 << 25, 0.0, flags=flags)
        try:
            s.import_state(lo, hi, amp)
            _, _, st = s.apply_ops(c.array())
            out.append((s.export(sort=False), st))
        finally:
            s.close()
    (a, sa), (b, sb) = out
    assert sa["u2_applied"] == sb["u2_applied"] == 2
    for x, y in zip(a, b):
        assert x.tobytes() == y.tobytes()


@pytest.mark.parametrize("case", ["handmade", "c0", "c1_small", "random_meas", "c3_small"])
def test_uniform_qubit_splits_match_index_path(sim, case):
    """Branching gates whose partner mask meets a qubit that is the same in
    every entry run without an index; the state, outcomes and counters are
    bitwise those of the index path (SIM_FLAG_NO_UNIFORM), and such gates do
    occur."""
    if case == "handmade":
        c = W.Circuit()
        for q in range(6):
            c.h(q)
        c.gate(W.K_X, 10, controls=(2,))
        c.h(10)
        c.h(11)
        c.measure(3, 0.4)
        c.h(3)
        c.gate(W.K_X, 20, controls=(30, 31))
        c.h(20)
        c.gate(W.K_RY, 12, controls=(0,), param=0.9)
        c.h(0)
        w = W.Workload("handmade", 40, 0.0, c.array(), 1 << 12)
    elif case == "c0":
        w = W.config0(seed=W.seed_for(0, 1))
    elif case == "c1_small":
        w = W.config1(71, w=10, adds=4, n=32)
    elif case == "random_meas":
        w = W.random_circuit(72, n=12, gates=600, h_frac=0.25, ctrl_max=3, measure_frac=0.03)
        w.capacity = 1 << 12
    else:
        w = W.config3(73, terms=20)
    out = []
    for flags in (0, sim.SIM_FLAG_NO_UNIFORM):
        s, outs, st = sim.run_workload(w, flags=flags)
        out.append((s.export(sort=False), list(outs), st))
        s.close()
    (a, oa, sa), (b, ob, sb) = out
    for x, y in zip(a, b):
        assert x.tobytes() == y.tobytes(), case
    assert oa == ob
    for k in ("u2_applied", "u2_skipped", "pruned", "updates", "peak_nnz", "measures"):
        assert sa[k] == sb[k], k
    assert sa["u2_split"] > 0 and sb["u2_split"] == 0
    o, oout, _ = oracle_run(w)
    assert list(oa) == list(oout)
    order = np.lexsort((a[0], a[1]))
    assert_same_state(tuple(x[order] for x in a), o.export(), 1e-12, case)


@pytest.mark.parametrize("n,seed,eps", [(9, 81, 0.0), (30, 82, 1e-9), (64, 83, 0.0), (65, 84, 1e-9),
                                        (100, 85, 0.0), (128, 86, 1e-9)])
def test_engine_flags_leave_results_unchanged(sim, n, seed, eps):
    """Every engine flag that only changes how a result is computed -- the
    separate count/scan/write passes, the global partner index for small
    states, the index for gates a uniform qubit splits, LDS planes instead of
    register planes -- gives the default's state, outcomes and counters bit
    for bit on random circuits of every gate kind with measurements; the
    default matches the oracle."""
    w = W.random_circuit(seed, n=n, gates=700, h_frac=0.15, ctrl_max=3, measure_frac=0.02, cap=1 << 15)
    w.capacity = 1 << 15
    w.eps = eps
    variants = [sim.SIM_FLAG_U2_TWO_PASS, sim.SIM_FLAG_U2_GLOBAL_INDEX, sim.SIM_FLAG_NO_UNIFORM,
                sim.SIM_FLAG_BS_LDS,
                sim.SIM_FLAG_U2_TWO_PASS | sim.SIM_FLAG_NO_UNIFORM | sim.SIM_FLAG_BS_LDS,
                sim.SIM_FLAG_U2_GLOBAL_INDEX | sim.SIM_FLAG_NO_UNIFORM]
    keys = ("u2_applied", "u2_skipped", "pruned", "updates", "peak_nnz", "measures")
    out = []
    for flags in [0] + variants:
        s, outs, st = sim.run_workload(w, flags=flags)
        out.append((s.export(sort=False), list(outs), st))
        s.close()
    a, oa, sa = out[0]
    for flags, (b, ob, sb) in zip(variants, out[1:]):
        for x, y in zip(a, b):
            assert x.tobytes() == y.tobytes(), flags
        assert oa == ob, flags
        for k in keys:
            assert sa[k] == sb[k], (flags, k)
    o, oout, _ = oracle_run(w)
    assert oa == list(oout)
    order = np.lexsort((a[0], a[1]))
    assert_same_state(tuple(x[order] for x in a), o.export(), 1e-12, w.name)


def _wrap_circuit(n, rounds, seed):
    """Branching gates cycling over 12 qubits in superposition (states of
    2^10..2^12 entries), with controlled ones, CNOTs and a few measurements:
    hundreds of gates that use the partner index."""
    rng = W.SplitMix64(seed)
    c = W.Circuit()
    for q in range(10):
        c.h(q)
    for k in range(rounds):
        q = k % 12
        if k % 3 == 0:
            c.gate(W.K_RY, q, param=(rng.uniform() - 0.5) * 2.0)
        elif k % 3 == 1:
            c.h(q, ctrls=((q + 5) % 12,) if k % 5 == 0 else ())
        else:
            c.gate(W.K_X, (q + 3) % 12, controls=(q,))
            c.h(q)
        if k % 97 == 96:
            c.measure((q + 7) % 12, rng.uniform())
    return W.Workload(f"wrap_{n}q", n, 1e-20, c.array(), 1 << 14)


@pytest.mark.parametrize("n", [40, 100])
def test_index_reused_over_many_gates(sim, n):
    """Over 530 branching gates on one handle (hundreds of them through the
    partner index) the global index, alone and in the two-pass form, gives the
    LDS index's state, outcomes and counters bit for bit, and the oracle's."""
    w = _wrap_circuit(n, 520, 5)
    out = []
    for flags in (0, sim.SIM_FLAG_U2_GLOBAL_INDEX, sim.SIM_FLAG_U2_GLOBAL_INDEX | sim.SIM_FLAG_U2_TWO_PASS):
        s, outs, st = sim.run_workload(w, flags=flags)
        out.append((s.export(sort=False), list(outs), st))
        s.close()
    (a, oa, sa) = out[0]
    assert sa["u2_applied"] - sa["u2_split"] > 2 * 255
    for b, ob, sb in out[1:]:
        for x, y in zip(a, b):
            assert x.tobytes() == y.tobytes()
        assert oa == ob
        for k in ("u2_applied", "u2_skipped", "pruned", "updates", "peak_nnz", "measures", "u2_split"):
            assert sa[k] == sb[k], k
    o, oout, _ = oracle_run(w)
    assert oa == list(oout)
    order = np.lexsort((a[0], a[1]))
    assert_same_state(tuple(x[order] for x in a), o.export(), 1e-12, w.name)


def test_index_reused_across_table_sizes(sim):
    """Hundreds of global-index gates alternate between stages on small
    tables and on large ones on one handle: slots a larger table used before
    never pair wrong partners later, and every stage matches the oracle."""
    n = 80
    s = sim.Simulator(n, 1 << 18, 1e-20, flags=sim.SIM_FLAG_U2_GLOBAL_INDEX)
    try:
        # Gates come in inverse pairs on random labels (few partners): the
        # first doubles the state, the second pairs every entry and brings it
        # back, and both use the index.
        stages = [("small", 200), ("large", 120), ("small", 250), ("large", 60)]
        for k, (kind, gates) in enumerate(stages):
            lo, hi, amp = W.random_state(1700 + k, 50_000 if kind == "large" else 1500, n)
            c = W.Circuit()
            for g in range(gates // 2):
                q = (7 * g) % 16 if kind == "large" else g % 11
                if g % 3 == 0:
                    c.gate(W.K_RY, q, param=0.3 + 0.01 * g)
                    c.gate(W.K_RY, q, param=-(0.3 + 0.01 * g))
                else:
                    ctrls = ((q + 1) % 16,) if g % 3 == 1 else ()
                    c.h(q, ctrls=ctrls)
                    c.h(q, ctrls=ctrls)
            s.import_state(lo, hi, amp)
            _, _, st = s.apply_ops(c.array())
            o = Oracle(n, 1e-20)
            o.import_state(lo, hi, amp)
            o.run(c.array())
            assert_same_state(s.export(), o.export(), what=f"stage {k} ({kind})")
    finally:
        s.close()


def test_results_do_not_depend_on_count_reads(sim):
    """The host sizes chunked launches from its bound on the entry count and
    reads the exact count only at some points; block ranges, and the sums
    grouped by them, depend on the count alone.  Splitting a circuit before
    applied branching gates (where fused runs end anyway: a gate the cap
    skips does not end one, and a cut between measurements would break their
    chain, which sums in another order by design) and reading the count there
    gives the unsplit run's state and outcomes bit for bit."""
    w = W.config2(71, n=100, h_qubits=15, gates=3000, round_gates=1000, meas_per_round=3)
    kinds = w.ops["kind"]
    o = Oracle(w.n_qubits, w.eps)
    o.set_basis(*w.basis)
    _, tr = o.run(w.ops, trace=True)
    cuts = [i for i in range(1, len(kinds)) if kinds[i] in (W.K_H, W.K_RX, W.K_RY) and tr["applied"][i]]
    assert len(cuts) >= 20
    s = sim.Simulator(w.n_qubits, w.capacity, w.eps)
    try:
        s.set_basis(*w.basis)
        outs, prev = [], 0
        for c in cuts + [len(kinds)]:
            _, o, _ = s.apply_ops(w.ops[prev:c])
            outs += list(o)
            assert s.nnz > 0        # reads the exact count
            prev = c
        split = s.export(sort=False)
    finally:
        s.close()
    s2 = sim.Simulator(w.n_qubits, w.capacity, w.eps)
    try:
        s2.set_basis(*w.basis)
        _, o2, _ = s2.apply_ops(w.ops)
        whole = s2.export(sort=False)
    finally:
        s2.close()
    assert outs == list(o2)
    for a, b in zip(whole, split):
        assert a.tobytes() == b.tobytes()
