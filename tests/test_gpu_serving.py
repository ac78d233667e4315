"""GPU tests of the continuous-batching server (srv_* through the C-ABI).

Each request's result must be the same alone and in a mix (bitwise: the
batched kernels cut every state into fixed 2048-entry units), match the
oracle at the parity bar (labels exact, amplitudes within 1e-12, same
measurement outcomes), and the admission rules must hold: FIFO order, the
pool budget never exceeded, oversized requests rejected, failures confined
to their request.
"""
import sys

import numpy as np
import pytest

from helpers import assert_same_state
from oracle import run_workload as oracle_run
from paper_2105_01533_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S():
    from paper_2105_01533_amd import sim
    import torch
    assert torch.cuda.is_available()
    return sim


def mix():
    ws = [
        W.config0(41, n=20, h_qubits=6, gates=1500, cap=1 << 10),
        W.config0(42, n=70, h_qubits=9, gates=3000, cap=1 << 12),
        W.config1(43, w=8, adds=6, n=24),
        W.config2(44, n=100, h_qubits=10, gates=6000, round_gates=2000, meas_per_round=3),
        W.config2(45, n=40, h_qubits=13, gates=4000, round_gates=1000, meas_per_round=2),
        W.config3(46, terms=30),
        W.random_circuit(47, n=9, gates=300, h_frac=0.2, ctrl_max=3, measure_frac=0.02),
        W.random_circuit(48, n=128, gates=200, h_frac=0.03, ctrl_max=4, measure_frac=0.01),
    ]
    ws[6].capacity = 1 << 9
    ws[7].capacity = 1 << 14
    return ws


def run_server(S, ws, budget=1 << 30, slots=64, graph=True, arena_bytes=0, lane=None, flags=0, max_run_ops=None,
               **tuning):
    """Every request batched unless `lane` (a lane threshold) is given."""
    srv = S.Server(budget, max_slots=slots, graph=graph, arena_bytes=arena_bytes,
                   lane_capacity=S.SRV_LANE_OFF if lane is None else lane, flags=flags, max_run_ops=max_run_ops)
    ids = [srv.submit_workload(w, **tuning) for w in ws]
    srv.run()
    out = []
    for rid in ids:
        st, err = srv.poll(rid)
        assert st == S.SRV_DONE, (st, err)
        out.append(srv.result(rid))
    stats = srv.stats()
    srv.close()
    return out, stats


def test_alone_equals_mix_and_oracle(S):
    ws = mix()
    say("[gpu] server: mix of", len(ws))
    together, stats = run_server(S, ws)
    assert stats["completed"] == len(ws) and stats["failed"] == 0
    assert stats["ticks"] < sum(r[4]["mono_passes"] + r[4]["u2_applied"] + r[4]["measures"] for r in together)
    for w, res in zip(ws, together):
        alone, _ = run_server(S, [w])
        for a, b in zip(alone[0][:4], res[:4]):
            assert a.tobytes() == b.tobytes(), w.name
        o, oout, _ = oracle_run(w)
        assert list(res[3]) == list(oout), w.name
        assert_same_state(res[:3], o.export(), what=w.name)
        t = o.totals()
        assert res[4]["updates"] == t["updates"] and res[4]["u2_applied"] == t["u2_applied"]
        assert res[4]["u2_skipped"] == t["u2_skipped"]


def test_graph_replay_equals_direct_launches(S):
    ws = mix()[:5]
    a, sa = run_server(S, ws, graph=True)
    b, sb = run_server(S, ws, graph=False)
    # (tick counts may differ: a request sits out a tick while its circuit is
    # still being compiled or its next run grouped in the background)
    assert sa["completed"] == sb["completed"] == len(ws)
    for x, y in zip(a, b):
        for p, q in zip(x[:4], y[:4]):
            assert p.tobytes() == q.tobytes()


def test_direct_mode_requests(S):
    ws = mix()[:4]
    res, _ = run_server(S, ws, mono_mode=S.SIM_MONO_DIRECT)
    for w, r in zip(ws, res):
        o, oout, _ = oracle_run(w)
        assert list(r[3]) == list(oout)
        assert_same_state(r[:3], o.export(), what=w.name)


def test_budget_fifo_and_queueing(S):
    small = W.config0(51, n=20, h_qubits=5, gates=400, cap=1 << 8)
    big = W.config0(52, n=20, h_qubits=5, gates=400, cap=1 << 14)
    cfg = lambda w: S.sim_config(n_qubits=w.n_qubits, capacity=w.capacity, eps=w.eps)
    fb, fs = S.srv_footprint(cfg(big)), S.srv_footprint(cfg(small))
    assert fb > 4 * fs
    budget = fb + fs                                 # room for big + one small, never big + two small
    srv = S.Server(budget, max_slots=8, lane_capacity=S.SRV_LANE_OFF)
    ids = [srv.submit_workload(w) for w in (small, big, small, small)]
    srv.tick()
    states = [srv.poll(i)[0] for i in ids]
    assert states[0] == S.SRV_RUNNING or states[0] == S.SRV_DONE
    assert states[1] in (S.SRV_RUNNING, S.SRV_DONE)
    # FIFO: the third request (small) may not overtake while memory is short
    assert states[2] == S.SRV_QUEUED or states[1] != S.SRV_QUEUED
    srv.run()
    st = srv.stats()
    assert st["completed"] == 4 and st["pool_peak_bytes"] <= budget
    srv.close()


def test_oversized_and_invalid_requests_rejected(S):
    srv = S.Server(1 << 22, max_slots=4)
    w = W.config0(53, n=20, h_qubits=5, gates=100, cap=1 << 20)
    with pytest.raises(S.ServerError) as e:
        srv.submit_workload(w)
    assert e.value.code == S.SIM_E_CAPACITY
    c = W.Circuit()
    c.x(3, (3,))
    with pytest.raises(S.ServerError) as e:
        srv.submit(S.sim_config(n_qubits=8, capacity=16), S.sim_gates_from_ops(c.array()))
    assert e.value.code == S.SIM_E_ARG
    assert srv.stats()["submitted"] == 0
    srv.close()


def test_failures_stay_in_their_request(S):
    srv = S.Server(1 << 28, max_slots=8, lane_capacity=S.SRV_LANE_OFF)
    good = W.config0(54, n=20, h_qubits=5, gates=300, cap=1 << 8)
    c = W.Circuit()
    for q in range(6):
        c.h(q)                                   # 64 entries > capacity 32
    over = W.Workload("over", 10, 0.0, c.array(), capacity=32)
    m = W.Circuit()
    m.h(0)
    m.measure(1, 0.0, forced=1)                  # qubit 1 is 0 everywhere
    zero = W.Workload("zero", 4, 0.0, m.array(), capacity=8)
    ids = [srv.submit_workload(w) for w in (good, over, zero, good)]
    srv.run()
    res = [srv.poll(i) for i in ids]
    assert res[0] == (S.SRV_DONE, 0) and res[3] == (S.SRV_DONE, 0)
    assert res[1] == (S.SRV_FAILED, S.SIM_E_CAPACITY)
    assert res[2] == (S.SRV_FAILED, S.SIM_E_STATE)
    a, b = srv.result(ids[0]), srv.result(ids[3])
    for p, q in zip(a[:4], b[:4]):
        assert p.tobytes() == q.tobytes()
    srv.close()


def test_small_arena_defers_runs_alone_equals_mix(S):
    """With a 1 MiB op arena the mix's fused runs cannot all share a tick:
    runs that do not fit wait whole for the next tick (they are never cut,
    which would change their rounding), so every result is still bitwise the
    same alone and in the mix, and matches the oracle."""
    ws = [W.config0(51 + k, n=24, h_qubits=8, gates=20000, cap=1 << 12) for k in range(6)]
    together, stats = run_server(S, ws, arena_bytes=1 << 20)
    assert stats["completed"] == len(ws)
    for w, res in zip(ws, together):
        alone, _ = run_server(S, [w], arena_bytes=1 << 20)
        for a, b in zip(alone[0][:4], res[:4]):
            assert a.tobytes() == b.tobytes(), w.name
        o, oout, _ = oracle_run(w)
        assert list(res[3]) == list(oout), w.name
        assert_same_state(res[:3], o.export(), what=w.name)


def test_arena_too_small_is_rejected(S):
    with pytest.raises(S.ServerError):
        S.Server(1 << 24, max_slots=4, arena_bytes=1 << 16)


@pytest.mark.skip(reason="the large-state lane is off: server runs with it ended in intermittent GPU "
                         "memory faults whose cause has not been found")
def test_large_lane_matches_single_state_and_oracle(S):
    """With the lane threshold at 2^12 entries, the mix's larger requests run
    whole through the single-state engine on the lane while the rest are
    batched: each lane result is bitwise the engine's own (the same code on a
    workspace from the pool), every result matches the oracle, and the lane
    counters add up."""
    ws = mix()
    lane = [w.capacity >= (1 << 12) for w in ws]
    assert any(lane) and not all(lane)
    srv = S.Server(1 << 30, max_slots=64, lane_capacity=1 << 12)
    ids = [srv.submit_workload(w) for w in ws]
    srv.run()
    stats = srv.stats()
    assert stats["completed"] == len(ws) and stats["failed"] == 0
    assert stats["lane_completed"] == sum(lane)
    for w, rid, on_lane in zip(ws, ids, lane):
        lo, hi, amp, outs, st = srv.result(rid)
        o, oout, _ = oracle_run(w)
        assert list(outs) == list(oout), w.name
        assert_same_state((lo, hi, amp), o.export(), what=w.name)
        if on_lane:
            s, eouts, est = S.run_workload(w)
            elo, ehi, eamp = s.export()
            s.close()
            assert np.array_equal(lo, elo) and np.array_equal(hi, ehi) and amp.tobytes() == eamp.tobytes(), w.name
            assert list(outs) == list(eouts) and st["updates"] == est["updates"]
    srv.close()


@pytest.mark.skip(reason="the large-state lane is off: server runs with it ended in intermittent GPU "
                         "memory faults whose cause has not been found")
def test_large_lane_fifo_and_failures(S):
    """Lane requests queue in their own FIFO, are admitted by pool memory,
    and a failing one (capacity exceeded) fails alone."""
    big = [W.config0(61 + k, n=30, h_qubits=10, gates=2000, cap=1 << 13) for k in range(4)]
    c = W.Circuit()
    for q in range(14):
        c.h(q)                                   # 2^14 entries > capacity 2^13
    over = W.Workload("over", 20, 0.0, c.array(), capacity=1 << 13)
    srv = S.Server(1 << 30, max_slots=8, lane_capacity=1 << 13)
    ids = [srv.submit_workload(w) for w in (big[0], over, big[1], big[2], big[3])]
    srv.run()
    res = [srv.poll(i) for i in ids]
    assert res[1] == (S.SRV_FAILED, S.SIM_E_CAPACITY)
    assert all(r == (S.SRV_DONE, 0) for k, r in enumerate(res) if k != 1)
    assert srv.stats()["lane_completed"] == 5
    for w, rid in zip([big[0], big[1], big[2], big[3]], [ids[0], ids[2], ids[3], ids[4]]):
        lo, hi, amp, outs, _ = srv.result(rid)
        o, oout, _ = oracle_run(w)
        assert list(outs) == list(oout)
        assert_same_state((lo, hi, amp), o.export(), what=w.name)
    srv.close()


def test_result_records_equal_arrays(S):
    """srv_result (key records) and srv_result_soa (separate arrays) return
    the same state, storage order, for narrow and wide requests."""
    import ctypes

    ws = mix()[:5]
    srv = S.Server(1 << 30, max_slots=64, lane_capacity=S.SRV_LANE_OFF)
    ids = [srv.submit_workload(w) for w in ws]
    srv.run()
    for w, rid in zip(ws, ids):
        lo, hi, amp, outs, st = srv.result(rid, sort=False)
        n = len(lo)
        assert n > 0, w.name
        keys = np.empty(n, S.KEY_DTYPE)
        amps = np.empty(n, np.complex128)
        o = np.empty(max(len(outs), 1), np.int32)
        nnz, nout = ctypes.c_uint64(), ctypes.c_uint64()
        assert S._lib.srv_result(srv.h, rid, S._ptr(keys), S._ptr(amps), n, ctypes.byref(nnz), S._ptr(o), len(o),
                                 ctypes.byref(nout), None) == 0
        assert nnz.value == n and nout.value == len(outs)
        assert np.array_equal(keys["lo"], lo) and np.array_equal(keys["hi"], hi), w.name
        assert amps.tobytes() == amp.tobytes(), w.name
        assert list(o[:nout.value]) == list(outs)
        if w.n_qubits <= 64:
            assert not hi.any()
    srv.close()


def test_small_states_lds_index_equals_global_index(S):
    """Branching gates of batched states of at most 8192 entries run one
    block per state with the partner index in LDS; the results are bit for bit
    those of the global-index kernels (SRV_FLAG_U2_GLOBAL_INDEX), alone and in
    the mix, and each matches the oracle."""
    ws = mix()
    a, sa = run_server(S, ws)
    b, sb = run_server(S, ws, flags=S.SRV_FLAG_U2_GLOBAL_INDEX)
    assert sa["completed"] == sb["completed"] == len(ws)
    for w, x, y in zip(ws, a, b):
        for p, q in zip(x[:4], y[:4]):
            assert p.tobytes() == q.tobytes(), w.name
    # a state that crosses the limit: 13 Hadamards reach 8192 entries, the
    # 14th and 15th run on 8192 and 16384 entries
    c = W.Circuit()
    for q in range(15):
        c.h(q)
    c.gate(W.K_RY, 3, controls=(20,), param=0.3)
    w = W.Workload("h15", 24, 0.0, c.array(), 1 << 16, (1 << 20, 0))
    for flags in (0, S.SRV_FLAG_U2_GLOBAL_INDEX):
        res, _ = run_server(S, [w, ws[0]], flags=flags)
        o, oout, _ = oracle_run(w)
        assert_same_state(res[0][:3], o.export(), what=f"h15 flags={flags}")


def test_large_states_register_plane_runs(S):
    """Fused runs of batched states of at least 2^16 entries take the
    register-plane kernel (one launch per run ahead of the tick's graph); the
    results are bit for bit those of the LDS-plane tile (SRV_FLAG_NO_RP), alone
    and in a mix with small states, and match the oracle."""
    ws = [W.config2(61, n=100, h_qubits=17, gates=3000, round_gates=1500, meas_per_round=2),
          W.config1(62, w=16, adds=2, n=40), mix()[0], mix()[6]]
    a, sa = run_server(S, ws)
    b, sb = run_server(S, ws, flags=S.SRV_FLAG_NO_RP)
    assert sa["rp_runs"] > 0 and sb["rp_runs"] == 0
    for w, x, y in zip(ws, a, b):
        for p, q in zip(x[:4], y[:4]):
            assert p.tobytes() == q.tobytes(), w.name
    alone, _ = run_server(S, [ws[0]])
    for p, q in zip(alone[0][:4], a[0][:4]):
        assert p.tobytes() == q.tobytes()
    for w, res in zip(ws[:2], a[:2]):
        say(f"[gpu] oracle {w.name}")
        o, oout, _ = oracle_run(w)
        assert list(res[3]) == list(oout), w.name
        assert_same_state(res[:3], o.export(), what=w.name)


def test_gate_after_run_shares_its_tick(S):
    """A branching gate or measurement right after a request's fused run runs
    in the run's tick, and consecutive measurements in one tick (later launch
    rounds); states, outcomes and per-request counters are bit for bit those
    of one segment per tick (SRV_FLAG_ONE_SEGMENT), with fewer ticks, also
    when a small arena defers runs, on register-plane states, and with every
    slot taken (four slots: a tick then has up to two first-round items per
    request)."""
    ws = mix() + [W.config2(63, n=100, h_qubits=17, gates=2000, round_gates=1000, meas_per_round=2)]
    keys = ("updates", "u2_applied", "u2_skipped", "measures", "mono_passes", "bitslice_passes", "peak_nnz")
    ref = None
    for arena, slots in ((0, 64), (1 << 20, 64), (0, 4)):
        say(f"[gpu] server: arena {arena} slots {slots}")
        a, sa = run_server(S, ws, arena_bytes=arena, slots=slots)
        b, sb = run_server(S, ws, arena_bytes=arena, slots=slots, flags=S.SRV_FLAG_ONE_SEGMENT)
        assert sa["completed"] == sb["completed"] == len(ws)
        assert sa["paired"] > 0 and sb["paired"] == 0
        assert sa["chained"] > 0 and sb["chained"] == 0
        assert sa["ticks"] < sb["ticks"], (sa["ticks"], sb["ticks"])
        assert sa["items"] == sb["items"]
        if arena == 0:
            ref = ref or a     # (the arena bounds run length, so rounding depends on its size)
        for w, x, y, z in zip(ws, a, b, ref if arena == 0 else a):
            for p, q, r in zip(x[:4], y[:4], z[:4]):
                assert p.tobytes() == q.tobytes() == r.tobytes(), (w.name, arena, slots)
            for k in keys:
                assert x[4][k] == y[4][k], (w.name, k)
    say(f"[gpu] oracle {ws[-1].name}")
    o, oout, _ = oracle_run(ws[-1])
    assert list(a[-1][3]) == list(oout)
    assert_same_state(a[-1][:3], o.export(), what=ws[-1].name)


def test_measurement_chains(S):
    """Runs of consecutive measurements (longer than one tick's limit of
    eight, on narrow and wide labels, forced and sampled) give the outcomes
    and states of one measurement per tick and of the oracle; a
    zero-probability forced outcome inside a chain fails its request with the
    outcomes before it kept, as one at a time, while the other requests of
    the tick finish."""
    def chain_circuit(n, forced_zero_at=None):
        c = W.Circuit()
        for q in range(12):
            c.h(q)
        c.gate(W.K_X, n - 1, controls=(0,))
        for k in range(11):                       # 11 consecutive measurements: rounds of 8 and 3
            q = k if k != forced_zero_at else 30
            c.measure(q, 0.37 + 0.05 * k, forced=1 if k in (2, forced_zero_at) else -1)
        c.h(3)
        c.measure(3, 0.5)
        c.measure(n - 1, 0.2)
        return c.array()
    ws = [W.Workload("chain40", 40, 0.0, chain_circuit(40), 1 << 13),
          W.Workload("chain100", 100, 0.0, chain_circuit(100), 1 << 13),
          mix()[0]]
    a, sa = run_server(S, ws)
    b, sb = run_server(S, ws, flags=S.SRV_FLAG_ONE_SEGMENT)
    assert sa["chained"] >= 2 * 10 and sb["chained"] == 0
    for w, x, y in zip(ws, a, b):
        for p, q in zip(x[:4], y[:4]):
            assert p.tobytes() == q.tobytes(), w.name
        o, oout, _ = oracle_run(w)
        assert list(x[3]) == list(oout), w.name
        assert_same_state(x[:3], o.export(), what=w.name)
    # qubit 30 is 0 in every entry: forcing 1 there fails the request
    bad = W.Workload("chain_zero", 40, 0.0, chain_circuit(40, forced_zero_at=5), 1 << 13)
    for flags in (0, S.SRV_FLAG_ONE_SEGMENT):
        srv = S.Server(1 << 30, max_slots=8, lane_capacity=S.SRV_LANE_OFF, flags=flags)
        ids = [srv.submit_workload(w) for w in (bad, ws[0])]
        srv.run()
        st, err = srv.poll(ids[0])
        assert st == S.SRV_FAILED and err == S.SIM_E_STATE, flags
        assert srv.poll(ids[1])[0] == S.SRV_DONE
        srv.close()


def test_run_cap_changes_rounding_only(S):
    """max_run_ops cuts each request's fused runs per tick: labels, outcomes
    and counters other than the pass counts do not depend on it, amplitudes
    agree to rounding, each setting gives the same bits alone and in a mix,
    and matches the oracle."""
    ws = [W.config1(64, w=12, adds=6, n=40), W.config2(65, n=100, h_qubits=10, gates=6000, round_gates=2000,
                                                        meas_per_round=3), mix()[1]]
    # (all with eps = 1e-20: a residue of a rounding difference is pruned either way)
    out = {}
    for cap in (64, 4096, 65536):
        srv = S.Server(1 << 30, max_slots=8, lane_capacity=S.SRV_LANE_OFF, max_run_ops=cap)
        assert srv.knobs["max_run_ops"] == cap
        ids = [srv.submit_workload(w) for w in ws]
        srv.run()
        out[cap] = [srv.result(i) for i in ids]
        srv.close()
        alone, _ = run_server(S, [ws[1]], max_run_ops=cap)
        for p, q in zip(alone[0][:4], out[cap][1][:4]):
            assert p.tobytes() == q.tobytes(), cap
    for w, a, b, c in zip(ws, out[64], out[4096], out[65536]):
        for x in (a, b):
            assert x[0].tobytes() == c[0].tobytes() and x[1].tobytes() == c[1].tobytes(), w.name
            assert list(x[3]) == list(c[3]), w.name
            for k in ("updates", "u2_applied", "u2_skipped", "measures", "peak_nnz"):
                assert x[4][k] == c[4][k], (w.name, k)
            assert np.max(np.abs(x[2] - c[2])) <= 1e-12, w.name
        assert a[4]["mono_passes"] >= c[4]["mono_passes"]
        o, oout, _ = oracle_run(w)
        assert list(a[3]) == list(oout), w.name
        assert_same_state(a[:3], o.export(), what=w.name)


def test_destroy_with_work_in_flight(S):
    """A server closed while requests are queued, compiling, running and
    being copied out shuts its background workers down cleanly; a new server
    afterwards still gives the oracle's results."""
    ws = mix()
    for rounds in (0, 1, 3):
        srv = S.Server(1 << 30, max_slots=4, lane_capacity=S.SRV_LANE_OFF)
        ids = [srv.submit_workload(w) for w in ws]
        for _ in range(rounds):
            srv.tick()
        srv.close()
    res, _ = run_server(S, ws[:2])
    for w, r in zip(ws[:2], res):
        o, oout, _ = oracle_run(w)
        assert list(r[3]) == list(oout), w.name
        assert_same_state(r[:3], o.export(), what=w.name)
