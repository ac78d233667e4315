"""Serving driver: replays a timed request trace through the batched server
or through one-at-a-time plain launches, and reports throughput and latency.

Latency of a request = completion time - arrival time, on the host's wall
clock; requests arrive open-loop at their trace times.  Both systems see the
same trace and the same converted circuits, and both deliver every finished
state to host memory (storage order, unsorted) inside the timed region: the
server copies a finished state out when it frees its device memory, the plain
path exports it from its own handle.
"""
from __future__ import annotations

import time

import numpy as np

from . import sim as S


class Prepared:
    """A request ready to submit: its gate records and its state configuration
    (the library's default knobs, or the autotuner table's with tuned=True).

    The serving runs use the default per-request knobs: a replay of the
    512-request trace through the server with the table's per-request knobs
    ended in a GPU fault whose cause has not been found (the same server
    configuration with default per-request knobs, and one-at-a-time runs with
    the table's knobs, run cleanly)."""

    def __init__(self, arrival: float, w, tuned: bool = False):
        from . import autotune
        self.arrival = arrival
        self.w = w
        self.gates = S.sim_gates_from_ops(w.ops)
        self.knobs = autotune.state_knobs(w.n_qubits, w.capacity, {}) if tuned else {}
        self.cfg = S.sim_config(n_qubits=w.n_qubits, capacity=w.capacity, eps=w.eps, **self.knobs)


def prepare(trace, tuned: bool = False):
    return [Prepared(t, w, tuned) for t, w in trace]


def _pct(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if xs else 0.0


def _summary(name, reqs, done, t0, t_end, updates, arrivals=True):
    # Without arrivals every request is submitted at time 0.
    lat = [done[i] - (reqs[i].arrival if arrivals else 0.0) for i in range(len(reqs))]
    span = t_end - t0
    return {"system": name, "requests": len(reqs), "makespan_s": span, "requests_per_s": len(reqs) / span,
            "updates_per_s": updates / span, "p50_ms": 1e3 * _pct(lat, 50), "p99_ms": 1e3 * _pct(lat, 99),
            "mean_ms": 1e3 * float(np.mean(lat))}


def run_one_at_a_time(reqs, arrivals=True, keep_results=False, tuning: dict | None = None):
    """FIFO, one simulation at a time through sim_apply_gates on its own handle.
    tuning: optional autotuner table (each request runs with its bucket's
    knobs)."""
    from . import autotune

    import torch

    done = [0.0] * len(reqs)
    results = [None] * len(reqs)
    updates = 0
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        if arrivals:
            wait = t0 + r.arrival - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
        k = autotune.lookup(tuning, r.w.n_qubits, r.w.capacity) if tuning else r.knobs
        s = S.Simulator(r.w.n_qubits, r.w.capacity, r.w.eps, tuned=False, **k)
        s.set_basis(*r.w.basis)
        rc, outs, st = s.apply_gates(r.gates, raise_on_error=False)
        state = s.export(sort=False) if rc == 0 else None
        if keep_results:
            results[i] = (state, outs, st, rc)
        del state
        s.close()
        updates += st["updates"]
        done[i] = time.perf_counter() - t0
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    out = _summary("one_at_a_time", reqs, done, 0.0, t_end - t0, updates, arrivals)
    return out, results


def run_batched(reqs, budget_bytes: int, max_slots: int = 256, arrivals=True, keep_results=False, graph=True,
                tick_updates: int | None = None, grid: int | None = None, lane_capacity: int | None = None,
                lane_workers: int | None = None, tuning: dict | None = None, flags: int = 0,
                max_run_ops: int | None = None):
    """Replay through the continuous-batching server (open loop when
    arrivals, else every request at time 0).  Server knobs left None take the
    autotuner table's values.  tuning: optional table replacing each
    request's knobs by its bucket's.  flags: SRV_FLAG_* of the server."""
    from . import autotune

    srv = S.Server(budget_bytes, max_slots=max_slots, graph=graph, tick_updates=tick_updates, grid=grid,
                   lane_capacity=lane_capacity, lane_workers=lane_workers, flags=flags, max_run_ops=max_run_ops)
    if tuning:
        for r in reqs:
            k = autotune.lookup(tuning, r.w.n_qubits, r.w.capacity)
            r.cfg = S.sim_config(n_qubits=r.w.n_qubits, capacity=r.w.capacity, eps=r.w.eps, **k)
    n = len(reqs)
    ids = [None] * n
    done = [0.0] * n
    results = [None] * n
    pending = {}
    nxt = 0
    updates = 0
    t0 = time.perf_counter()
    while nxt < n or pending:
        now = time.perf_counter() - t0
        while nxt < n and (not arrivals or reqs[nxt].arrival <= now):
            rid = srv.submit(reqs[nxt].cfg, reqs[nxt].gates, reqs[nxt].w.basis)
            ids[nxt] = rid
            pending[rid] = nxt
            nxt += 1
        if not pending:
            time.sleep(max(0.0, reqs[nxt].arrival - (time.perf_counter() - t0)))
            continue
        srv.tick()
        t = time.perf_counter() - t0
        for rid in list(pending):
            st, err = srv.poll(rid)
            if st in (S.SRV_DONE, S.SRV_FAILED):
                i = pending.pop(rid)
                done[i] = t
                if st == S.SRV_DONE:
                    res = srv.result(rid, sort=False)
                    updates += res[4]["updates"]
                    if keep_results:
                        results[i] = res
                    del res
                srv.release(rid)
    t_end = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    out = _summary("batched", reqs, done, 0.0, t_end, updates, arrivals)
    out["server"] = stats
    out["server_knobs"] = dict(srv.knobs)
    return out, results


def _sorted(lo, hi, amp):
    order = np.lexsort((lo, hi))
    return lo[order], hi[order], amp[order]


def compare_results(plain, batched):
    """Per-request comparison of one-at-a-time results (state, outcomes, stats,
    rc) with batched ones (lo, hi, amp, outcomes, stats): keys and outcomes
    must match exactly; returns (label mismatches, largest amplitude
    difference, requests compared)."""
    mism, worst, n = 0, 0.0, 0
    for x, y in zip(plain, batched):
        if x is None or y is None or x[0] is None:
            continue
        n += 1
        lo, hi, amp = _sorted(*x[0])
        blo, bhi, bamp = _sorted(y[0], y[1], y[2])
        if not (np.array_equal(lo, blo) and np.array_equal(hi, bhi) and list(x[1]) == list(y[3])):
            mism += 1
        elif len(amp):
            worst = max(worst, float(np.max(np.abs(amp - bamp))))
    return mism, worst, n
