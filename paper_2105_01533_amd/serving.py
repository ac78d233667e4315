"""Serving driver: replays a timed request trace through the batched server
or through one-at-a-time plain launches, and reports throughput and latency.

Latency of a request = completion time - arrival time, on the host's wall
clock; requests arrive open-loop at their trace times.  Both systems see the
same trace and the same converted circuits.
"""
from __future__ import annotations

import time

import numpy as np

from . import sim as S


class Prepared:
    def __init__(self, arrival: float, w):
        self.arrival = arrival
        self.w = w
        self.gates = S.sim_gates_from_ops(w.ops)
        self.cfg = S.sim_config(n_qubits=w.n_qubits, capacity=w.capacity, eps=w.eps)


def prepare(trace):
    return [Prepared(t, w) for t, w in trace]


def _pct(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if xs else 0.0


def _summary(name, reqs, done, t0, t_end, updates, arrivals=True):
    # Without arrivals every request is submitted at time 0.
    lat = [done[i] - (reqs[i].arrival if arrivals else 0.0) for i in range(len(reqs))]
    span = t_end - t0
    return {"system": name, "requests": len(reqs), "makespan_s": span, "requests_per_s": len(reqs) / span,
            "updates_per_s": updates / span, "p50_ms": 1e3 * _pct(lat, 50), "p99_ms": 1e3 * _pct(lat, 99),
            "mean_ms": 1e3 * float(np.mean(lat))}


def run_one_at_a_time(reqs, arrivals=True, keep_results=False):
    """FIFO, one simulation at a time through sim_apply_gates on its own handle."""
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
        s = S.Simulator(r.w.n_qubits, r.w.capacity, r.w.eps)
        s.set_basis(*r.w.basis)
        rc, outs, st = s.apply_gates(r.gates, raise_on_error=False)
        if keep_results:
            results[i] = (s.export() if rc == 0 else None, outs, st, rc)
        s.close()
        updates += st["updates"]
        done[i] = time.perf_counter() - t0
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    out = _summary("one_at_a_time", reqs, done, 0.0, t_end - t0, updates, arrivals)
    return out, results


def run_batched(reqs, budget_bytes: int, max_slots: int = 256, arrivals=True, keep_results=False, graph=True,
                tick_updates: int = 1 << 27, tuning: dict | None = None):
    """Replay through the continuous-batching server (open loop when
    arrivals, else every request at time 0).  tuning: optional autotuner
    table; each request then runs with the knobs of its bucket."""
    from . import autotune

    srv = S.Server(budget_bytes, max_slots=max_slots, graph=graph, tick_updates=tick_updates)
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
                    res = srv.result(rid)
                    updates += res[4]["updates"]
                    if keep_results:
                        results[i] = res
                srv.release(rid)
    t_end = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    out = _summary("batched", reqs, done, 0.0, t_end, updates, arrivals)
    out["server"] = stats
    return out, results
