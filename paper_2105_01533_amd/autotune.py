"""Autotuner for the launch knobs of the simulator and the server.

Per-state knobs: fusion depth (fuse_max), the run length from which the
bit-sliced fused pass is used (bs_min_gates), per-entry or bit-sliced fused
passes (mono_mode), the per-entry pass block shape (block) and the hash-index
load factor (load_factor).  (Which bit-sliced kernel runs, register planes
or LDS planes, is fixed at creation and not searched.)  None of them changes which labels
survive; they change speed and, between fused-pass kernels, floating-point
rounding only.

Server knobs: the batched tick's grid (blocks per kernel, grid) and its
per-request update cap (tick_updates: a fused run is cut so that it makes at
most that many gate-entry updates in one tick; 0 = no cap), tuned for the p99
latency of a reduced serving trace replayed at 0.8x the one-at-a-time rate.
(The large-state lane stays off and is not searched.)  The grid changes speed
only; a per-tick cap also changes where a request's runs are cut, and with
that its floating-point rounding, never its labels.

For each bucket (label width: <= 64 qubits or more; state size: log2 of the
capacity) a representative random circuit of that size is timed on one live
handle (sim_set_tuning changes the knobs without reallocating), with a greedy
coordinate search: knobs are visited in a fixed order, each set to its best
value with the others held, for a given number of sweeps.  The result is a
JSON table keyed by bucket (plus a "server" entry); ``lookup`` returns the
knobs for the nearest bucket and ``server_knobs`` the server's.  ``Simulator``
and ``Server`` apply the committed table (tuning_mi355x.json) by default to
every knob the caller leaves unset; ``tuned=False`` or the environment
variable SPARSESIM_TUNING=off turns that off.
"""
from __future__ import annotations

import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning_mi355x.json")

SPACE = {
    "fuse_max": [16, 256, 4096, 65536],
    "bs_min_gates": [4, 16, 64],
    "mono_mode": [0, 1],                # auto (bit-sliced for long runs), per-entry only
    "block": [64, 128, 256],
    "load_factor": [0.25, 0.5, 0.7],
}
DEFAULTS = {"fuse_max": 65536, "bs_min_gates": 16, "mono_mode": 0, "flags": 0, "block": 256, "load_factor": 0.5}
KNOBS = tuple(DEFAULTS)

SERVER_SPACE = {
    "grid": [512, 1024, 2048, 4096],
    "tick_updates": [0, 1 << 30, 1 << 32],
    "max_run_ops": [1024, 4096, 16384, 65536],
}
# The lane is off (lane_capacity 0): server runs with it ended in intermittent
# GPU memory faults whose cause is not known, so it is neither used nor tuned.
SERVER_DEFAULTS = {"lane_capacity": 0, "lane_workers": 8, "grid": 2048, "tick_updates": 0, "max_run_ops": 4096}


def bucket_key(n_qubits: int, capacity: int) -> str:
    return f"{'wide' if n_qubits > 64 else 'narrow'}_lg{max(1, math.ceil(math.log2(max(capacity, 2))))}"


def greedy_search(measure, space=SPACE, start=DEFAULTS, sweeps: int = 1, min_gain: float = 0.0):
    """Coordinate search: measure(knobs) -> seconds (lower is better).  A
    value replaces the held one only if it is faster by more than the
    fraction min_gain (so timing noise does not move a knob off its
    default)."""
    best = dict(start)
    best_t = measure(best)
    trials = [(dict(best), best_t)]
    for _ in range(sweeps):
        for name, values in space.items():
            held = best[name]                    # already measured with the others held
            for v in values:
                if v == held:
                    continue
                cand = dict(best)
                cand[name] = v
                t = measure(cand)
                trials.append((cand, t))
                if t < best_t * (1.0 - min_gain):
                    best, best_t = cand, t
    return best, best_t, trials


def enabled() -> bool:
    """False when the environment variable SPARSESIM_TUNING is off/0/false."""
    return os.environ.get("SPARSESIM_TUNING", "on").lower() not in ("off", "0", "false", "no")


_TABLE = None


def table() -> dict:
    """The committed table (loaded once)."""
    global _TABLE
    if _TABLE is None:
        _TABLE = load()
    return _TABLE


def state_knobs(n_qubits: int, capacity: int, given: dict) -> dict:
    """The per-state knobs: those in `given` that are not None, the table's
    for the others (or the defaults when tuning is off)."""
    base = lookup(table(), n_qubits, capacity) if enabled() else dict(DEFAULTS)
    return {k: (given[k] if given.get(k) is not None else base.get(k, DEFAULTS[k])) for k in KNOBS}


def server_knobs(given: dict | None = None) -> dict:
    """The server knobs: those in `given` that are not None, the table's for
    the others (or the defaults when tuning is off)."""
    given = given or {}
    base = dict(SERVER_DEFAULTS)
    if enabled():
        base.update(table().get("server", {}).get("knobs", {}))
    return {k: (given[k] if given.get(k) is not None else base[k]) for k in SERVER_DEFAULTS}


def representative(W, n_qubits: int, log2cap: int, gates: int, seed: int = 99):
    """Config-2-style random circuit at this size: H on log2cap qubits, then
    `gates` random gates with capped H and two measurement rounds."""
    return W.config2(seed, n=n_qubits, h_qubits=log2cap, gates=gates, round_gates=max(1, gates // 2),
                     meas_per_round=min(4, log2cap), cap=1 << log2cap)


def tune(buckets=((24, 12), (24, 16), (100, 16), (100, 20), (100, 22)), gates: int = 20_000,
         repeats: int = 3, sweeps: int = 1, cache: str | None = DEFAULT_CACHE, server: bool = False,
         min_gain: float = 0.03, log=print):
    """Tune every (n_qubits, log2 capacity) bucket on the GPU, then (server)
    the server knobs; returns the table and writes it to `cache` (JSON)
    unless cache is None."""
    from . import sim as S
    from . import workloads as W

    table = {}
    for nq, lg in buckets:
        w = representative(W, nq, lg, gates)
        s = S.Simulator(nq, w.capacity, w.eps, load_factor=min(SPACE["load_factor"]), tuned=False)
        g = S.sim_gates_from_ops(w.ops)

        def measure(knobs):
            S.sim_set_tuning(s.h, **knobs)
            ts = []
            for _ in range(repeats):
                s.set_basis(*w.basis)
                t0 = time.perf_counter()
                s.apply_gates(g)
                ts.append(time.perf_counter() - t0)
            return sorted(ts)[len(ts) // 2]

        measure(DEFAULTS)                              # warm
        best, best_t, trials = greedy_search(measure, sweeps=sweeps, min_gain=min_gain)
        s.close()
        key = bucket_key(nq, w.capacity)
        table[key] = {"knobs": best, "seconds": best_t, "default_seconds": trials[0][1],
                      "n_qubits": nq, "log2_capacity": lg, "gates": gates, "trials": len(trials)}
        log(f"[autotune] {key}: {best} {best_t * 1e3:.2f} ms (default {trials[0][1] * 1e3:.2f} ms)")
    if server:
        table["server"] = tune_server(min_gain=min_gain, log=log)
    if cache:
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return table


def tune_server(requests: int = 128, max_log2: int = 22, max_gates: int = 100_000, repeats: int = 2,
                budget_gib: int = 32, min_gain: float = 0.03, log=print) -> dict:
    """Greedy search over SERVER_SPACE for the p99 latency of a reduced
    serving trace (seed 7: config-0..2 families, caps 2^8..2^max_log2,
    1e3..max_gates gates) replayed open loop at 0.8x the one-at-a-time service
    rate (measured first, closed loop, on the same requests), with the default
    per-state knobs."""
    from . import serving, workloads as W

    trace = W.serving_trace(7, requests=requests, rate=1.0, cap_log2=(8, max_log2), gates_range=(1000, max_gates))
    reqs = serving.prepare(trace, tuned=False)
    closed, _ = serving.run_one_at_a_time(reqs, arrivals=False)
    rate = 0.8 * closed["requests_per_s"]
    for r, (t, _) in zip(reqs, trace):
        r.arrival = t / rate

    def measure(knobs):
        ps = []
        for _ in range(repeats):
            out, _ = serving.run_batched(reqs, budget_gib << 30, arrivals=True, **knobs)
            ps.append(out["p99_ms"] * 1e-3)
        return min(ps)

    base, _ = serving.run_one_at_a_time(reqs, arrivals=True)
    measure(SERVER_DEFAULTS)                           # warm
    best, best_t, trials = greedy_search(measure, space=SERVER_SPACE, start=SERVER_DEFAULTS, min_gain=min_gain)
    log(f"[autotune] server: {best} p99 {best_t * 1e3:.1f} ms (default {trials[0][1] * 1e3:.1f} ms; "
        f"one at a time {base['p99_ms']:.1f} ms at {rate:.1f} requests/s)")
    return {"knobs": best, "p99_s": best_t, "default_p99_s": trials[0][1], "one_at_a_time_p99_s": base["p99_ms"] * 1e-3,
            "rate_per_s": rate, "trials": len(trials),
            "trace": f"{requests} requests (seed 7), caps 2^8..2^{max_log2}, 1e3..{max_gates} gates, Poisson at "
                     f"0.8x the one-at-a-time rate"}


def load(cache: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(cache):
        return {}
    with open(cache) as f:
        return json.load(f)


def lookup(table: dict, n_qubits: int, capacity: int) -> dict:
    """Knobs of the bucket with the same label width and the nearest size;
    the defaults if the table has no bucket of that width."""
    width = "wide" if n_qubits > 64 else "narrow"
    lg = max(1, math.ceil(math.log2(max(capacity, 2))))
    cands = [(abs(v["log2_capacity"] - lg), k) for k, v in table.items() if k.startswith(width)]
    if not cands:
        return dict(DEFAULTS)
    return {**DEFAULTS, **table[min(cands)[1]]["knobs"]}


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="Tune launch knobs on this GPU and write the table.")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--gates", type=int, default=20_000)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--server", action="store_true",
                    help="also tune the server's tick grid, per-tick update cap and run cap (p99 of a reduced trace)")
    ap.add_argument("--server-only", action="store_true",
                    help="keep the table's per-state buckets (read from --table) and tune only the server")
    ap.add_argument("--table", default=DEFAULT_CACHE, help="table read by --server-only")
    args = ap.parse_args()
    if args.server_only:
        t = load(args.table)
        t["server"] = tune_server()
        with open(args.out, "w") as f:
            json.dump(t, f, indent=1, sort_keys=True)
    else:
        tune(gates=args.gates, repeats=args.repeats, cache=args.out, server=args.server)
