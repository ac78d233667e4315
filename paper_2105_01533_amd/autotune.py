"""Autotuner for the launch knobs of the simulator.

Knobs: fusion depth (fuse_max), the run length from which the bit-sliced
fused pass is used (bs_min_gates), the fused-pass kernel (mono_mode), the
per-entry pass block shape (block) and the hash-index load factor
(load_factor).  None of them changes which labels survive; they change speed
and, between fused-pass kernels, floating-point rounding only.

For each bucket (label width: <= 64 qubits or more; state size: log2 of the
capacity) a representative random circuit of that size is timed on one live
handle (sim_set_tuning changes the knobs without reallocating), with a greedy
coordinate search: knobs are visited in a fixed order, each set to its best
value with the others held, for a given number of sweeps.  The result is a
JSON table keyed by bucket; ``lookup`` returns the knobs for the nearest
bucket, and ``Simulator``/``Server`` callers pass them as sim_config fields.
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
DEFAULTS = {"fuse_max": 65536, "bs_min_gates": 16, "mono_mode": 0, "block": 256, "load_factor": 0.5}


def bucket_key(n_qubits: int, capacity: int) -> str:
    return f"{'wide' if n_qubits > 64 else 'narrow'}_lg{max(1, math.ceil(math.log2(max(capacity, 2))))}"


def greedy_search(measure, space=SPACE, start=DEFAULTS, sweeps: int = 1):
    """Coordinate search: measure(knobs) -> seconds (lower is better)."""
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
                if t < best_t:
                    best, best_t = cand, t
    return best, best_t, trials


def representative(W, n_qubits: int, log2cap: int, gates: int, seed: int = 99):
    """Config-2-style random circuit at this size: H on log2cap qubits, then
    `gates` random gates with capped H and two measurement rounds."""
    return W.config2(seed, n=n_qubits, h_qubits=log2cap, gates=gates, round_gates=max(1, gates // 2),
                     meas_per_round=min(4, log2cap), cap=1 << log2cap)


def tune(buckets=((24, 12), (24, 16), (100, 16), (100, 20), (100, 22)), gates: int = 4000, repeats: int = 3,
         sweeps: int = 1, cache: str | None = DEFAULT_CACHE, log=print):
    """Tune every (n_qubits, log2 capacity) bucket on the GPU; returns the
    table and writes it to `cache` (JSON) unless cache is None."""
    from . import sim as S
    from . import workloads as W

    table = {}
    for nq, lg in buckets:
        w = representative(W, nq, lg, gates)
        s = S.Simulator(nq, w.capacity, w.eps, load_factor=min(SPACE["load_factor"]))
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
        best, best_t, trials = greedy_search(measure, sweeps=sweeps)
        s.close()
        key = bucket_key(nq, w.capacity)
        table[key] = {"knobs": best, "seconds": best_t, "default_seconds": trials[0][1],
                      "n_qubits": nq, "log2_capacity": lg, "gates": gates, "trials": len(trials)}
        log(f"[autotune] {key}: {best} {best_t * 1e3:.2f} ms (default {trials[0][1] * 1e3:.2f} ms)")
    if cache:
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return table


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
    return dict(table[min(cands)[1]]["knobs"])


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="Tune launch knobs on this GPU and write the table.")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--gates", type=int, default=4000)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args()
    tune(gates=args.gates, repeats=args.repeats, cache=args.out)
