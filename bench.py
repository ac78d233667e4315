"""Benchmark: nonzero-amplitude gate updates/s of the sparse simulator on one MI355X.

A step simulates one whole synthetic circuit from its initial basis state
through the C-ABI (state resident in HBM; the op list, its conversion and
upload are inside the timed region).  Default workload: the 100-qubit random
circuit (H on 24 qubits -> 2^24 entries, 200,000 gates, 8 measurements every
20,000 gates).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c0": ("config0", "plain sparse sim, 24 qubits, 1,024 -> <=2^16 entries, 5,000 gates, measure q0..q3"),
    "c1": ("config1", "CDKM adder x50 on a 2^20-entry register, 64 qubits, Rz ladder, H layer"),
    "c2": ("config2", "random circuit, 100 qubits, 2^24 entries, 200,000 gates (80% X/CNOT/Toffoli, "
                      "15% Z/S/T/Rz, 5% H capped at 2^24), 8 measurements every 20,000 gates"),
    "c3": ("config3", "Trotter-like step, 40 qubits, 500 random 4-local Pauli exponentials, eps 1e-10"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, seconds_budget: float = 20.0):
    """The oracle as it stands, single-threaded, on a bounded prefix of the
    same workload: the initial H layer plus as many following gates as fit the
    budget (estimated from a short calibration prefix)."""
    import numpy as np

    from oracle import Oracle
    from paper_2105_01533_amd import workloads as W

    ops = w.ops
    kinds = ops["kind"]
    first_body = int(np.argmax(~np.isin(kinds, (W.K_H,)))) if np.any(kinds != W.K_H) else len(ops)
    best = None
    n_body = 64
    while True:
        o = Oracle(w.n_qubits, w.eps)
        o.set_basis(*w.basis)
        t0 = time.perf_counter()
        o.run(ops[:first_body + n_body])
        dt = time.perf_counter() - t0
        best = (n_body, dt, o.totals()["updates"])
        del o
        if dt > seconds_budget / 3 or first_body + n_body >= len(ops):
            break
        n_body = min(len(ops) - first_body, int(n_body * max(2.0, 0.9 * seconds_budget / max(dt, 1e-3))))
    n_body, dt, upd = best
    return {"value": upd / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{w.name}: initial {first_body} H gates + next {n_body} gates, "
                      f"{upd} updates in {dt:.1f} s, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2105_01533_amd import sim, workloads as W

    fn, desc = WORKLOADS[args.workload]
    w = getattr(W, fn)()
    log(f"[bench] workload {w.name}: {len(w.ops)} ops, capacity {w.capacity}")
    s = sim.Simulator(w.n_qubits, w.capacity, w.eps)
    gates = sim.sim_gates_from_ops(w.ops)
    for i in range(args.warmup):
        s.set_basis(*w.basis)
        _, _, st = s.apply_gates(gates)
        log(f"[bench] warmup {i}: {st}")
    torch.cuda.synchronize()
    updates = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        s.set_basis(*w.basis)
        _, _, st = s.apply_gates(gates)
        updates += st["updates"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps in {dt:.3f} s; last stats {st}")
    value = updates / dt
    out = {
        "metric": "nonzero-amplitude gate updates/s",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "description": desc, "n_qubits": w.n_qubits,
                   "ops": int(len(w.ops)), "capacity": w.capacity, "eps": w.eps,
                   "updates_per_step": st["updates"], "peak_nnz": st["peak_nnz"]},
        "roofline": None,
    }
    s.close()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
