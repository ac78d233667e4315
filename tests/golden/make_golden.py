"""Write the oracle's results for the full-size workloads whose oracle run is
too slow to repeat inside a test (config 1: 64-qubit adder, ~1 min; config 3:
40-qubit Trotter step, ~2.5 min; the same Trotter step as native Pauli
terms, ~20 s).  Calls only the oracle and the workload
generators; run from the repository root:

    python tests/golden/make_golden.py

Each JSON file holds the entry count, a SHA-256 of the sorted labels (lo
words then hi words, little-endian uint64), the measurement outcomes, the
update counters, and every `stride`-th sorted entry with its amplitude as
exact hex floats.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import run_pauli_workload, run_workload  # noqa: E402
from paper_2105_01533_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLES = 1024


def keys_digest(lo: np.ndarray, hi: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(lo, "<u8").tobytes() + np.ascontiguousarray(hi, "<u8").tobytes()
                          ).hexdigest()


def golden(name: str, w):
    t0 = time.time()
    if isinstance(w, W.PauliWorkload):
        o, _ = run_pauli_workload(w)
        outcomes, n_ops = [], len(w.terms)
    else:
        o, outcomes, _ = run_workload(w)
        n_ops = len(w.ops)
    lo, hi, amp = o.export()
    tot = o.totals()
    stride = max(1, len(lo) // N_SAMPLES)
    idx = np.arange(0, len(lo), stride)[:N_SAMPLES]
    doc = {
        "workload": name, "seed": w.meta.get("seed"), "n_qubits": w.n_qubits, "eps": w.eps,
        "n_ops": n_ops, "nnz": int(len(lo)), "keys_sha256": keys_digest(lo, hi),
        "norm2": float(np.sum(np.abs(amp) ** 2)).hex(),
        "outcomes": [int(x) for x in outcomes],
        "updates": int(tot["updates"]), "u2_applied": int(tot["u2_applied"]),
        "u2_skipped": int(tot["u2_skipped"]), "peak_nnz": int(tot["peak_nnz"]),
        "stride": int(stride),
        "samples": [[int(lo[i]), int(hi[i]), float(amp[i].real).hex(), float(amp[i].imag).hex()] for i in idx],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(doc, f, indent=0)
    print(name, doc["nnz"], doc["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    golden("config1_full", W.config1())
    golden("config3_full", W.config3())
    golden("config3_native_full", W.config3_terms())
