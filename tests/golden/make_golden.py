"""Write the oracle's results for the full-size workloads whose oracle run is
too slow to repeat inside a test (config 1: 64-qubit adder, ~1 min; config 3:
40-qubit Trotter step, ~2.5 min; the same Trotter step as native Pauli
terms, ~20 s; the first three measurement rounds of the 100-qubit random
circuit at 2^24 entries, about an hour on eight threads).  Calls only the
oracle and the workload generators; run from the repository root:

    python tests/golden/make_golden.py            # configs 1 and 3
    python tests/golden/make_golden.py config2    # the random circuit's rounds

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

from oracle import Oracle, run_pauli_workload, run_workload  # noqa: E402
from paper_2105_01533_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLES = 1024


def keys_digest(lo: np.ndarray, hi: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(lo, "<u8").tobytes() + np.ascontiguousarray(hi, "<u8").tobytes()
                          ).hexdigest()


def state_digest(o, n_samples: int = N_SAMPLES) -> dict:
    """Entry count, label hash, norm and every stride-th sorted entry."""
    lo, hi, amp = o.export()
    stride = max(1, len(lo) // n_samples)
    idx = np.arange(0, len(lo), stride)[:n_samples]
    return {
        "nnz": int(len(lo)), "keys_sha256": keys_digest(lo, hi),
        "norm2": float(np.sum(np.abs(amp) ** 2)).hex(), "stride": int(stride),
        "samples": [[int(lo[i]), int(hi[i]), float(amp[i].real).hex(), float(amp[i].imag).hex()] for i in idx],
    }


def golden_config2_rounds(rounds: int = 3, threads: int = 0):
    """The 100-qubit random circuit (2^24 entries, 20,000 gates per round,
    then 8 measurements), run by the oracle with its Sec. 5 threads.  For
    each of the first `rounds` rounds the file holds the state just before
    the round's measurements (2^24 entries after the first round's fused
    runs; rounds 2 and 3 regrow from the collapsed state through branching
    gates) and the state after them, the outcomes, each measurement's P0 and
    P1, and the cumulative counters."""
    w = W.config2()
    ops = w.ops
    meas = np.nonzero(ops["kind"] == W.K_MEASURE)[0]
    o = Oracle(w.n_qubits, w.eps)
    used = o.set_threads(threads)
    o.set_basis(*w.basis)
    t0 = time.time()
    doc = {"workload": w.name, "seed": w.meta["seed"], "n_qubits": w.n_qubits, "eps": w.eps,
           "n_ops": int(len(ops)), "oracle_threads": int(used), "rounds": []}
    start = 0
    for r in range(rounds):
        m0 = int(meas[8 * r])
        m1 = int(meas[8 * r + 7]) + 1
        o.run(ops[start:m0])
        tot = o.totals()
        pre = state_digest(o, 4 * N_SAMPLES)
        pre.update({"op_end": m0, "updates": int(tot["updates"]), "u2_applied": int(tot["u2_applied"]),
                    "u2_skipped": int(tot["u2_skipped"]), "peak_nnz": int(tot["peak_nnz"]),
                    "pruned": int(tot["pruned"])})
        outcomes, tr = o.run(ops[m0:m1], trace=True)
        tot = o.totals()
        post = state_digest(o, 4 * N_SAMPLES)
        post.update({"op_end": m1, "updates": int(tot["updates"]),
                     "outcomes": [int(x) for x in outcomes],
                     "u": [float(x).hex() for x in ops["param"][m0:m1]],
                     "p0": [float(x).hex() for x in tr["p0"]], "p1": [float(x).hex() for x in tr["p1"]]})
        doc["rounds"].append({"pre_measure": pre, "post_measure": post})
        print(f"round {r + 1}: pre nnz {pre['nnz']}, post nnz {post['nnz']}, outcomes {post['outcomes']}, "
              f"{time.time() - t0:.0f} s", flush=True)
        start = m1
    doc["oracle_seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, "config2_rounds.json"), "w") as f:
        json.dump(doc, f, indent=0)


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
    if sys.argv[1:] == ["config2"]:
        golden_config2_rounds()
        sys.exit(0)
    golden("config1_full", W.config1())
    golden("config3_full", W.config3())
    golden("config3_native_full", W.config3_terms())
