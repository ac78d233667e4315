"""Summaries of rocprofv3 runs of bench.py, for the committed profiles.

  stats   <kernel-trace dir> <out.md> <command> [<title>]
          per-kernel calls / total / average duration
  sq      <counter dir> [<counter dir> ...] <out.md> <title> <command...>
          per-kernel SQ counters per dispatch (one counter run per dir) and,
          for the fused pass, instructions per wave and issue shares
  traffic <FETCH_SIZE dir> <WRITE_SIZE dir> <out.md> <out.json> <workload> <command...>
          per-kernel KiB per dispatch from the two counter runs, scaled by what
          the same counters read for the reference copy kernel (k_copy16, which
          moves a known number of bytes each way), and the fused pass's HBM
          bytes per launch with a SHA-256 of its sources (bench.py reports the
          figure only while they are unchanged).

Reads the SQLite database (kernel trace) or the counter-collection CSV that
rocprofv3 writes; runs on the host after the GPU run.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
FUSED_PREFIXES = ("k_mono_rp<", "k_mono_bs<", "k_mono<")
FUSED_SOURCES = ["paper_2105_01533_amd/csrc/mono_regplane.hip", "paper_2105_01533_amd/csrc/regplane_tile.h",
                 "paper_2105_01533_amd/csrc/mono_bitslice.hip", "paper_2105_01533_amd/csrc/bitslice_tile.h",
                 "paper_2105_01533_amd/csrc/sim_kernels.hip", "paper_2105_01533_amd/csrc/run_compiler.hip"]
COPY_BYTES = 1 << 30


def is_fused(k: str) -> bool:
    return k.startswith(FUSED_PREFIXES)


def short(name: str) -> str:
    return name.replace("sparsesim::(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def sources_sha256() -> str:
    h = hashlib.sha256()
    for s in FUSED_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_stats(trace_dir: str) -> dict:
    dbs = glob.glob(os.path.join(trace_dir, "**", "*.db"), recursive=True)
    if not dbs:
        raise SystemExit(f"no kernel-trace database under {trace_dir}")
    agg = collections.defaultdict(lambda: [0, 0.0, float("inf"), 0.0])
    for db in dbs:
        con = sqlite3.connect(db)
        for name, start, end in con.execute("select name, start, end from kernels"):
            ms = (end - start) * 1e-6
            a = agg[short(name)]
            a[0] += 1
            a[1] += ms
            a[2] = min(a[2], ms)
            a[3] = max(a[3], ms)
        con.close()
    return dict(agg)


def write_stats(trace_dir: str, out_md: str, command: str, title: str):
    agg = kernel_stats(trace_dir)
    total = sum(v[1] for v in agg.values())
    lines = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "```", command, "```", "",
             "| kernel | calls | total ms | avg ms | min ms | max ms | share |", "|---|---:|---:|---:|---:|---:|---:|"]
    for k, (n, t, lo, hi) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{k}` | {n} | {t:.3f} | {t / n:.4f} | {lo:.4f} | {hi:.4f} | {100 * t / total:.1f}% |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return agg


def counter(dir_: str, name: str) -> dict:
    files = glob.glob(os.path.join(dir_, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter CSV under {dir_}")
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == name:
                    per[short(r["Kernel_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in per.items()}   # (dispatches, KiB per dispatch)


def write_traffic(fetch_dir: str, write_dir: str, out_md: str, out_json: str, commands: list[str], workload: str):
    fe, wr = counter(fetch_dir, "FETCH_SIZE"), counter(write_dir, "WRITE_SIZE")
    if "k_copy16" not in fe or "k_copy16" not in wr:
        raise SystemExit("the counter runs need the reference copy (bench.py --calibrate-copy)")
    fs = COPY_BYTES / (fe["k_copy16"][1] * 1024)
    ws = COPY_BYTES / (wr["k_copy16"][1] * 1024)
    launches = sum(fe[k][0] for k in fe if is_fused(k))
    rd = sum(fe[k][0] * fe[k][1] * 1024 * fs for k in fe if is_fused(k)) / max(launches, 1)
    wt = sum(wr[k][0] * wr[k][1] * 1024 * ws for k in wr if is_fused(k)) / max(launches, 1)
    doc = {"kernel": "mono_pass", "workload": workload, "launches": launches, "fetch_scale": fs, "write_scale": ws,
           "traffic_bytes_per_launch": rd + wt, "fetch_bytes_per_launch": rd, "write_bytes_per_launch": wt,
           "sources": FUSED_SOURCES, "sources_sha256": sources_sha256()}
    with open(out_json, "w") as f:
        json.dump(doc, f, indent=1)
    lines = [f"# HBM traffic, fused phase/permutation pass, {workload} (one step)", "",
             "Two counter runs (one counter each), from the repository root on one MI355X:", "", "```", *commands, "```",
             "", f"Calibration: `--calibrate-copy` first runs `sim_device_copy` (a plain 16-byte-per-thread streaming "
             f"copy) of 1 GiB three times. Per dispatch it reads FETCH_SIZE = {fe['k_copy16'][1]:.0f} KiB and "
             f"WRITE_SIZE = {wr['k_copy16'][1]:.0f} KiB against 1,048,576 KiB moved each way, so FETCH_SIZE is "
             f"scaled by {fs:.3f} and WRITE_SIZE by {ws:.3f}.", "",
             "Per kernel (KiB per dispatch, raw counter values):", "",
             "| kernel | dispatches | FETCH_SIZE | WRITE_SIZE |", "|---|---:|---:|---:|"]
    for k in sorted(set(fe) | set(wr), key=lambda k: -(fe.get(k, (0, 0))[1] * fe.get(k, (0, 0))[0])):
        n = fe.get(k, wr.get(k))[0]
        lines.append(f"| `{k}` | {n} | {fe.get(k, (0, 0.0))[1]:.1f} | {wr.get(k, (0, 0.0))[1]:.1f} |")
    lines += ["", f"Fused pass (all {launches} launches of `k_mono_rp` and `k_mono`): scaled traffic "
              f"{(rd + wt) / 1e6:.1f} MB per launch ({rd / 1e6:.1f} MB read, {wt / 1e6:.1f} MB written).", "",
              "`profiles/mono_pass_traffic.json` holds the per-launch figure with a SHA-256 of the fused-pass "
              "sources; the bench reports `traffic` only while those sources are unchanged."]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return doc


def counters_all(dirs: list[str]) -> dict:
    """{kernel: {counter: (dispatches, value per dispatch)}} over counter runs."""
    out = collections.defaultdict(dict)
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter CSV under {d}")
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        for fn in files:
            with open(fn) as f:
                for r in csv.DictReader(f):
                    per[(short(r["Kernel_Name"]), r["Counter_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
        for (k, c), v in per.items():
            out[k][c] = (len(v), sum(v.values()) / len(v))
    return out


def write_sq(dirs: list[str], out_md: str, title: str, commands: list[str]):
    agg = counters_all(dirs)
    names = sorted({c for v in agg.values() for c in v})
    lines = [f"# {title}", "", "Counter runs (one per line, each with its own set of SQ counters), from the repository "
             "root on one MI355X:", "", "```", *commands, "```", "",
             "Per kernel, counter value per dispatch (SQ_*_CYCLES and SQ_WAIT_* are in units of four cycles, "
             "summed over waves):", "", "| kernel | dispatches | " + " | ".join(n.replace("SQ_", "") for n in names) + " |",
             "|---|---:|" + "---:|" * len(names)]
    for k in sorted(agg, key=lambda k: -agg[k].get("SQ_WAVE_CYCLES", (0, 0))[1]):
        d = next(iter(agg[k].values()))[0]
        lines.append(f"| `{k}` | {d} | " + " | ".join(f"{agg[k][n][1]:.4g}" if n in agg[k] else "" for n in names) + " |")
    fused = [k for k in agg if is_fused(k) and "SQ_WAVES" in agg[k]]
    if fused:
        lines += ["", "Fused pass, summed over its kernels (per wave):", ""]
        def tot(c):
            return sum(agg[k][c][0] * agg[k][c][1] for k in fused if c in agg[k])
        waves = tot("SQ_WAVES")
        insts = {c: tot(c) for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_SMEM",
                                    "SQ_INSTS_BRANCH", "SQ_INSTS_VMEM") if any(c in agg[k] for k in fused)}
        n_all = sum(insts.values())
        for c, v in insts.items():
            lines.append(f"- {c}: {v / waves:.4g} per wave ({100 * v / n_all:.1f} % of the instructions counted)")
        for c in ("SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU",
                  "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_ANY"):
            if any(c in agg[k] for k in fused):
                lines.append(f"- {c}: {tot(c) / waves:.4g} per wave")
        if "SQ_WAVE_CYCLES" in agg[fused[0]]:
            wc = tot("SQ_WAVE_CYCLES")
            lines.append(f"- instructions per wave-cycle (x4 cycles): {n_all / wc:.3f}")
            for c in ("SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS"):
                if any(c in agg[k] for k in fused):
                    lines.append(f"- {c} / SQ_WAVE_CYCLES: {tot(c) / wc:.3f}")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        write_stats(argv[1], argv[2], argv[3], argv[4] if len(argv) > 4 else "Kernel time")
    elif len(argv) >= 5 and argv[0] == "sq":
        # sq <dir>... <out.md> <title> <command...>: dirs are the leading
        # arguments that exist as directories.
        k = 1
        while k < len(argv) and os.path.isdir(argv[k]):
            k += 1
        write_sq(argv[1:k], argv[k], argv[k + 1], argv[k + 2:])
    elif len(argv) >= 6 and argv[0] == "traffic":
        write_traffic(argv[1], argv[2], argv[3], argv[4], argv[6:], argv[5])
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
