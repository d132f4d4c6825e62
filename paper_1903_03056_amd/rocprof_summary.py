"""Summarise rocprofv3 output of bench.py into short text files under profiles/.

    python -m paper_1903_03056_amd.rocprof_summary TRACE_DIR FETCH_DIR WRITE_DIR OUT_PREFIX
    python -m paper_1903_03056_amd.rocprof_summary --stats TRACE_DIR OUT_MD COMMAND...

TRACE_DIR holds the --kernel-trace --stats csv output, FETCH_DIR / WRITE_DIR the
--pmc FETCH_SIZE / --pmc WRITE_SIZE csv output of `bench.py --copy-probe`.  The
counters are calibrated against the plain device copy of the copy probe, whose true
traffic is known (256 MiB read, 256 MiB written): factor = true bytes / counter bytes.
Writes OUT_PREFIX_kernel_stats.md, OUT_PREFIX_hbm_counters.md and, for the gain kernel,
profiles/gain_kernel_traffic.json (read by bench.py while the kernel source is unchanged).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 * 1024 * 1024
COPY_KERNEL = "__amd_rocclr_copyBuffer"


GAIN_SOURCES = ("gain.hpp", "fft.hpp", "passes.hpp", "tiles_32.hip", "gain_mfma.hip")


def gain_source_digest() -> str:
    """SHA-256 over the sources the N=32 gain kernels (FFT and matrix-core) are compiled from."""
    h = hashlib.sha256()
    for name in GAIN_SOURCES:
        with open(os.path.join(ROOT, "paper_1903_03056_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _one(pattern):
    hits = glob.glob(pattern)
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def _counters(d, counter):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))))
    out = []
    for r in rows:
        if r["Counter_Name"] == counter:
            out.append((r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))   # KiB -> bytes
    return out


def short(name):
    name = name.replace("dgfs::", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def main(trace_dir, fetch_dir, write_dir, prefix, command):
    stats = list(csv.DictReader(open(_one(os.path.join(trace_dir, "*kernel_stats.csv")))))
    with open(prefix + "_kernel_stats.md", "w") as fh:
        fh.write(f"# rocprofv3 kernel statistics\n\nCommand:\n\n```\n{command['trace']}\n```\n\n")
        fh.write("| kernel | calls | average us | min us | max us | share % |\n|---|---|---|---|---|---|\n")
        for r in stats:
            fh.write(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |\n")
    fetch = _counters(fetch_dir, "FETCH_SIZE")
    write = _counters(write_dir, "WRITE_SIZE")
    fcopy = max(v for k, v in fetch if k == COPY_KERNEL)   # the 256 MiB probe copy
    wcopy = max(v for k, v in write if k == COPY_KERNEL)
    ff, fw = COPY_BYTES / fcopy, COPY_BYTES / wcopy
    with open(prefix + "_hbm_counters.md", "w") as fh:
        fh.write("# HBM traffic per dispatch (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n\nCommands:\n\n```\n"
                 f"{command['fetch']}\n{command['write']}\n```\n\n"
                 f"Calibration on the plain copy of 256 MiB: FETCH_SIZE reads {fcopy / 2**20:.1f} MiB "
                 f"(factor {ff:.3f}), WRITE_SIZE reads {wcopy / 2**20:.1f} MiB (factor {fw:.3f}).\n\n"
                 "| kernel | FETCH raw MiB | WRITE raw MiB | calibrated read MiB | calibrated write MiB |\n"
                 "|---|---|---|---|---|\n")
        for (k, fv), (k2, wv) in zip(fetch, write):
            if k != k2:
                continue
            fh.write(f"| `{short(k)}` | {fv / 2**20:.1f} | {wv / 2**20:.1f} | {fv * ff / 2**20:.1f} | "
                     f"{wv * fw / 2**20:.1f} |\n")
    gain = [(k, fv, wv) for (k, fv), (k2, wv) in zip(fetch, write) if "gain_kernel" in k and k == k2]
    if gain:
        kname, fv, wv = gain[-1]
        rec = {"kernel": short(kname),
               "workload": "256-node N=32 slab (bench.py)",
               "bytes_per_launch": fv * ff + wv * fw,
               "read_bytes": fv * ff, "write_bytes": wv * fw,
               "fetch_factor": ff, "write_factor": fw,
               "kernel_source_sha256": gain_source_digest(),
               "commands": command}
        with open(os.path.join(ROOT, "profiles", "gain_kernel_traffic.json"), "w") as fh:
            json.dump(rec, fh, indent=1)


def stats_only(trace_dir, out_path, command):
    """Kernel statistics alone (a workload without counter passes)."""
    stats = list(csv.DictReader(open(_one(os.path.join(trace_dir, "*kernel_stats.csv")))))
    with open(out_path, "w") as fh:
        fh.write(f"# rocprofv3 kernel statistics\n\nCommand:\n\n```\n{command}\n```\n\n")
        fh.write("| kernel | calls | average us | min us | max us | share % |\n|---|---|---|---|---|---|\n")
        for r in stats:
            fh.write(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |\n")


if __name__ == "__main__":
    if sys.argv[1] == "--stats":
        # python -m paper_1903_03056_amd.rocprof_summary --stats TRACE_DIR OUT_MD COMMAND...
        stats_only(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
        sys.exit(0)
    t, f, w, p = sys.argv[1:5]
    cmds = {
        "trace": "rocprofv3 --kernel-trace --stats -d DIR -o trace --output-format csv -- "
                 "python3 bench.py --steps 20 --warmup 2 --no-cpu-baseline --no-plain --no-extra",
        "fetch": "rocprofv3 --pmc FETCH_SIZE -d DIR -o fetch --output-format csv -- "
                 "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-plain --no-extra --copy-probe",
        "write": "rocprofv3 --pmc WRITE_SIZE -d DIR -o write --output-format csv -- "
                 "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-plain --no-extra --copy-probe",
    }
    main(t, f, w, p, cmds)
