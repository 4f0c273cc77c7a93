"""Summaries of rocprofv3 output for the measurement records kept with the project.

* ``stats_markdown``: the ``--kernel-trace --stats`` kernel table as a short markdown table.
* ``traffic_record``: HBM bytes per launch of one kernel from two ``--pmc`` runs (FETCH_SIZE,
  then WRITE_SIZE, both in KiB per dispatch), each scaled by what the same counter reads for a
  plain device copy of known size run in the same process (the rocclr copy kernel that
  ``bench.py --calib-copy-mib`` issues).

    python -m paper_2604_02624_amd.profiling stats <kernel_stats.csv> <command...>
    python -m paper_2604_02624_amd.profiling traffic <fetch.csv> <write.csv> <copy_mib> \\
        <kernel substring> <pass name> <command...>
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2604_02624_amd/csrc/pass_kernels.hpp", "paper_2604_02624_amd/csrc/dpx_pass.hip",
                  "paper_2604_02624_amd/csrc/dpx_kernels.hip", "paper_2604_02624_amd/csrc/fft.hpp",
                  "paper_2604_02624_amd/csrc/phase.hpp"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats_markdown(stats_csv: str, command: str, top: int = 14) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join([f"Command: `{command}`", "", *out, ""])


def _per_dispatch(csv_path: str, counter: str):
    vals = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        k = int(r["Dispatch_Id"])
        vals[k] += float(r["Counter_Value"])
        names[k] = r["Kernel_Name"]
    return [(k, names[k], vals[k]) for k in sorted(vals)]


def traffic_record(fetch_csv: str, write_csv: str, copy_mib: int, kernel_sub: str, pass_name: str,
                   command: str) -> dict:
    copy_bytes = copy_mib * (1 << 20)
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")

    def copy_value(rows):
        big = [v for _, n, v in rows if "copyBuffer" in n]
        return max(big) * 1024 if big else None

    cf, cw = copy_value(fetch), copy_value(write)
    f_scale = copy_bytes / cf if cf else 1.0
    w_scale = copy_bytes / cw if cw else 1.0
    fk = [v * 1024 * f_scale for _, n, v in fetch if kernel_sub in n]
    wk = [v * 1024 * w_scale for _, n, v in write if kernel_sub in n]
    return dict(
        kernel=kernel_sub, pass_name=pass_name, kernel_source_sha=kernel_source_sha(),
        command=command, copy_bytes=copy_bytes,
        fetch_scale=round(f_scale, 4), write_scale=round(w_scale, 4),
        launches=len(fk),
        fetch_bytes_per_launch=int(sum(fk) / max(len(fk), 1)),
        write_bytes_per_launch=int(sum(wk) / max(len(wk), 1)),
        hbm_bytes_per_launch=int((sum(fk) + sum(wk)) / max(len(fk), 1)),
    )


def main(argv):
    if argv[0] == "stats":
        print(stats_markdown(argv[1], " ".join(argv[2:])))
    elif argv[0] == "traffic":
        rec = traffic_record(argv[1], argv[2], int(argv[3]), argv[4], argv[5], " ".join(argv[6:]))
        print(json.dumps(rec, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
