"""Summaries of rocprofv3 output for the measurement records kept with the project.

* ``stats_markdown``: the ``--kernel-trace --stats`` kernel table as a short markdown table.
* ``traffic_record``: HBM bytes per launch of one kernel from two ``--pmc`` runs (FETCH_SIZE,
  then WRITE_SIZE, both in KiB per dispatch), each scaled by what the same counter reads for a
  plain device copy of known size run in the same process (the rocclr copy kernel that
  ``bench.py --calib-copy-mib`` issues).

    python -m paper_2604_02624_amd.profiling stats <kernel_stats.csv> <command...>
    python -m paper_2604_02624_amd.profiling traffic <fetch.csv> <write.csv> <copy_mib> \\
        <kernel substring> <pass name> <workload> <column variant> <column radix plan> <command...>
    python -m paper_2604_02624_amd.profiling counters <A.csv> <B.csv> <fetch.csv> <write.csv> \\
        <copy_mib> <kernel substring> <command...>
    python -m paper_2604_02624_amd.profiling valu <V1.csv> <V2.csv> <kernel substring> <command...>
    python -m paper_2604_02624_amd.profiling lds <counters.csv> <command...>
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the sources that define the pass kernels (their code, launch shapes and argument structs); a
# traffic record taken on other versions of them no longer describes the kernel
KERNEL_SOURCES = ["paper_2604_02624_amd/csrc/pass_kernels.hpp", "paper_2604_02624_amd/csrc/dpx_pass.hip",
                  "paper_2604_02624_amd/csrc/fft.hpp", "paper_2604_02624_amd/csrc/phase.hpp",
                  "paper_2604_02624_amd/csrc/dpx_internal.hpp"]


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
                   command: str, workload: int = 4, column_variant: str = "", column_plan: str = "") -> dict:
    """The record names the benchmark workload and column configuration it was taken on; bench.py
    reports it only for that workload and configuration (and only on the same kernel sources)."""
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
        kernel=kernel_sub, pass_name=pass_name, workload=workload, column_variant=column_variant,
        column_radix_plan=column_plan, kernel_source_sha=kernel_source_sha(),
        command=command, copy_bytes=copy_bytes,
        fetch_scale=round(f_scale, 4), write_scale=round(w_scale, 4),
        launches=len(fk),
        fetch_bytes_per_launch=int(sum(fk) / max(len(fk), 1)),
        write_bytes_per_launch=int(sum(wk) / max(len(wk), 1)),
        hbm_bytes_per_launch=int((sum(fk) + sum(wk)) / max(len(fk), 1)),
    )


def _dispatch_counters(csv_path: str):
    """{dispatch: {counter: summed value, "_kernel": name, "_ns": duration}}"""
    out = defaultdict(lambda: defaultdict(float))
    for r in csv.DictReader(open(csv_path)):
        d = out[int(r["Dispatch_Id"])]
        d[r["Counter_Name"]] += float(r["Counter_Value"])
        d["_kernel"] = r["Kernel_Name"]
        d["_ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    return out


def counters_markdown(a_csv: str, b_csv: str, fetch_csv: str, write_csv: str, copy_mib: int,
                      kernel_filter: str, command: str, n_cu: int = 256, n_xcd: int = 8) -> str:
    """Per-kernel table from four counter passes over the same program: A (SQ_WAVES
    SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_WAIT_INST_LDS
    SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE GRBM_GUI_ACTIVE), B (SQ_INSTS_LDS SQ_WAIT_ANY ...),
    FETCH_SIZE and WRITE_SIZE.  Averages over the dispatches of each kernel."""
    A, B = _dispatch_counters(a_csv), _dispatch_counters(b_csv)
    F, W = _dispatch_counters(fetch_csv), _dispatch_counters(write_csv)
    copy_bytes = copy_mib * (1 << 20)

    def copy_scale(rows, counter):
        big = [d[counter] * 1024 for d in rows.values() if "copyBuffer" in d["_kernel"]]
        return copy_bytes / max(big) if big else 1.0

    fs, ws = copy_scale(F, "FETCH_SIZE"), copy_scale(W, "WRITE_SIZE")
    per = defaultdict(list)
    for k, a in A.items():
        name = a["_kernel"]
        if kernel_filter not in name:
            continue
        b = B.get(k, {})
        cyc = a["GRBM_GUI_ACTIVE"] / n_xcd  # GRBM counts once per XCD
        waves = max(a["SQ_WAVES"], 1.0)
        per[name].append(dict(
            ms=a["_ns"] / 1e6, clock=cyc / max(a["_ns"], 1) , valu=a["SQ_ACTIVE_INST_VALU"] / (n_cu * cyc),
            vi=a["SQ_INSTS_VALU"] / waves, li=b.get("SQ_INSTS_LDS", 0.0) / waves,
            vm=b.get("SQ_INSTS_VMEM_RD", 0.0) / waves,
            wait=b.get("SQ_WAIT_ANY", 0.0) / max(a["SQ_WAVE_CYCLES"], 1.0),
            conf=a["SQ_LDS_BANK_CONFLICT"] / max(a["SQ_LDS_IDX_ACTIVE"], 1.0),
            rd=F.get(k, {}).get("FETCH_SIZE", 0.0) * 1024 * fs / 1e9,
            wr=W.get(k, {}).get("WRITE_SIZE", 0.0) * 1024 * ws / 1e9))
    rows = ["| kernel | launches | ms | clock GHz | VALU busy | VALU instr / wave | LDS instr / wave | "
            "VMEM rd / wave | wave time waiting | LDS conflict cycles | HBM read GB | HBM write GB |",
            "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(x["ms"] for x in kv[1])):
        m = {key: sum(x[key] for x in v) / len(v) for key in v[0]}
        rows.append(f"| `{name[:60]}` | {len(v)} | {m['ms']:.2f} | {m['clock']:.2f} | {100 * m['valu']:.0f}% | "
                    f"{m['vi']:.0f} | {m['li']:.0f} | {m['vm']:.0f} | {100 * m['wait']:.0f}% | "
                    f"{100 * m['conf']:.0f}% | {m['rd']:.2f} | {m['wr']:.2f} |")
    note = (f"VALU busy = SQ_ACTIVE_INST_VALU / ({n_cu} CUs x GRBM_GUI_ACTIVE / {n_xcd} XCDs); clock = "
            f"GRBM_GUI_ACTIVE / {n_xcd} / duration; wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES; LDS conflict = "
            f"SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE.  HBM bytes: FETCH_SIZE x {fs:.2f} and WRITE_SIZE x "
            f"{ws:.2f} (a {copy_mib} MiB device copy in the same process calibrates both).")
    return "\n".join([f"Command (four passes): `{command}`", "", note, "", *rows, ""])


VALU_TYPES = ["SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32",
              "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64",
              "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64", "SQ_INSTS_VALU_CVT"]


def valu_types_markdown(v1_csv: str, v2_csv: str, kernel_filter: str, command: str, top: int = 6) -> str:
    """Vector instructions per wave by type, from two counter passes (the FP32 / FP64 adds,
    multiplies, fused multiply-adds and transcendentals; then INT32, INT64, conversions, all
    VALU, SQ_WAVES, LDS, SALU, VMEM reads), summed over the dispatches of each kernel."""
    V1, V2 = _dispatch_counters(v1_csv), _dispatch_counters(v2_csv)
    agg = defaultdict(lambda: defaultdict(float))
    for D in (V1, V2):
        for d in D.values():
            if kernel_filter not in d["_kernel"]:
                continue
            for c, v in d.items():
                if not c.startswith("_"):
                    agg[d["_kernel"]][c] += v
    rows = ["| kernel | VALU / wave | F32 add | F32 mul | F32 fma | F32 trans | F64 add | F64 mul | F64 fma | "
            "F64 trans | INT32 | INT64 | cvt | other VALU | LDS / wave |",
            "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    order = sorted(agg, key=lambda k: -agg[k].get("SQ_INSTS_VALU", 0.0))[:top]
    for k in order:
        a = agg[k]
        w = max(a.get("SQ_WAVES", 0.0), 1.0)
        per = {c: a.get(c, 0.0) / w for c in VALU_TYPES + ["SQ_INSTS_VALU", "SQ_INSTS_LDS"]}
        other = per["SQ_INSTS_VALU"] - sum(per[c] for c in VALU_TYPES)
        cells = [per[c] for c in ("SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F32",
                                  "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                                  "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64",
                                  "SQ_INSTS_VALU_CVT")]
        rows.append(f"| `{k[:64]}` | {per['SQ_INSTS_VALU']:.0f} | " + " | ".join(f"{c:.0f}" for c in cells) +
                    f" | {other:.0f} | {per['SQ_INSTS_LDS']:.0f} |")
    return "\n".join([f"Command (two passes): `{command}`", "", *rows, ""])


# index patterns of probes/lds_bank_probe.hip (float2 slot of lane i), in its order
LDS_PATTERNS = [
    ("linear", lambda i: i),
    ("stride 2", lambda i: 2 * i),
    ("stride 4", lambda i: 4 * i),
    ("stride 16", lambda i: 16 * i),
    ("16-lane runs 32 apart", lambda i: i % 16 + 32 * (i // 16)),
    ("4-lane runs 64 apart", lambda i: i % 4 + 64 * (i // 4)),
    ("1024 stage-0 write, shift 5", lambda i: 8 * i + ((8 * i) >> 5)),
    ("1024 stage-0 write, shift 4", lambda i: 8 * i + ((8 * i) >> 4)),
    ("1024 stage-1 write, shift 5", lambda i: (i // 8) * 64 + i % 8 + (((i // 8) * 64 + i % 8) >> 5)),
    ("1024 stage-1 write, 8 per 64", lambda i: (i // 8) * 64 + i % 8 + (((i // 8) * 64 + i % 8) // 64) * 8),
    ("column staging, 1148-slot regions", lambda i: (i % 8) * 1148 + i // 8),
    ("column staging, 1146-slot regions", lambda i: (i % 8) * 1146 + i // 8),
]


def lds_write_model_cycles(slots) -> int:
    """Cycles of one 8-byte write of a wavefront under the model the probe fits: four groups of
    16 lanes, each group as many cycles as the most dwords that fall on one of 32 banks."""
    total = 0
    for q in range(4):
        banks = defaultdict(set)
        for a in slots[16 * q:16 * q + 16]:
            for d in (2 * a, 2 * a + 1):
                banks[d % 32].add(d)
        total += max(len(v) for v in banks.values())
    return total


def lds_markdown(csv_path: str, command: str) -> str:
    """Per pattern: LDS cycles and bank-conflict cycles per access of the probe's write and read
    kernels (the read kernel's 144 initial linear writes are taken out), next to the write model."""
    agg = defaultdict(lambda: defaultdict(float))
    for d in _dispatch_counters(csv_path).values():
        name = d["_kernel"]
        kind = "wr" if "wr_k<" in name else "rd" if "rd_k<" in name else None
        if kind is None:
            continue
        pat = int(name.split("<")[1].split(">")[0])
        for c in ("SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_LDS"):
            agg[(pat, kind)][c] += d[c]
    rows = ["| pattern | write cycles | write conflict cycles | model write cycles | read cycles | read conflict cycles |",
            "|---|---:|---:|---:|---:|---:|"]
    for p, (label, f) in enumerate(LDS_PATTERNS):
        w, r = agg.get((p, "wr")), agg.get((p, "rd"))
        if not w or not r:
            continue
        wi = w["SQ_INSTS_LDS"]
        # read kernel: 144 linear writes (4 cycles, no conflicts) per 2048 reads
        ri = r["SQ_INSTS_LDS"] * 2048 / 2192
        ract = (r["SQ_LDS_IDX_ACTIVE"] - 4 * r["SQ_INSTS_LDS"] * 144 / 2192) / ri
        rows.append(f"| {label} | {w['SQ_LDS_IDX_ACTIVE'] / wi:.2f} | {w['SQ_LDS_BANK_CONFLICT'] / wi:.2f} | "
                    f"{lds_write_model_cycles([f(i) for i in range(64)])} | {ract:.2f} | "
                    f"{r['SQ_LDS_BANK_CONFLICT'] / ri:.2f} |")
    return "\n".join([f"Command: `{command}`", "", *rows, ""])


def main(argv):
    if argv[0] == "stats":
        print(stats_markdown(argv[1], " ".join(argv[2:])))
    elif argv[0] == "counters":
        print(counters_markdown(argv[1], argv[2], argv[3], argv[4], int(argv[5]), argv[6], " ".join(argv[7:])))
    elif argv[0] == "valu":
        print(valu_types_markdown(argv[1], argv[2], argv[3], " ".join(argv[4:])))
    elif argv[0] == "lds":
        print(lds_markdown(argv[1], " ".join(argv[2:])))
    elif argv[0] == "traffic":
        rec = traffic_record(argv[1], argv[2], int(argv[3]), argv[4], argv[5], " ".join(argv[9:]),
                             workload=int(argv[6]), column_variant=argv[7], column_plan=argv[8])
        print(json.dumps(rec, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
