"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2310_00810_amd.profiling trace <stats.csv> <out.md> "<command>"
    python -m paper_2310_00810_amd.profiling traffic <fetch_counters.csv> <write_counters.csv> \
        <copy_bytes> <out.json> <out.md> "<command>"
    python -m paper_2310_00810_amd.profiling sq <sq_counters.csv> <out.md> "<command>"
    python -m paper_2310_00810_amd.profiling overlap <kernel_trace.csv> <out.md>
    python -m paper_2310_00810_amd.profiling mfma <counters.csv> <out.md> "<command>"

`trace` turns a `--kernel-trace --stats --output-format csv` kernel-stats file
into a Markdown table.  `traffic` turns two `--pmc FETCH_SIZE` / `--pmc
WRITE_SIZE` counter-collection files into HBM bytes per launch of each LBM
kernel.  Each counter is scaled by what it reads for the largest plain copy
kernel in the same run (a device-to-device copy of `copy_bytes` bytes: it
reads and writes exactly that many bytes), so FETCH_SIZE / WRITE_SIZE units
and granularity drop out.  The JSON carries the hash of the kernel sources it
was measured on; the benchmark reports the figure only while that hash still
matches.  `sq` turns a run of SQ_* instruction counters into per-wavefront
counts per kernel, with the VALU issue time they imply (a wave64 VALU
instruction occupies a 16-lane SIMD for 4 cycles; 1024 SIMDs at 2.4 GHz).
"""
import csv
import collections
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("lbm_device.hpp", "lbm_kernels.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    n = name.split("(")[0]
    for pre in ("void ", "lbm::", "nn::"):
        n = n.replace(pre, "")
    return n


def trace(stats_csv, out_md, command):
    rows = list(csv.DictReader(open(stats_csv)))
    with open(out_md, "w") as f:
        f.write(f"# rocprofv3 kernel statistics\n\nCommand:\n\n    {command}\n\n")
        f.write("| kernel | calls | total (us) | average (us) | min (us) | max (us) | % |\n|---|---|---|---|---|---|---|\n")
        for r in rows[:20]:
            f.write(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.0f} | "
                    f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                    f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |\n")


def overlap(trace_csv, out_md, top=6):
    """Appends to out_md each kernel's average duration split by whether its
    dispatch ran alone or overlapped another dispatch in time (a recompute on
    the second stream beside the adjoint stretches both), from a
    --kernel-trace dispatch file."""
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
                for r in csv.DictReader(open(trace_csv)))
    # sorted by start, dispatch i overlaps another iff an earlier one ends after it starts or the
    # next one starts before it ends
    beside = [False] * len(ev)
    prefix_end = -1
    for i, (s0, e0, _) in enumerate(ev):
        beside[i] = prefix_end > s0 or (i + 1 < len(ev) and ev[i + 1][0] < e0)
        prefix_end = max(prefix_end, e0)
    acc = collections.defaultdict(lambda: [0, 0.0, 0, 0.0])
    for (s0, e0, name), b in zip(ev, beside):
        a = acc[name]
        a[2 * b] += 1
        a[2 * b + 1] += (e0 - s0) / 1e3
    names = sorted(acc, key=lambda k: -(acc[k][1] + acc[k][3]))[:top]
    with open(out_md, "a") as f:
        f.write("\nDispatches that ran alone and dispatches that overlapped another one in time:\n\n"
                "| kernel | alone: calls | alone: average (us) | overlapped: calls | overlapped: average (us) |\n"
                "|---|---|---|---|---|\n")
        for k in names:
            n0, t0, n1, t1 = acc[k]
            f.write(f"| `{k}` | {n0} | {t0 / max(n0, 1):.2f} | {n1} | {t1 / max(n1, 1):.2f} |\n")


def _per_kernel(path):
    agg = collections.defaultdict(list)
    copies = []
    for r in csv.DictReader(open(path)):
        v = float(r["Counter_Value"])
        name = r["Kernel_Name"]
        if "copyBuffer" in name:
            copies.append(v)
        agg[short_name(name)].append(v)
    return agg, max(copies) if copies else None


def traffic(fetch_csv, write_csv, copy_bytes, out_json, out_md, command):
    fa, fcopy = _per_kernel(fetch_csv)
    wa, wcopy = _per_kernel(write_csv)
    if not fcopy or not wcopy:
        raise SystemExit("no copy kernel in the counter runs")
    fs, ws = copy_bytes / fcopy, copy_bytes / wcopy
    out = {"source_hash": kernel_source_hash(), "copy_bytes": copy_bytes,
           "fetch_scale_bytes_per_unit": fs, "write_scale_bytes_per_unit": ws, "command": command}
    lines = []
    for k in sorted(fa):
        if not (k.startswith("k_step") or k.startswith("k_adj")):
            continue
        fb = sum(fa[k]) / len(fa[k]) * fs
        wb = sum(wa.get(k, [0])) / max(len(wa.get(k, [1])), 1) * ws
        out[k] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb, "launches": len(fa[k]),
                  "source_hash": out["source_hash"]}
        lines.append(f"| `{k}` | {len(fa[k])} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} |")
    json.dump(out, open(out_json, "w"), indent=1)
    with open(out_md, "w") as f:
        f.write("# HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n\n")
        f.write(f"Commands (two runs, one counter each):\n\n    {command}\n\n")
        f.write(f"Calibration: the largest device copy in the run moves {copy_bytes / 2**30:.0f} GiB each way; "
                f"FETCH_SIZE scale {fs:.1f} B/unit, WRITE_SIZE scale {ws:.1f} B/unit.  Kernel source hash "
                f"{out['source_hash']}.\n\n")
        f.write("| kernel | launches | fetched MB | written MB | total MB |\n|---|---|---|---|---|\n")
        f.write("\n".join(lines) + "\n")


def sq(counters_csv, out_md, command):
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(counters_csv)):
        agg[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = ["SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
             "SQ_INSTS_SMEM"]
    with open(out_md, "w") as f:
        f.write("# Instructions per wavefront (rocprofv3 SQ counters)\n\n")
        f.write(f"Command:\n\n    {command}\n\n")
        f.write("| kernel | waves | " + " | ".join(n[9:] for n in names) + " | VALU issue time (us) |\n")
        f.write("|---" * (len(names) + 3) + "|\n")
        for k in sorted(agg):
            if not (k.startswith("k_step") or k.startswith("k_adj")):
                continue
            m = {c: sum(v) / len(v) for c, v in agg[k].items()}
            w = m.get("SQ_WAVES", 0.0)
            if not w:
                continue
            valu_us = w * m.get("SQ_INSTS_VALU", 0.0) / w * 4 / 1024 / 2.4e9 * 1e6
            f.write(f"| `{k}` | {w:.0f} | " + " | ".join(f"{m.get(n, 0.0) / w:.0f}" for n in names) +
                    f" | {valu_us:.1f} |\n")


def mfma(counters_csv, out_md, command, prefixes=("k_conv", "k_wgrad")):
    """Per network kernel: BF16 MFMA rate and LDS counters.  TFLOP/s =
    SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512 flop over the dispatches' own
    durations (start / end timestamps of the counter rows), and its fraction
    of the 2.5 PFLOP/s dense peak; MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES /
    (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs): GRBM_GUI_ACTIVE comes summed over the
    8 XCDs (it reads about 8 x the clock times the duration); LDS
    bank-conflict cycles per LDS instruction; LDS wait cycles per wavefront."""
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    calls = collections.Counter()
    for r in csv.DictReader(open(counters_csv)):
        k = short_name(r["Kernel_Name"])
        if not k.startswith(prefixes):
            continue
        agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
        if r["Counter_Name"] == "SQ_WAVES":
            calls[k] += 1
            agg[k]["duration_ns"] += float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    with open(out_md, "w") as f:
        f.write("# MFMA and LDS counters of the network kernels (rocprofv3)\n\n")
        f.write(f"Command:\n\n    {command}\n\n")
        f.write("| kernel | launches | waves / launch | avg launch (us) | BF16 TFLOP/s | of peak | MFMA busy "
                "| LDS insts / wave | bank-conflict cycles / LDS inst | LDS wait cycles / wave |\n"
                "|---|---|---|---|---|---|---|---|---|---|\n")
        for k in sorted(agg, key=lambda k: -agg[k].get("duration_ns", 0.0)):
            m = agg[k]
            w = m.get("SQ_WAVES", 0.0)
            if not w:
                continue
            gui = m.get("GRBM_GUI_ACTIVE", 0.0)
            mb = m.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) * 8 / (gui * 1024) if gui else 0.0
            lds = m.get("SQ_INSTS_LDS", 0.0)
            dur = m.get("duration_ns", 0.0)
            tf = m.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) * 512 / dur / 1e3 if dur else 0.0
            f.write(f"| `{k}` | {calls[k]} | {w / max(calls[k], 1):.0f} | {dur / 1e3 / max(calls[k], 1):.1f} | "
                    f"{tf:.0f} | {tf / 2500:.3f} | {mb:.3f} | {lds / w:.1f} | "
                    f"{m.get('SQ_LDS_BANK_CONFLICT', 0.0) / max(lds, 1):.2f} | "
                    f"{m.get('SQ_WAIT_INST_LDS', 0.0) / w:.0f} |\n")


if __name__ == "__main__":
    if sys.argv[1] == "mfma":
        mfma(sys.argv[2], sys.argv[3], sys.argv[4])
        sys.exit(0)
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6], sys.argv[7])
    elif sys.argv[1] == "overlap":
        overlap(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "sq":
        sq(sys.argv[2], sys.argv[3], sys.argv[4])
