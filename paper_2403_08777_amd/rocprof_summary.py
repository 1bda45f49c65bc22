"""Turn rocprofv3 output into the short text summaries kept under profiles/.

    python -m paper_2403_08777_amd.rocprof_summary stats KERNEL_STATS_CSV --command CMD
    python -m paper_2403_08777_amd.rocprof_summary counters PASS_A.csv PASS_B.csv ... \\
        --workload NAME --title TEXT --command CMD_A --command CMD_B ... \\
        [--trace STATS_CSV --trace-command CMD] --json-out profiles/counters_NAME.json

``stats`` prints a markdown table of per-kernel call counts and durations from
a ``--kernel-trace --stats -f csv`` run.  ``counters`` reads several ``--pmc``
passes over one workload (each run with ``bench.py --copy-calibration``, whose
plain 1 GiB device copy calibrates FETCH_SIZE and WRITE_SIZE), prints a
markdown table per kernel and writes the JSON record ``bench.py`` reads: HBM
bytes, executed FP64/FP32 flops, per-wave instruction and LDS counters and the
L2 hit rate of every assembly kernel, tagged with a digest of the HIP sources
so that it is used only while the kernels are unchanged.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sqlite3
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_08777_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    name = name.replace("nsasm::(anonymous namespace)::", "")
    m = re.match(r"(?:void )?([\w:]+(?:<[^()]*>)?)", name)
    return m.group(1) if m else name[:60]


def read_counters(path: str):
    """[(kernel name, grid size, counter, value)] from a CSV or rocpd DB."""
    rows = []
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        cur = con.execute("select kernel_name, grid_size, counter_name, value from counters_collection")
        rows = [(k, int(g), c, float(v)) for k, g, c, v in cur]
    else:
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append((r["Kernel_Name"], int(r["Grid_Size"]), r["Counter_Name"], float(r["Counter_Value"])))
    return rows


def median_by_kernel(rows, counter):
    """Median per-dispatch value of `counter` for each (kernel, grid size)."""
    acc = defaultdict(list)
    for k, g, c, v in rows:
        if c == counter:
            acc[(short_name(k), g)].append(v)
    return {key: sorted(v)[len(v) // 2] for key, v in acc.items()}


def copy_scale(rows, counter):
    """Bytes per counter unit, from the 1 GiB device copy (the largest copy
    dispatch of the run)."""
    kib = max((v for k, g, c, v in rows if c == counter and "copyBuffer" in k), default=None)
    if not kib:
        raise SystemExit("no copy kernel found: run bench.py with --copy-calibration")
    return COPY_BYTES / (kib * 1024.0), kib


def stats(args):
    with open(args.csv) as f:
        rows = list(csv.DictReader(f))
    res = {}
    if args.dispatches:
        # LDS and scratch bytes per workgroup from the dispatch records of the same run
        with open(args.dispatches) as f:
            for r in csv.DictReader(f):
                res.setdefault(short_name(r["Kernel_Name"]), (r["LDS_Block_Size"], r["Scratch_Size"]))
    print(f"Command: `{args.command}`\n")
    cols = " | LDS B | scratch B" if res else ""
    print(f"| kernel | calls | avg us | min us | max us | total %{cols} |")
    print("|---|---:|---:|---:|---:|---:|" + ("---:|" * 2 if res else ""))
    for r in rows[: args.top]:
        name = short_name(r["Name"])
        extra = "".join(f" | {v}" for v in res.get(name, ("",) * 2)) if res else ""
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f}{extra} |")


SIMDS = 256 * 4        # MI355X: 256 compute units, 4 SIMDs each
CLOCK_HZ = 2.4e9       # peak engine clock
VALU_CYCLES = 4        # a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles
FLOP_COUNTERS = {p: [f"SQ_INSTS_VALU_{op}_{p}" for op in ("ADD", "MUL", "FMA", "TRANS")] for p in ("F64", "F32")}


def counters(args):
    """One record per workload from several --pmc passes over the same short
    bench run (each with --copy-calibration): per kernel the median
    per-dispatch value of every counter, HBM bytes from FETCH_SIZE and
    WRITE_SIZE scaled by what each counter reads for the 1 GiB device copy of
    its own pass, executed flops from the VALU type counters, the L2 hit rate,
    plus a markdown table with the VALU-busy estimate from the kernel-trace
    durations."""
    per_pass = [read_counters(path) for path in args.pmc]
    rows = [r for rs in per_pass for r in rs]
    names = sorted({c for _, _, c, _ in rows})
    med = {c: median_by_kernel(rows, c) for c in names}
    scale = {}
    for rs in per_pass:
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            if any(c == ctr for _, _, c, _ in rs):
                scale[ctr] = copy_scale(rs, ctr)
    pat = re.compile(args.kernels)
    # one grid per kernel: the workload's (the one dispatched most often)
    count = defaultdict(int)
    for k, g, c, _ in rows:
        if c == "SQ_WAVES":
            count[(short_name(k), g)] += 1
    best = {}
    for (k, g), n in count.items():
        if pat.search(k) and (k not in best or n > count[(k, best[k])]):
            best[k] = g
    dur = {}
    if args.trace:
        with open(args.trace) as f:
            for r in csv.DictReader(f):
                dur[short_name(r["Name"])] = float(r["AverageNs"]) * 1e-9
    have = {p: [c for c in cs if c in med] for p, cs in FLOP_COUNTERS.items()}

    def flops(key, prec):
        return 64.0 * sum(med[c].get(key, 0.0) * (2.0 if "_FMA_" in c else 1.0) for c in have[prec])

    l2 = next(((h, m) for h, m in (("TCC_HIT_sum", "TCC_MISS_sum"), ("TCC_HIT", "TCC_MISS"))
               if h in med and m in med), None)
    shown = [c for c in names if c not in ("SQ_WAVES", "FETCH_SIZE", "WRITE_SIZE") and not c.startswith("TCC_")]
    rec = {"workload": args.workload, "source_sha256": args.source_sha256 or source_digest(), "commands": args.command,
           "trace_command": args.trace_command,
           "copy_calibration": {ctr: {"copy_bytes": COPY_BYTES, "counter_kib": kib, "bytes_per_kib": sc * 1024.0}
                                for ctr, (sc, kib) in scale.items()},
           "kernels": {}}
    print(f"# Counters: {args.title}\n")
    print("Commands (run from the repository root on one MI355X, one `--pmc` pass each):\n")
    for c in args.command:
        print(f"- `{c}`")
    if args.trace_command:
        print(f"\nDurations: `{args.trace_command}`\n")
    print("\nPer-dispatch medians per kernel; per-wave counts divide by SQ_WAVES (a wave is 64 elements in "
          "the element phase, 64 nodes in the gather). HBM bytes = FETCH_SIZE and WRITE_SIZE, each scaled by "
          "what it reads for a plain 1 GiB device copy in the same pass. Executed flops = 64 lanes x (ADD + "
          "MUL + 2 FMA + TRANS) VALU instructions of the type. VALU busy = SQ_INSTS_VALU x 4 cycles / "
          "(1024 SIMDs x 2.4 GHz x average duration). Conflict share = SQ_LDS_BANK_CONFLICT / "
          "SQ_LDS_IDX_ACTIVE. L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS).\n")
    print("| kernel | grid | waves | " + " | ".join(c.replace("SQ_", "") + "/wave" for c in shown) +
          " | HBM MB | F64 flop/item | F32 flop/item | conflict share | L2 hit | avg us | VALU busy |")
    print("|---|---:|---:|" + "---:|" * len(shown) + "---:|---:|---:|---:|---:|---:|---:|")
    for kname, grid in sorted(best.items()):
        key = (kname, grid)
        waves = med["SQ_WAVES"].get(key, 0.0)
        if not waves:
            continue
        pw = {c: med[c][key] / waves for c in shown if key in med[c]}
        ent = {"grid": grid, "waves": waves, "per_wave": pw}
        hb = 0.0
        for ctr, name in (("FETCH_SIZE", "fetch_bytes"), ("WRITE_SIZE", "write_bytes")):
            if ctr in med and key in med[ctr] and ctr in scale:
                ent[name] = med[ctr][key] * 1024.0 * scale[ctr][0]
                hb += ent[name]
        ent["hbm_bytes"] = hb if ("fetch_bytes" in ent and "write_bytes" in ent) else None
        if have["F64"] or have["F32"]:
            ent["f64_flops"], ent["f32_flops"] = flops(key, "F64"), flops(key, "F32")
        if l2:
            hit, miss = med[l2[0]].get(key, 0.0), med[l2[1]].get(key, 0.0)
            ent["l2_hit_rate"] = hit / (hit + miss) if hit + miss else None
        rec["kernels"][kname] = ent
        d = dur.get(kname)
        busy = (pw["SQ_INSTS_VALU"] * waves * VALU_CYCLES / (SIMDS * CLOCK_HZ * d)
                if d and "SQ_INSTS_VALU" in pw else float("nan"))
        act = pw.get("SQ_LDS_IDX_ACTIVE")
        share = f"{pw.get('SQ_LDS_BANK_CONFLICT', 0.0) / act:.2f}" if act else "-"
        l2s = f"{ent['l2_hit_rate']:.2f}" if ent.get("l2_hit_rate") is not None else "-"
        hbs = f"{ent['hbm_bytes'] / 1e6:.1f}" if ent.get("hbm_bytes") else "-"
        print(f"| `{kname}` | {grid} | {waves:.0f} | " + " | ".join(f"{pw.get(c, float('nan')):.1f}" for c in shown)
              + f" | {hbs} | {ent.get('f64_flops', 0.0) / grid:.1f} | {ent.get('f32_flops', 0.0) / grid:.1f} | "
              f"{share} | {l2s} | {d * 1e6 if d else float('nan'):.1f} | {busy:.2f} |")
    with open(args.json_out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--dispatches", help="kernel_trace.csv of the same run, for LDS and scratch columns")
    c = sub.add_parser("counters")
    c.add_argument("pmc", nargs="+", help="counter CSVs (or rocpd databases) of --pmc passes over one workload")
    c.add_argument("--workload", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", required=True, help="the command of each pass, in order")
    c.add_argument("--trace", help="kernel_stats.csv of a --kernel-trace --stats run of the same workload")
    c.add_argument("--trace-command", default="")
    c.add_argument("--kernels", default=r"^k_assemble_patch<|^k_gather_partials<")
    c.add_argument("--json-out", required=True, help="the JSON record bench.py reads (counters_<workload>.json)")
    c.add_argument("--source-sha256", default="",
                   help="digest of the HIP sources the passes ran with (default: the sources here now)")
    args = ap.parse_args()
    {"stats": stats, "counters": counters}[args.cmd](args)


if __name__ == "__main__":
    main()
