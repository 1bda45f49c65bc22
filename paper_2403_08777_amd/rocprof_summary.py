"""Turn rocprofv3 output into the short text summaries kept under profiles/.

    python -m paper_2403_08777_amd.rocprof_summary stats KERNEL_STATS_CSV --command CMD
    python -m paper_2403_08777_amd.rocprof_summary traffic --fetch F --write W \\
        --workload NAME --command-fetch CMD --command-write CMD
    python -m paper_2403_08777_amd.rocprof_summary counters PMC_CSV [PMC_CSV ...] --trace STATS_CSV \\
        --command CMD --trace-command CMD [--json-out FILE]

``stats`` prints a markdown table of per-kernel call counts and durations from
a ``--kernel-trace --stats -f csv`` run.  ``traffic`` reads two ``--pmc`` runs
(FETCH_SIZE, then WRITE_SIZE; CSV or rocpd database), scales each counter by
what it reads for the plain 1 GiB device copy that ``bench.py
--copy-calibration`` performs, and prints a JSON record of the HBM bytes per
assembly call (forward, VJP) tagged with a digest of the HIP sources, which
``bench.py`` uses only while the kernels are unchanged.  ``counters`` reads one
``--pmc`` run of SQ instruction counters (and the kernel-trace statistics of
the same workload for durations) and prints per-wave instruction counts and an
estimate of how busy the vector ALUs were.
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


def traffic(args):
    f_rows, w_rows = read_counters(args.fetch), read_counters(args.write)
    fetch, write = median_by_kernel(f_rows, "FETCH_SIZE"), median_by_kernel(w_rows, "WRITE_SIZE")
    fs, fkib = copy_scale(f_rows, "FETCH_SIZE")
    ws, wkib = copy_scale(w_rows, "WRITE_SIZE")
    calls = {}

    def targs(name):
        m = re.match(r"(\w+)<(.*)>$", name)
        return (m.group(1), [a.strip() for a in m.group(2).split(",")]) if m else (name, [])

    # the benchmark's calls: k_assemble_patch<double, EDDY none, CONV advective,
    # MODE, GATHER> followed by k_gather_partials<double, 3>
    for mode, tag in (("fwd", "0"), ("vjp", "1")):
        parts = [key for key in fetch if targs(key[0]) == ("k_assemble_patch", ["double", "0", "0", tag, "true"])]
        gathers = [key for key in fetch if targs(key[0]) == ("k_gather_partials", ["double", "3"])]
        keys = parts + gathers
        if not parts:
            continue
        fb = sum(fetch[k] for k in keys) * 1024.0 * fs
        wb = sum(write.get(k, 0.0) for k in keys) * 1024.0 * ws
        calls[mode] = {"kernels": [f"{k[0]} (grid {k[1]})" for k in keys], "fetch_bytes": fb,
                       "write_bytes": wb, "bytes": fb + wb}
    rec = {"workload": args.workload, "scatter": args.scatter, "source_sha256": source_digest(),
           "command_fetch": args.command_fetch, "command_write": args.command_write,
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": fkib, "write_kib": wkib,
                                "fetch_scale": fs, "write_scale": ws},
           "calls": calls}
    json.dump(rec, sys.stdout, indent=1)
    print()


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


def counters(args):
    rows = [r for path in args.pmc for r in read_counters(path)]
    names = sorted({c for _, _, c, _ in rows})
    med = {c: median_by_kernel(rows, c) for c in names}
    dur = {}
    with open(args.trace) as f:
        for r in csv.DictReader(f):
            dur[short_name(r["Name"])] = float(r["AverageNs"]) * 1e-9
    pat = re.compile(args.kernels)
    keys = sorted(k for k in med.get("SQ_WAVES", {}) if pat.search(k[0]))
    shown = [c for c in names if c != "SQ_WAVES"]
    # executed floating-point operations: a wave instruction is 64 lane
    # operations, an FMA two flops
    flop_sets = {p: [f"SQ_INSTS_VALU_{op}_{p}" for op in ("ADD", "MUL", "FMA", "TRANS")] for p in ("F64", "F32")}
    have = {p: [c for c in cs if c in med] for p, cs in flop_sets.items()}

    def flops(key, prec):
        return 64.0 * sum(med[c].get(key, 0.0) * (2.0 if "_FMA_" in c else 1.0) for c in have[prec])
    print(f"Commands: `{args.command}`\n")
    print(f"Durations: `{args.trace_command}`\n")
    print("Per-wave medians over the dispatches of each kernel (a wave is 64 elements in the element "
          "phase). VALU busy = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz x average duration), an "
          "estimate of the share of SIMD cycles spent issuing vector instructions: 4 cycles is what a "
          "wave64 FP64 FMA takes on a 16-lane SIMD (instructions that issue faster make it an "
          "overestimate) and 2.4 GHz is the peak clock (a lower clock makes it an underestimate).\n")
    if have["F64"] or have["F32"]:
        print("Executed flops per grid item (an element, or a node for the gather) = 64 lanes x "
              "(ADD + MUL + 2 FMA + TRANS instructions) / grid size, counting every lane of a wave "
              "instruction.\n")
    extra = [p for p in ("F64", "F32") if have[p]]
    lds_ratio = "SQ_LDS_BANK_CONFLICT" in med and "SQ_LDS_IDX_ACTIVE" in med
    l2 = next(((h, m) for h, m in (("TCC_HIT_sum", "TCC_MISS_sum"), ("TCC_HIT", "TCC_MISS"))
               if h in med and m in med), None)
    if l2:
        print("L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS) over the kernel's L2 requests.\n")
    if lds_ratio:
        print("Conflict share = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE: the fraction of the LDS's "
              "indexed-active cycles spent stalled on bank conflicts (a ratio of two counters that "
              "aggregate the same way).\n")
    print("| kernel | grid | waves | " + " | ".join(c.replace("SQ_", "") + "/wave" for c in shown) +
          "".join(f" | {p} flop/item" for p in extra) + (" | conflict share" if lds_ratio else "") +
          (" | L2 hit rate" if l2 else "") + " | avg us | VALU busy |")
    print("|---|---:|---:|" + "---:|" * (len(shown) + len(extra) + int(lds_ratio) + int(bool(l2))) + "---:|---:|")
    rec = {"source_sha256": source_digest(), "command": args.command, "kernels": {}}
    for key in keys:
        waves = med["SQ_WAVES"][key]
        vals = " | ".join(f"{med[c].get(key, float('nan')) / waves:.1f}" for c in shown)
        fl = "".join(f" | {flops(key, p) / key[1]:.1f}" for p in extra)
        if lds_ratio:
            act = med["SQ_LDS_IDX_ACTIVE"].get(key, 0.0)
            fl += f" | {med['SQ_LDS_BANK_CONFLICT'].get(key, 0.0) / act:.2f}" if act else " | -"
        if l2:
            hit, miss = med[l2[0]].get(key, 0.0), med[l2[1]].get(key, 0.0)
            fl += f" | {hit / (hit + miss):.2f}" if hit + miss else " | -"
        d = dur.get(key[0])
        busy = (med["SQ_INSTS_VALU"][key] * VALU_CYCLES / (SIMDS * CLOCK_HZ * d)
                if d and "SQ_INSTS_VALU" in med else float("nan"))
        print(f"| `{key[0]}` | {key[1]} | {waves:.0f} | {vals}{fl} | "
              f"{d * 1e6 if d else float('nan'):.1f} | {busy:.2f} |")
        rec["kernels"][f"{key[0]} (grid {key[1]})"] = {
            "waves": waves, "per_wave": {c: med[c].get(key) / waves for c in shown if key in med[c]},
            **{f"{p.lower()}_flops": flops(key, p) for p in extra}}
    if args.json_out:
        # per benchmark call: the patch kernel of the mode plus its gather
        calls = {}
        for mode, tag in (("fwd", "0"), ("vjp", "1")):
            ks = [k for k in keys if k[0] in (f"k_assemble_patch<double, 0, 0, {tag}, true>",
                                              "k_gather_partials<double, 3>")]
            if len(ks) == 2 and have["F64"]:
                calls[mode] = {"kernels": [f"{k[0]} (grid {k[1]})" for k in ks],
                               "fp64_flops": sum(flops(k, "F64") for k in ks)}
        rec["calls"] = calls
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
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--scatter", default="patch_gather")
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    c = sub.add_parser("counters")
    c.add_argument("pmc", nargs="+", help="counter CSVs of one or more --pmc passes over the same workload")
    c.add_argument("--trace", required=True, help="kernel_stats.csv of a --kernel-trace --stats run")
    c.add_argument("--command", required=True)
    c.add_argument("--trace-command", required=True)
    c.add_argument("--kernels", default=r"k_assemble_patch<\w+, 0, 0, [01], true>|k_gather_partials")
    c.add_argument("--json-out", help="also write the per-kernel figures and the FP64 flops of the "
                                      "benchmark calls as a JSON record tagged with the source digest")
    args = ap.parse_args()
    {"stats": stats, "traffic": traffic, "counters": counters}[args.cmd](args)


if __name__ == "__main__":
    main()
