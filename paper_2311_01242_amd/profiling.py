"""Summaries of rocprofv3 output for the benchmark's roofline accounting.

Three sub-commands, both reading the CSV files rocprofv3 writes with
``--output-format csv``:

``stats``   kernel-trace statistics (``*_kernel_stats.csv``) grouped into the
            evaluation's phases, as a markdown table (stdout).

``counters`` instruction mix and issue/wait fractions per kernel from the
            SQ counters of several ``--pmc`` passes (summed over dispatches).

``traffic`` HBM bytes per launch of each phase's kernels from two ``--pmc``
            runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), scaled by
            what the same counters read for a plain device copy of known size
            (``bench.py --calibrate-copy``: 3 copies of 2 GiB).  Writes the
            JSON that ``bench.py`` reads for ``roofline.traffic`` (keyed by
            phase, with the sha256 of the kernel source it was measured on)
            and prints a markdown table.

Phase of a kernel: k_prun<1,...> / k_run_fwd / k_small_fwd forward,
k_prun<2,...> / k_run_adj / k_small_adj adjoint, k_ppool pool sweep, k_hx_ci /
k_ci_scatter / k_ci_gather / k_hx_packed / k_hx_sector / k_hx_dense /
k_small_hx H-apply.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_01242_amd", "csrc")
PHASE_SOURCE = {"forward": "k_packed.hip", "adjoint": "k_packed.hip", "h_apply": "k_hx_ci.hip"}
COPY_BYTES = 2 ** 31


def phase_of(name: str):
    if "k_prun<1" in name or "k_run_fwd" in name or "k_small_fwd" in name:
        return "forward"
    if "k_prun<2" in name or "k_run_adj" in name or "k_small_adj" in name:
        return "adjoint"
    if "k_small_hx" in name:
        return "h_apply"
    if "k_ppool" in name:
        return "pool_sweep"
    if any(k in name for k in ("k_hx_ci", "k_ci_scatter", "k_ci_gather", "k_hx_packed",
                               "k_hx_sector", "k_hx_dense")):
        return "h_apply"
    return None


def short(name: str) -> str:
    name = name.replace("void ", "").replace("vqe::", "")
    return name.split("(")[0]


def cmd_stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    by_phase = collections.defaultdict(lambda: [0, 0.0])
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---:|---:|---:|---:|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        calls, ns = int(r["Calls"]), float(r["TotalDurationNs"])
        print(f"| {short(r['Name'])} | {calls} | {ns / 1e6:.2f} | {ns / calls / 1e3:.2f} | "
              f"{100 * ns / total:.1f} |")
        ph = phase_of(r["Name"])
        if ph:
            by_phase[ph][0] += calls
            by_phase[ph][1] += ns
    print()
    print("| phase | calls | total ms | avg us per launch |")
    print("|---|---:|---:|---:|")
    for ph, (calls, ns) in sorted(by_phase.items()):
        print(f"| {ph} | {calls} | {ns / 1e6:.2f} | {ns / calls / 1e3:.2f} |")


def _sum_counter(path):
    """Counter totals per phase, and the phase's launches: for the H-apply only
    the k_hx_* kernels count (the order conversions' bytes are charged to
    them, as bench.py's phase time includes them)."""
    tot = collections.defaultdict(float)
    cnt = collections.Counter()
    for r in csv.DictReader(open(path)):
        ph = phase_of(r["Kernel_Name"]) or short(r["Kernel_Name"])
        tot[ph] += float(r["Counter_Value"])
        if ph != "h_apply" or "k_hx_" in r["Kernel_Name"]:
            cnt[ph] += 1
    return tot, cnt


def _sha(name):
    with open(os.path.join(CSRC, name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def cmd_traffic(args):
    f, fc = _sum_counter(args.fetch)
    w, _ = _sum_counter(args.write)
    cf, _ = _sum_counter(args.copy_fetch)
    cw, _ = _sum_counter(args.copy_write)
    copy_key = next(k for k in cf if "copyBuffer" in k)
    kf = 3 * COPY_BYTES / (cf[copy_key] * 1024)
    kw = 3 * COPY_BYTES / (cw[copy_key] * 1024)
    out = {"calibration": {"fetch_factor": kf, "write_factor": kw,
                           "copy_bytes": COPY_BYTES, "copies": 3},
           "evaluations": args.evals, "workload": args.workload, "kernels": {}}
    print(f"calibration: FETCH_SIZE factor {kf:.3f}, WRITE_SIZE factor {kw:.3f}")
    print()
    print("| phase | launches / eval | fetch GB / eval | write GB / eval | bytes per launch |")
    print("|---|---:|---:|---:|---:|")
    for ph in ("forward", "h_apply", "adjoint"):
        if ph not in f:
            continue
        fetch = f[ph] * 1024 * kf / args.evals
        write = w.get(ph, 0.0) * 1024 * kw / args.evals
        launches = fc[ph] / args.evals
        per = (fetch + write) / launches
        out["kernels"][ph] = {"source_sha256": _sha(PHASE_SOURCE[ph]), "source": PHASE_SOURCE[ph],
                              "fetch_bytes_per_eval": fetch, "write_bytes_per_eval": write,
                              "launches_per_eval": launches, "bytes_per_launch": per}
        print(f"| {ph} | {launches:.0f} | {fetch / 1e9:.2f} | {write / 1e9:.2f} | {per / 1e6:.2f} MB |")
    with open(args.out, "w") as fo:
        json.dump(out, fo, indent=1, sort_keys=True)


# derived per-kernel figures from summed SQ counters (all per dispatch sums
# over the whole GPU): instruction mix per wave, and fractions of the waves'
# resident time (SQ_WAVE_CYCLES) spent issuing or waiting
ISSUE_ROWS = [
    ("waves", lambda c, n: c["SQ_WAVES"] / n, "{:.0f}"),
    ("VALU / wave", lambda c, n: c["SQ_INSTS_VALU"] / c["SQ_WAVES"], "{:.0f}"),
    ("SALU / wave", lambda c, n: c["SQ_INSTS_SALU"] / c["SQ_WAVES"], "{:.0f}"),
    ("LDS / wave", lambda c, n: c["SQ_INSTS_LDS"] / c["SQ_WAVES"], "{:.0f}"),
    ("VMEM rd+wr / wave", lambda c, n: (c["SQ_INSTS_VMEM_RD"] + c["SQ_INSTS_VMEM_WR"]) / c["SQ_WAVES"],
     "{:.1f}"),
    ("SMEM / wave", lambda c, n: c["SQ_INSTS_SMEM"] / c["SQ_WAVES"], "{:.1f}"),
    ("branch / wave", lambda c, n: c["SQ_INSTS_BRANCH"] / c["SQ_WAVES"], "{:.0f}"),
    ("FP64 FMA / VALU", lambda c, n: c["SQ_INSTS_VALU_FMA_F64"] / c["SQ_INSTS_VALU"], "{:.3f}"),
    ("issuing (ACTIVE_INST_ANY / WAVE_CYCLES)",
     lambda c, n: c["SQ_ACTIVE_INST_ANY"] / c["SQ_WAVE_CYCLES"], "{:.3f}"),
    ("VALU issuing (ACTIVE_INST_VALU / WAVE_CYCLES)",
     lambda c, n: c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"], "{:.3f}"),
    ("LDS issuing (ACTIVE_INST_LDS / WAVE_CYCLES)",
     lambda c, n: c["SQ_ACTIVE_INST_LDS"] / c["SQ_WAVE_CYCLES"], "{:.3f}"),
    ("waiting on a dependency (WAIT_INST_ANY / WAVE_CYCLES)",
     lambda c, n: c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"], "{:.3f}"),
    ("waiting on LDS (WAIT_INST_LDS / WAVE_CYCLES)",
     lambda c, n: c["SQ_WAIT_INST_LDS"] / c["SQ_WAVE_CYCLES"], "{:.3f}"),
    ("waiting, any reason incl. barriers (WAIT_ANY / WAVE_CYCLES)",
     lambda c, n: c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"], "{:.3f}"),
    ("LDS bank-conflict cycles / LDS active cycles",
     lambda c, n: c["SQ_LDS_BANK_CONFLICT"] / c["SQ_LDS_IDX_ACTIVE"], "{:.3f}"),
    ("active lanes per VALU instruction (THREAD_CYCLES_VALU / ACTIVE_INST_VALU)",
     lambda c, n: c["SQ_THREAD_CYCLES_VALU"] / c["SQ_ACTIVE_INST_VALU"], "{:.1f}"),
]


def cmd_counters(args):
    """Sum every counter over the dispatches of each selected kernel (name
    prefix match) across the given pmc CSV files and print the derived
    figures that the collected counters allow."""
    tot = {k: collections.defaultdict(float) for k in args.kernel}
    disp = {k: set() for k in args.kernel}
    for path in args.csv:
        for r in csv.DictReader(open(path)):
            name = short(r["Kernel_Name"]).replace(" ", "")
            for k in args.kernel:
                if name.startswith(k.replace(" ", "")):
                    tot[k][r["Counter_Name"]] += float(r["Counter_Value"])
                    disp[k].add((path, r["Dispatch_Id"]))
    print("| figure | " + " | ".join(args.kernel) + " |")
    print("|---|" + "---:|" * len(args.kernel))
    nd = {k: max(1, len(disp[k]) // max(1, len(args.csv))) for k in args.kernel}
    print("| dispatches | " + " | ".join(str(nd[k]) for k in args.kernel) + " |")
    for label, fn, fmt in ISSUE_ROWS:
        vals = []
        for k in args.kernel:
            try:
                vals.append(fmt.format(fn(tot[k], nd[k])))
            except (KeyError, ZeroDivisionError):
                vals.append("-")
        if any(v != "-" for v in vals):
            print(f"| {label} | " + " | ".join(vals) + " |")


def cmd_derived(args):
    """Mean over the dispatches of each selected kernel of every counter in
    the given pmc CSV files (for rocprofv3's derived metrics, which are per
    dispatch ratios: VALUBusy, OccupancyPercent, ...), one row per kernel."""
    vals = {k: collections.defaultdict(list) for k in args.kernel}
    names = []
    for path in args.csv:
        for r in csv.DictReader(open(path)):
            name = short(r["Kernel_Name"]).replace(" ", "")
            for k in args.kernel:
                if name.startswith(k.replace(" ", "")):
                    c = r["Counter_Name"]
                    if c not in names:
                        names.append(c)
                    vals[k][c].append(float(r["Counter_Value"]))
    print("| kernel | " + " | ".join(names) + " |")
    print("|---|" + "---:|" * len(names))
    for k in args.kernel:
        row = [f"{sum(vals[k][c]) / len(vals[k][c]):.2f}" if vals[k][c] else "-" for c in names]
        print(f"| {k} | " + " | ".join(row) + " |")


def main():
    ap = argparse.ArgumentParser(prog="python -m paper_2311_01242_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--evals", type=float, required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--workload", required=True, help="bench workload the counters were taken on")
    c = sub.add_parser("counters")
    c.add_argument("--kernel", action="append", required=True,
                   help="kernel name prefix as rocprof prints it, e.g. 'k_prun<2, 512, 3>'")
    c.add_argument("csv", nargs="+", help="*_counter_collection.csv files of the pmc passes")
    d = sub.add_parser("derived")
    d.add_argument("--kernel", action="append", required=True,
                   help="kernel name prefix as rocprof prints it, e.g. 'k_prun<2, 512, 3>'")
    d.add_argument("csv", nargs="+", help="*_counter_collection.csv files of the pmc passes")
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters, "derived": cmd_derived}[a.cmd](a)


if __name__ == "__main__":
    main()
