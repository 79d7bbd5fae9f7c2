"""Short text summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2307_05388_amd.rocprof_summary kernels STATS_CSV --title T --command C > profiles/X.md
      per-kernel table from `rocprofv3 --kernel-trace --stats --output-format csv`
      (the *_kernel_stats.csv file).

  python -m paper_2307_05388_amd.rocprof_summary mfma COUNTER_CSV --type F64 --workload W --command C > profiles/Z.md
      matrix-core flops, rate and busy fraction per dispatch from one counter
      run (SQ_INSTS_VALU_MFMA_MOPS_F64 or _F32, SQ_VALU_MFMA_BUSY_CYCLES,
      GRBM_GUI_ACTIVE).

  python -m paper_2307_05388_amd.rocprof_summary traffic FETCH_CSV WRITE_CSV --copy-mb M --workload W \\
          --command-fetch C1 --command-write C2 > profiles/Y.md
      HBM bytes per dispatch of every kernel from two counter runs
      (`rocprofv3 --pmc FETCH_SIZE ...` and `rocprofv3 --pmc WRITE_SIZE ...`,
      csv output, *_counter_collection.csv), each counter scaled by what it
      reads for a plain copy of known size run in the same process
      (`bench.py --copy-mb M`: a fill that writes M MiB and copies that read
      and write M MiB).  The summary ends with one JSON line that bench.py
      reads back, tagged with the SHA-256 of the kernel source it was measured
      on, so the figure is dropped once the kernels change.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "fdfd_kernels.hip")
TRAFFIC_TAG = "traffic-json:"


def kernel_source_sha256() -> str:
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def short_name(name: str) -> str:
    m = re.search(r"::(k_[a-z_0-9]+)(<([\w, ]+)>)?\(", name)
    if m:
        return m.group(1) + (f"<{m.group(3).replace(' ', '')}>" if m.group(3) else "")
    n = name.replace("void ", "")
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):   # drop the argument list (outside template brackets)
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            cut = i
            break
    return n[:cut][:70]


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def kernels(args):
    rows = list(csv.DictReader(open(args.stats)))
    tot = sum(float(_col(r, "TotalDurationNs")) for r in rows)
    out = [f"# {args.title}", "", "Command (from the repository root, one MI355X):", "", "```",
           args.command, "```", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(_col(r, "TotalDurationNs")))[:args.top]:
        out.append(f"| {short_name(_col(r, 'Name'))} | {_col(r, 'Calls')} | "
                   f"{float(_col(r, 'TotalDurationNs')) / 1e6:.3f} | {float(_col(r, 'AverageNs')) / 1e3:.2f} | "
                   f"{float(_col(r, 'MinNs')) / 1e3:.2f} | {float(_col(r, 'MaxNs')) / 1e3:.2f} | "
                   f"{100 * float(_col(r, 'TotalDurationNs')) / tot:.1f} |")
    print("\n".join(out))


def _per_dispatch(path, counter):
    """{kernel: [values per dispatch]} for one counter (KiB)."""
    vals = collections.defaultdict(dict)
    for r in csv.DictReader(open(path)):
        if _col(r, "Counter_Name") != counter:
            continue
        k = _col(r, "Kernel_Name")
        d = _col(r, "Dispatch_Id")
        vals[k][d] = vals[k].get(d, 0.0) + float(_col(r, "Counter_Value"))
    return {k: list(v.values()) for k, v in vals.items()}


def traffic(args):
    fetch = _per_dispatch(args.fetch, "FETCH_SIZE")
    write = _per_dispatch(args.write, "WRITE_SIZE")
    kib = args.copy_mb * 1024.0
    # the copy reads copy_mb MiB (the largest FETCH of a copy kernel); the fill writes copy_mb MiB
    copy_fetch = max((max(v) for k, v in fetch.items() if "copy" in k.lower()), default=0.0)
    fill_write = max((max(v) for k, v in write.items() if "fill" in k.lower()), default=0.0)
    fs = kib / copy_fetch if copy_fetch else None
    ws = kib / fill_write if fill_write else None
    out = [f"# HBM traffic per dispatch: {args.workload}", "",
           "Commands (from the repository root, one MI355X):", "", "```", args.command_fetch, args.command_write,
           "```", "",
           f"Calibration with a plain copy of {args.copy_mb} MiB in the same process: FETCH_SIZE reads "
           f"{copy_fetch:.1f} KiB for {kib:.0f} KiB read (scale {fs if fs else float('nan'):.3f}); "
           f"WRITE_SIZE reads {fill_write:.1f} KiB for {kib:.0f} KiB written "
           f"(scale {ws if ws else float('nan'):.3f}).", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB (scaled) | written MB (scaled) |",
           "|---|---:|---:|---:|---:|---:|"]
    per = {}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("void fdfd"):
            continue
        f = sum(fetch.get(k, [0])) / max(1, len(fetch.get(k, [0])))
        w = sum(write.get(k, [0])) / max(1, len(write.get(k, [0])))
        rb = f * 1024 * (fs or 0)
        wb = w * 1024 * (ws or 0)
        per[short_name(k)] = {"read_bytes": rb, "write_bytes": wb, "bytes": rb + wb}
        out.append(f"| {short_name(k)} | {len(fetch.get(k, []))} | {f:.1f} | {w:.1f} | {rb / 1e6:.2f} | {wb / 1e6:.2f} |")
    out += ["", "Machine-readable (bench.py reads this line; it applies only to the kernel source with this hash):",
            "", TRAFFIC_TAG + " " + json.dumps({"workload": args.workload, "source_sha256": kernel_source_sha256(),
                                               "fetch_scale": fs, "write_scale": ws, "kernels": per})]
    print("\n".join(out))


def _dispatch_rows(path):
    """{kernel: {dispatch: {counter: [values], "ns": duration}}}."""
    out = collections.defaultdict(dict)
    for r in csv.DictReader(open(path)):
        k = _col(r, "Kernel_Name")
        d = out[k].setdefault(_col(r, "Dispatch_Id"), {"ns": float(_col(r, "End_Timestamp")) -
                                                        float(_col(r, "Start_Timestamp"))})
        d.setdefault(_col(r, "Counter_Name"), []).append(float(_col(r, "Counter_Value")))
    return out


def mfma(args):
    """Matrix-core use per dispatch from one counter run with
    SQ_INSTS_VALU_MFMA_MOPS_<type> (512 flops per count), SQ_VALU_MFMA_BUSY_CYCLES
    and GRBM_GUI_ACTIVE: MFMA flops the hardware executed, their rate over the
    dispatch, and the busy fraction of all SIMDs (busy / (active x SIMDs))."""
    rows = _dispatch_rows(args.csv)
    mops = f"SQ_INSTS_VALU_MFMA_MOPS_{args.type}"
    out = [f"# Matrix-core use per dispatch: {args.workload}", "", "Command (from the repository root, one MI355X):",
           "", "```", args.command, "```", "",
           f"MFMA flops = {mops} x 512; busy = SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x {args.simds} SIMDs), "
           f"active cycles = GRBM_GUI_ACTIVE (reported summed over the {args.xcds} XCDs) / {args.xcds}.",
           "", "| kernel | dispatches | avg us | MFMA GFLOP per dispatch | MFMA TFLOP/s | MFMA busy % |",
           "|---|---:|---:|---:|---:|---:|"]
    for k in sorted(rows):
        if not k.startswith("void fdfd"):
            continue
        ds = [d for d in rows[k].values() if mops in d]
        if not ds:
            continue
        fl = sum(sum(d[mops]) * 512 for d in ds) / len(ds)
        ns = sum(d["ns"] for d in ds) / len(ds)
        # GRBM_GUI_ACTIVE arrives summed over the XCDs: per-XCD active cycles x XCDs
        busy = [sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", [0])) /
                (sum(d.get("GRBM_GUI_ACTIVE", [1])) / args.xcds * args.simds) for d in ds]
        out.append(f"| {short_name(k)} | {len(ds)} | {ns / 1e3:.1f} | {fl / 1e9:.3f} | {fl / ns / 1e3:.2f} | "
                   f"{100 * sum(busy) / len(busy):.2f} |")
    print("\n".join(out))


def read_traffic(path):
    """The JSON line of a traffic summary if it was measured on the current kernels, else None."""
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith(TRAFFIC_TAG):
                    d = json.loads(line[len(TRAFFIC_TAG):])
                    return d if d.get("source_sha256") == kernel_source_sha256() else None
    except OSError:
        return None
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("stats")
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--top", type=int, default=20)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("--copy-mb", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    mf = sub.add_parser("mfma")
    mf.add_argument("csv")
    mf.add_argument("--type", default="F64")
    mf.add_argument("--simds", type=int, default=1024)
    mf.add_argument("--xcds", type=int, default=8)
    mf.add_argument("--workload", required=True)
    mf.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    {"kernels": kernels, "traffic": traffic, "mfma": mfma}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
