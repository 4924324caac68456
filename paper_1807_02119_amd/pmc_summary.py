"""Turn rocprofv3 counter-collection CSVs into the HBM traffic record that
bench.py reports in its roofline.

Four counter runs are needed, each a separate rocprofv3 --pmc invocation with
--output-format csv: FETCH_SIZE and WRITE_SIZE of bench.py (the contraction
kernel), and the same two counters of ``bench.py --pmc-calibrate BYTES`` (a
plain device-to-device copy of known size).  The counters report KiB per
dispatch; the copy run gives the factor between the counters and real bytes
(it should read BYTES and write BYTES), and the kernel's per-dispatch
counters are scaled by it.

    python -m paper_1807_02119_amd.pmc_summary --kernel engine \\
        --fetch DIR_F --write DIR_W --cal-fetch DIR_CF --cal-write DIR_CW \\
        --cal-bytes 268435456 --json profiles/engine_traffic.json \\
        --md profiles/engine_q3_200_600_traffic.md
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics


def _rows(directory):
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {directory}")
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def per_dispatch(directory, counter, name_filter):
    """{dispatch id: counter value} over dispatches whose kernel name contains
    name_filter (values of one dispatch are summed over dimensions)."""
    vals = {}
    names = {}
    for r in _rows(directory):
        if r.get("Counter_Name") != counter or name_filter not in r.get("Kernel_Name", ""):
            continue
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return vals, names


def source_hash(root):
    h = hashlib.sha256()
    for f in ("engine.hip", "program.h", "decode.h", "checks.h"):
        with open(os.path.join(root, "paper_1807_02119_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters_main(argv):
    """Median per dispatch of every counter in one or more --pmc runs, for the
    kernels whose name contains --kernel: a markdown table (and JSON)."""
    ap = argparse.ArgumentParser(prog="pmc_summary counters")
    ap.add_argument("--kernel", default="engine")
    ap.add_argument("--dirs", nargs="+", required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--title", default="rocprofv3 counters")
    ap.add_argument("--note", default="")
    ap.add_argument("--command", default="")
    args = ap.parse_args(argv)
    table = {}
    for d in args.dirs:
        names = sorted({r["Counter_Name"] for r in _rows(d)})
        for c in names:
            vals, kn_ = per_dispatch(d, c, args.kernel)
            if vals:
                table[c] = (statistics.median(vals.values()), len(vals), sorted(set(kn_.values())))
    with open(args.md, "w") as f:
        f.write(f"# {args.title}\n\n")
        if args.note:
            f.write(args.note + "\n\n")
        f.write("| counter | median per dispatch | dispatches | kernel |\n|---|---|---|---|\n")
        for c, (v, n, k) in sorted(table.items()):
            f.write(f"| {c} | {v:.6g} | {n} | `{', '.join(k)}` |\n")
        if args.command:
            f.write("\nCommands:\n\n```\n" + args.command + "\n```\n")
    print(json.dumps({c: v for c, (v, n, k) in table.items()}))


def main():
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        return counters_main(sys.argv[2:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", default="engine")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--cal-fetch", required=True)
    ap.add_argument("--cal-write", required=True)
    ap.add_argument("--cal-bytes", type=int, required=True)
    ap.add_argument("--cal-kernel", default="", help="substring of the copy kernel's name")
    ap.add_argument("--json", required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--command", default="")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    cf, _ = per_dispatch(args.cal_fetch, "FETCH_SIZE", args.cal_kernel)
    cw, _ = per_dispatch(args.cal_write, "WRITE_SIZE", args.cal_kernel)
    # the copy: the largest dispatches are the copies of the known size
    kib = args.cal_bytes / 1024.0
    fetch_factor = kib / statistics.median(sorted(cf.values())[-3:])
    write_factor = kib / statistics.median(sorted(cw.values())[-3:])

    kf, names = per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    kw, _ = per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    kname = sorted(set(names.values()))
    fetch_kib = statistics.median(kf.values())
    write_kib = statistics.median(kw.values())
    fetch_b = fetch_kib * 1024.0 * fetch_factor
    write_b = write_kib * 1024.0 * write_factor
    rec = {"kernel": kname, "dispatches": [len(kf), len(kw)],
           "fetch_kib_per_dispatch": fetch_kib, "write_kib_per_dispatch": write_kib,
           "calibration_bytes": args.cal_bytes, "fetch_factor": fetch_factor,
           "write_factor": write_factor, "fetch_bytes": fetch_b, "write_bytes": write_b,
           "source_hash": source_hash(root), "command": args.command}
    data = {}
    if os.path.exists(args.json):
        with open(args.json) as f:
            data = json.load(f)
    data["engine<double>"] = rec
    with open(args.json, "w") as f:
        json.dump(data, f, indent=1)
    with open(args.md, "w") as f:
        f.write("# HBM traffic of the contraction kernel (rocprofv3 PMC)\n\n")
        f.write(f"Kernel: `{', '.join(kname)}`; dispatches measured: {len(kf)} (FETCH_SIZE), "
                f"{len(kw)} (WRITE_SIZE); median per dispatch.\n\n")
        f.write("| counter | KiB per dispatch | calibration factor | bytes per dispatch |\n")
        f.write("|---|---|---|---|\n")
        f.write(f"| FETCH_SIZE | {fetch_kib:.1f} | {fetch_factor:.4f} | {fetch_b:.4g} |\n")
        f.write(f"| WRITE_SIZE | {write_kib:.1f} | {write_factor:.4f} | {write_b:.4g} |\n\n")
        f.write(f"Calibration: a device-to-device copy of {args.cal_bytes} bytes "
                f"(`bench.py --pmc-calibrate {args.cal_bytes}`); factor = bytes copied / "
                "counter reading of that copy.\n\n")
        if args.command:
            f.write("Commands:\n\n```\n" + args.command + "\n```\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
