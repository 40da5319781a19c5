"""Summarise rocprofv3 hardware-counter runs of a kernel into HBM bytes per
launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch, summed over the
dispatches of the kernel), each scaled by what the same counter reads for a
plain device copy of known size.

    python -m paper_1405_4644_amd.pmc_summary --fetch F.csv --write W.csv \\
        --cal-fetch CF.csv --cal-write CW.csv --cal-bytes 1073741824 \\
        --kernel-regex k_syrk_update_f32 --source paper_1405_4644_amd/csrc/k_update.hip \\
        --schedule 4,0,0 --input "..." --kernel "..." --workload "..." --command "..." --out X.json

The record keeps the sha256 of the kernel's source and the factorisation
schedule the counters ran under; bench.py reports the traffic only while
both still match.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import re
import sys


def _per_dispatch(path, regex):
    vals = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if regex and not re.search(regex, r.get("Kernel_Name", "")):
                continue
            key = r.get("Dispatch_Id") or r.get("Correlation_Id") or str(len(vals))
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"{path}: no dispatch matches {regex!r}")
    return sum(vals.values()) / len(vals), len(vals)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    for a in ("--fetch", "--write", "--cal-fetch", "--cal-write", "--out", "--source", "--kernel-regex"):
        ap.add_argument(a, required=True)
    ap.add_argument("--cal-bytes", type=int, required=True)
    ap.add_argument("--cal-regex", default="copyBuffer", help="the copy kernel's name in the calibration run")
    ap.add_argument("--schedule", required=True,
                    help="group,upd_slots,small_tiles of the factorisation the counters ran under")
    ap.add_argument("--input", default="")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--workload", default="")
    ap.add_argument("--command", action="append", default=[])
    args = ap.parse_args(argv)
    fetch, nd = _per_dispatch(args.fetch, args.kernel_regex)
    write, nw = _per_dispatch(args.write, args.kernel_regex)
    cf, _ = _per_dispatch(args.cal_fetch, args.cal_regex)
    cw, _ = _per_dispatch(args.cal_write, args.cal_regex)
    # calibration: the copy reads and writes cal_bytes each
    ff = cf * 1024.0 / args.cal_bytes
    fw = cw * 1024.0 / args.cal_bytes
    rd = fetch * 1024.0 / ff
    wr = write * 1024.0 / fw
    with open(args.source, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    g, s, sm = (int(x) for x in args.schedule.split(","))
    rec = {
        "kernel": args.kernel, "workload": args.workload, "input": args.input,
        "schedule": {"group": g, "upd_slots": s, "small_tiles": sm},
        "dispatches": nd, "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
        "copy_calibration": {"bytes": args.cal_bytes, "fetch_kib": cf, "write_kib": cw,
                             "fetch_factor": ff, "write_factor": fw},
        "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr, "traffic_bytes_per_launch": rd + wr,
        "source_sha256": sha, "source": args.source, "commands": args.command,
    }
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: rec[k] for k in ("dispatches", "traffic_bytes_per_launch", "schedule")}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
