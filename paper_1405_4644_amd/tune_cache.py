"""Write a factorisation-schedule cache (the autotuner's choices) for given
orders and precisions, for SPD_TUNE_CACHE or to ship with the package.

    python -m paper_1405_4644_amd.tune_cache --out tune_cache.json 16384:fp32,fp16,fp64 70000:fp32,fp64

Each entry is timed on this GPU by spd_autotune (orders are rounded to a
power of two in the key) and stored in the JSON file by the library itself.
"""
from __future__ import annotations

import argparse
import json
import os
import sys


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True, help="cache file to write (replaced)")
    ap.add_argument("specs", nargs="+", help="n:prec[,prec...]")
    args = ap.parse_args(argv)
    out = os.path.abspath(args.out)
    if os.path.exists(out):
        os.remove(out)
    os.environ["SPD_TUNE_CACHE"] = out
    import paper_1405_4644_amd as spd
    spd.autotune_clear()
    for spec in args.specs:
        n, precs = spec.split(":")
        for p in precs.split(","):
            r = spd.autotune(int(n), p)
            print(f"n={n} {p}: {r}", flush=True)
    with open(out) as f:
        json.load(f)  # written by the library; check it parses
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
