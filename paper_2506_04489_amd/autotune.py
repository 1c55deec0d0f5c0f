"""Autotune the pass launch shapes on the current GPU and write the table.

For every requested n and tier this creates a plan (h = 2/n, R = 40),
precomputes it and calls ``psp_autotune``, which times every (radix plan,
tile) candidate of every pass and keeps the fastest.  The table is JSON:

    {"device": "...", "reps": 5,
     "entries": [{"n": 256, "dtype": "f64", "plan": [...], "tile": [...],
                  "pass_ms": [...], "candidates_ms": [...]}, ...]}

``psp.load_tuning`` reads it back; the binding loads
``tuning_gfx950.json`` next to this file on first use.

Usage: python -m paper_2506_04489_amd.autotune --out table.json [--n 64 128] [--dtype f64 f32]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

SIZES = [16, 24, 32, 48, 64, 96, 128, 192, 256, 384]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, nargs="*", default=SIZES)
    ap.add_argument("--dtype", nargs="*", default=["f64", "f32"])
    ap.add_argument("--reps", type=int, default=31)
    args = ap.parse_args(argv)
    import os
    os.environ["PSP_TUNING_FILE"] = "none"      # start from the default shapes
    import torch
    from paper_2506_04489_amd import psp as B
    entries = []
    for dt in args.dtype:
        for n in args.n:
            t0 = time.time()
            p = B.Plan(n, 2.0 / n, 40, dtype=dt).precompute()
            res = p.autotune(reps=args.reps)
            torch.cuda.synchronize()
            entries.append({"n": n, "dtype": dt, **res})
            print("n=%d %s plan=%s tile=%s pass_ms=%s (%.1f s)" % (
                n, dt, res["plan"], res["tile"], ["%.4f" % x for x in res["pass_ms"]], time.time() - t0),
                flush=True)
            for i, row in enumerate(res["candidates_ms"]):
                print("    H%d candidates (plan*21+tile): %s" % (i + 1, [x for x in row if x >= 0]), flush=True)
            del p
    doc = {"device": torch.cuda.get_device_name(0), "reps": args.reps, "entries": entries}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
