"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_1905_13746_amd.rocprof_summary traffic \\
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --kernel SUBSTRING --algo-bytes N --sources FILE [FILE ...] --out JSON

reads the rocpd databases that `rocprofv3 --pmc FETCH_SIZE` / `--pmc
WRITE_SIZE` wrote for the kernel under study and for a plain device copy of
known size (`bench.py --copy-calibration`), scales each counter by what it
reads for the copy, and writes HBM bytes per launch next to the algorithmic
bytes, with a hash of the kernel's source files (a summary is only valid for
the source it was taken on).

    python -m paper_1905_13746_amd.rocprof_summary stats DIR [SUBSTRING]

prints per-kernel dispatch counts and mean/min/max durations from a
`--kernel-trace` database.

    python -m paper_1905_13746_amd.rocprof_summary counters DIR [SUBSTRING]

prints, per kernel, the mean per dispatch of every counter a `--pmc` run
collected (values summed over the counter's instances per dispatch).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)


def source_hash(paths) -> str:
    """SHA-256 over the named source files (repository-relative), in order."""
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(p.encode() + b"\0" + f.read())
    return h.hexdigest()


def _db(d):
    dbs = sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))
    if not dbs:
        raise FileNotFoundError(f"no rocpd database under {d}")
    return sqlite3.connect(dbs[0])


def counter_per_dispatch(d, counter, kernel):
    """Mean of `counter` over the dispatches whose kernel name contains
    `kernel` (values summed over the counter's instances per dispatch)."""
    c = _db(d)
    per = {}
    for name, cn, val, disp in c.execute(
            "select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        if kernel in name and cn == counter:
            per[disp] = per.get(disp, 0.0) + float(val)
    if not per:
        raise ValueError(f"{counter} for '{kernel}' not found in {d}")
    return sum(per.values()) / len(per), len(per)


def traffic(a):
    fetch, nd = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
    write, _ = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel)
    cf, _ = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw, _ = counter_per_dispatch(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    fetch_factor = a.copy_bytes / (cf * 1024.0)
    write_factor = a.copy_bytes / (cw * 1024.0)
    hbm = fetch * 1024.0 * fetch_factor + write * 1024.0 * write_factor
    out = {"kernel": a.kernel, "fetch_kib_per_dispatch_raw": fetch, "write_kib_per_dispatch_raw": write,
           "dispatches": nd,
           "copy_calibration": {"bytes_per_dispatch": a.copy_bytes, "fetch_kib_raw": cf, "write_kib_raw": cw,
                                "fetch_factor": fetch_factor, "write_factor": write_factor},
           "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": a.algo_bytes,
           "traffic_over_algorithmic": hbm / a.algo_bytes,
           "sources": a.sources, "source_sha256": source_hash(a.sources)}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def stats(a):
    c = _db(a.dir)
    rows = {}
    for name, start, end in c.execute("select name, start, \"end\" from kernels"):
        if a.kernel and a.kernel not in name:
            continue
        rows.setdefault(name, []).append((end - start) / 1e3)
    for name, ds in sorted(rows.items(), key=lambda kv: -sum(kv[1])):
        print(f"{len(ds):6d}  mean {sum(ds) / len(ds):10.2f} us  min {min(ds):10.2f}  max {max(ds):10.2f}  {name[:110]}")


def counters(a):
    c = _db(a.dir)
    per = {}
    for name, cn, val, disp in c.execute(
            "select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        if a.kernel and a.kernel not in name:
            continue
        d = per.setdefault(name, {}).setdefault(cn, {})
        d[disp] = d.get(disp, 0.0) + float(val)
    for name, cs in sorted(per.items()):
        print(name[:140])
        for cn, ds in sorted(cs.items()):
            print(f"    {cn:32s} {sum(ds.values()) / len(ds):20.1f}   ({len(ds)} dispatches)")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-kernel", default="copy")
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--algo-bytes", type=float, required=True)
    t.add_argument("--sources", nargs="+", required=True)
    t.add_argument("--out", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("kernel", nargs="?", default="")
    k = sub.add_parser("counters")
    k.add_argument("dir")
    k.add_argument("kernel", nargs="?", default="")
    a = ap.parse_args(argv)
    {"traffic": traffic, "stats": stats, "counters": counters}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
