"""Turn rocprofv3 CSV output into the short summaries kept with the code.

    # kernel time table (from `rocprofv3 --kernel-trace --stats -f csv`)
    python -m paper_1605_04521_amd.profiling stats --csv OUT_kernel_stats.csv

    # HBM traffic per launch (from two `rocprofv3 --pmc ... -f csv` runs of
    # `bench.py --workload kernels`, one with FETCH_SIZE, one with WRITE_SIZE)
    python -m paper_1605_04521_amd.profiling traffic --fetch F_counter_collection.csv \\
        --write W_counter_collection.csv --precision fp64 --nrhs 1 --out profiles/traffic.json

FETCH_SIZE and WRITE_SIZE count, in KiB per dispatch, the bytes the L2
caches request from and send to memory.  Each is scaled by the reading it
gives for a device copy of known size (1 GiB read, 1 GiB written) in the same
run, so the figures are bytes, whatever the counter's aggregation over the
chip's cache instances.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel key -> (name pattern, source file)
KERNELS = {
    "lu": (r"k_lu(_queue)?<", "lu_kernels.hip"),
    "local_solve_multi": (r"k_local_solve_multi(_tall)?<", "multi_solve.hip"),
    "local_solve": (r"k_local_solve<", "solve_kernels.hip"),
    "spmv": (r"k_sp(mv|mm)(_il)?[<(]", "solve_kernels.hip"),
}


def source_hash(name: str) -> str:
    h = hashlib.sha256()
    with open(os.path.join(HERE, "csrc", name), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def kernel_key(name: str):
    for key, (pat, _) in KERNELS.items():
        if re.search(pat, name):
            return key
    return None


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(f"none of {names} in {list(row)}")


def read_counters(path: str, counter: str):
    """[(kernel name, value)] per dispatch for one counter."""
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if _col(row, "Counter_Name") != counter:
                continue
            out.append((_col(row, "Kernel_Name"), float(_col(row, "Counter_Value"))))
    return out


def copy_scale(rows, copy_bytes: int) -> float:
    """Bytes per counter unit, from the largest copy dispatch."""
    cands = [v for name, v in rows if "copy" in name.lower()]
    if not cands or max(cands) <= 0:
        raise ValueError("no copy dispatch with a non-zero reading found")
    return copy_bytes / max(cands)


def traffic(fetch_csv: str, write_csv: str, copy_bytes: int = 1 << 30):
    fetch = read_counters(fetch_csv, "FETCH_SIZE")
    write = read_counters(write_csv, "WRITE_SIZE")
    sf, sw = copy_scale(fetch, copy_bytes), copy_scale(write, copy_bytes)
    res = {}
    for key in KERNELS:
        fv = [v for name, v in fetch if kernel_key(name) == key]
        wv = [v for name, v in write if kernel_key(name) == key]
        if not fv or not wv:
            continue
        fb, wb = sf * sum(fv) / len(fv), sw * sum(wv) / len(wv)
        res[key] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                    "dispatches": [len(fv), len(wv)], "copy_scale": [sf, sw],
                    "source_hash": source_hash(KERNELS[key][1])}
    return res


def stats_table(path: str, top: int = 20) -> str:
    rows = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            rows.append((_col(row, "Name", "KernelName"), int(float(_col(row, "Calls"))),
                         float(_col(row, "TotalDurationNs")) / 1e6, float(_col(row, "AverageNs")) / 1e6,
                         float(_col(row, "Percentage"))))
    rows.sort(key=lambda r: -r[2])
    lines = ["| kernel | calls | total ms | average ms | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows[:top]:
        lines.append(f"| `{name[:90]}` | {calls} | {tot:.2f} | {avg:.4f} | {pct:.2f} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--csv", required=True)
    a.add_argument("--top", type=int, default=20)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--precision", required=True)
    b.add_argument("--nrhs", type=int, required=True)
    b.add_argument("--nsub", default="", help="partition of the run (part of the record's key)")
    b.add_argument("--out", required=True)
    b.add_argument("--copy-bytes", type=int, default=1 << 30)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_table(args.csv, args.top))
        return
    res = traffic(args.fetch, args.write, args.copy_bytes)
    data = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            data = json.load(f)
    for key, rec in res.items():
        data[f"{key}|{args.precision}|{args.nrhs}" + (f"|{args.nsub}" if args.nsub else "")] = rec
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    json.dump(res, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
