"""Summaries of rocprofv3 CSV output for the kernels of this library.

    python -m paper_2006_06775_amd.rocprof_summary trace  <prefix>_kernel_trace.csv
    python -m paper_2006_06775_amd.rocprof_summary pmc    <prefix>_counter_collection.csv
    python -m paper_2006_06775_amd.rocprof_summary traffic --fetch F.csv --write W.csv --n N \
        --copy-bytes B --out traffic.json

`trace` prints per-kernel call counts and mean/min/max durations (the first call of each kernel
is dropped from the mean: it pays the first-touch page faults of fresh allocations).  `pmc`
prints per-kernel per-dispatch means of every collected counter.  `traffic` turns FETCH_SIZE
and WRITE_SIZE (KiB per dispatch) of the binary64 mechanics kernel into HBM bytes per launch,
each scaled by what the same counter reads for the copy kernel of a known size in the same run
(a copy of B bytes reads B and writes B), and writes the JSON that bench.py reports as
`roofline.traffic`, keyed by the digest of the kernel's sources.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MECH_SOURCES = ("paper_2006_06775_amd/csrc/k_mech.hip", "paper_2006_06775_amd/csrc/record8.hpp",
                "paper_2006_06775_amd/csrc/common.hpp")
MECH_KERNEL = "k_mech<64"
COPY_KERNEL = "copyBuffer"


def source_digest(paths=MECH_SOURCES):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str, width: int = 48) -> str:
    s = name.split("(")[0]
    if s.startswith("void "):
        s = s[5:]
    return s[:width]


def trace(path):
    durs = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            durs[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    rows = []
    for k, v in durs.items():
        body = v[1:] if len(v) > 1 else v
        rows.append((sum(v), short(k), len(v), statistics.mean(body), min(body), max(body)))
    rows.sort(reverse=True)
    print(f"{'kernel':48s} {'calls':>6s} {'mean_us':>9s} {'min_us':>9s} {'max_us':>9s}")
    for _, k, n, m, lo, hi in rows:
        print(f"{k:48s} {n:6d} {m:9.1f} {lo:9.1f} {hi:9.1f}")


def per_dispatch(path):
    """{kernel: {counter: [value of each dispatch]}} (values summed over the counter's instances)."""
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    with open(path) as f:
        for r in csv.DictReader(f):
            acc[(r["Kernel_Name"], r["Counter_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    out = collections.defaultdict(dict)
    for (k, c), d in acc.items():
        out[k][c] = [d[i] for i in sorted(d, key=int)]
    return out


def pmc(path):
    tab = per_dispatch(path)
    for k in sorted(tab, key=lambda k: -max(statistics.mean(v) for v in tab[k].values())):
        nd = max(len(v) for v in tab[k].values())
        vals = "  ".join(f"{c}={statistics.mean(v):.4g}" for c, v in sorted(tab[k].items()))
        print(f"{short(k):48s} dispatches={nd:3d}  {vals}")


def counter_of(tab, kernel_sub, counter, largest=False):
    """Mean per dispatch of `counter` for the kernel whose name contains kernel_sub; with
    `largest`, only over the dispatches within a factor 2 of the largest (the big copies)."""
    for k, v in tab.items():
        if kernel_sub in k and counter in v:
            vals = v[counter]
            if largest:
                top = max(vals)
                vals = [x for x in vals if x >= 0.5 * top]
            return statistics.mean(vals)
    raise KeyError(f"{counter} for {kernel_sub} not found")


def traffic(fetch_csv, write_csv, n, copy_bytes, out):
    tf, tw = per_dispatch(fetch_csv), per_dispatch(write_csv)
    kib = 1024.0
    copy_f = counter_of(tf, COPY_KERNEL, "FETCH_SIZE", largest=True) * kib
    copy_w = counter_of(tw, COPY_KERNEL, "WRITE_SIZE", largest=True) * kib
    f_scale, w_scale = copy_bytes / copy_f, copy_bytes / copy_w
    mech_f = counter_of(tf, MECH_KERNEL, "FETCH_SIZE") * kib * f_scale
    mech_w = counter_of(tw, MECH_KERNEL, "WRITE_SIZE") * kib * w_scale
    res = dict(n=n, kernel="k_mech<binary64>", fetch_bytes=mech_f, write_bytes=mech_w,
               bytes_per_launch=mech_f + mech_w, fetch_scale=f_scale, write_scale=w_scale,
               copy_bytes=copy_bytes, source_digest=source_digest())
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("trace")
    a.add_argument("csv")
    a = sub.add_parser("pmc")
    a.add_argument("csv")
    a = sub.add_parser("traffic")
    a.add_argument("--fetch", required=True)
    a.add_argument("--write", required=True)
    a.add_argument("--n", type=int, required=True)
    a.add_argument("--copy-bytes", type=int, required=True)
    a.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "trace":
        trace(args.csv)
    elif args.cmd == "pmc":
        pmc(args.csv)
    else:
        traffic(args.fetch, args.write, args.n, args.copy_bytes, args.out)


if __name__ == "__main__":
    main()
