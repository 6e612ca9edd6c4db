"""Summaries of rocprofv3 CSV output for the kernels of this library.

    python -m paper_2006_06775_amd.rocprof_summary trace  <prefix>_kernel_trace.csv
    python -m paper_2006_06775_amd.rocprof_summary pmc    <prefix>_counter_collection.csv
    python -m paper_2006_06775_amd.rocprof_summary bytes  --read R.csv --write W.csv --n N
    python -m paper_2006_06775_amd.rocprof_summary traffic --read R.csv --write W.csv --n N \
        --copy-bytes B --out traffic.json

`trace` prints per-kernel call counts and mean/min/max durations.  `pmc` prints per-kernel
per-dispatch means of every collected counter.  Both drop the first call of each kernel from
the mean: it pays the first-touch page faults of fresh allocations, and the first grid build
after generation sorts agents that arrive in id order rather than in the box order of a last
step (its gathers read about 900 B per agent instead of about 50).

HBM bytes: R.csv is a counter pass of TCC_EA0_RDREQ_32B_sum, TCC_EA0_RDREQ_64B_sum and
TCC_EA0_RDREQ_128B_sum (the L2's read requests to memory by size), W.csv one of WRITE_SIZE
(KiB, 32- and 64-byte write requests).  Read bytes are 32, 64 and 128 times the three counts.
(rocprofv3's FETCH_SIZE prices 128-byte requests through TCC_BUBBLE, which stays zero on this
device, and so counts each 128-byte read as 64 bytes.)  `bytes` prints every kernel's read and
write bytes per launch and per agent, and their sum over the kernels that run once per step
(as often as the mechanics kernel).  `traffic` writes the binary64 mechanics kernel's bytes per
launch as the JSON that bench.py reports as `roofline.traffic`, keyed by the digest of the
kernel's sources, with the copy kernel of B bytes in the same run as a check (a copy reads B
and writes B).
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
        body = steady(v)
        rows.append((sum(v), short(k), len(v), statistics.mean(body), min(body), max(body)))
    rows.sort(reverse=True)
    print(f"{'kernel':48s} {'calls':>6s} {'mean_us':>9s} {'min_us':>9s} {'max_us':>9s}")
    for _, k, n, m, lo, hi in rows:
        print(f"{k:48s} {n:6d} {m:9.1f} {lo:9.1f} {hi:9.1f}")


def steady(v):
    """The values of a kernel's calls without the first (when there are more)."""
    return v[1:] if len(v) > 1 else v


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
    for k in sorted(tab, key=lambda k: -max(statistics.mean(steady(v)) for v in tab[k].values())):
        nd = max(len(v) for v in tab[k].values())
        vals = "  ".join(f"{c}={statistics.mean(steady(v)):.4g}" for c, v in sorted(tab[k].items()))
        print(f"{short(k):48s} dispatches={nd:3d}  {vals}")


READ_SIZES = (("TCC_EA0_RDREQ_32B_sum", 32.0), ("TCC_EA0_RDREQ_64B_sum", 64.0), ("TCC_EA0_RDREQ_128B_sum", 128.0))


def dispatch_bytes(read_csv, write_csv):
    """{kernel: (read bytes of each dispatch, write bytes of each dispatch)}."""
    tr, tw = per_dispatch(read_csv), per_dispatch(write_csv)
    out = {}
    for k in set(tr) | set(tw):
        r = tr.get(k, {})
        nd = max([len(v) for v in r.values()] + [len(tw.get(k, {}).get("WRITE_SIZE", []))])
        rd = [sum(size * r[c][i] for c, size in READ_SIZES if c in r) for i in range(nd)]
        wr = tw.get(k, {}).get("WRITE_SIZE", [0.0] * nd)
        out[k] = (rd, [w * 1024.0 for w in wr])
    return out


def kernel_bytes(tab, kernel_sub, largest=False):
    """Mean (read, write) bytes per dispatch of the kernel whose name contains kernel_sub,
    without its first dispatch; with `largest`, only over the dispatches whose bytes are within
    a factor 2 of the largest (the big copies)."""
    for k, (rd, wr) in tab.items():
        if kernel_sub in k:
            pairs = list(zip(rd, wr))
            if largest:
                top = max(a + b for a, b in pairs)
                pairs = [p for p in pairs if sum(p) >= 0.5 * top]
            else:
                pairs = steady(pairs)
            return statistics.mean(p[0] for p in pairs), statistics.mean(p[1] for p in pairs)
    raise KeyError(f"no bytes for {kernel_sub}")


def bytes_table(read_csv, write_csv, n):
    tab = dispatch_bytes(read_csv, write_csv)
    steps = len(tab[next(k for k in tab if MECH_KERNEL in k)][0])
    rows = []
    for k, (rd, wr) in tab.items():
        r, w = statistics.mean(steady(rd)), statistics.mean(steady(wr))
        rows.append((r + w, short(k), len(rd), r, w))
    rows.sort(reverse=True)
    print(f"{'kernel':48s} {'calls':>6s} {'read_MB':>9s} {'write_MB':>9s} {'read_B/agent':>13s} {'write_B/agent':>14s}")
    tot_r = tot_w = 0.0
    for _, k, nd, r, w in rows:
        print(f"{k:48s} {nd:6d} {r / 1e6:9.1f} {w / 1e6:9.1f} {r / n:13.1f} {w / n:14.1f}")
        if nd == steps and not k.startswith("__amd"):
            tot_r += r
            tot_w += w
    print(f"per step (the library's kernels called {steps} times): read {tot_r / n:.1f} + write "
          f"{tot_w / n:.1f} = {(tot_r + tot_w) / n:.1f} B per agent")


def traffic(read_csv, write_csv, n, copy_bytes, out):
    tab = dispatch_bytes(read_csv, write_csv)
    copy_r, copy_w = kernel_bytes(tab, COPY_KERNEL, largest=True)
    mech_r, mech_w = kernel_bytes(tab, MECH_KERNEL)
    res = dict(n=n, kernel="k_mech<binary64>", fetch_bytes=mech_r, write_bytes=mech_w,
               bytes_per_launch=mech_r + mech_w,
               method="reads: 32/64/128 x TCC_EA0_RDREQ_{32B,64B,128B}; writes: WRITE_SIZE; first launch dropped",
               copy_read_ratio=copy_r / copy_bytes, copy_write_ratio=copy_w / copy_bytes,
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
    a = sub.add_parser("bytes")
    a.add_argument("--read", required=True)
    a.add_argument("--write", required=True)
    a.add_argument("--n", type=int, required=True)
    a = sub.add_parser("traffic")
    a.add_argument("--read", required=True)
    a.add_argument("--write", required=True)
    a.add_argument("--n", type=int, required=True)
    a.add_argument("--copy-bytes", type=int, required=True)
    a.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "trace":
        trace(args.csv)
    elif args.cmd == "pmc":
        pmc(args.csv)
    elif args.cmd == "bytes":
        bytes_table(args.read, args.write, args.n)
    else:
        traffic(args.read, args.write, args.n, args.copy_bytes, args.out)


if __name__ == "__main__":
    main()
