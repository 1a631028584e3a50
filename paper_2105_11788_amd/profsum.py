"""Condense rocprofv3 CSV output into the short text summaries kept with the
project (per-kernel durations, per-dispatch counter means, calibrated memory
traffic).

    python -m paper_2105_11788_amd.profsum stats  KERNEL_STATS.csv
    python -m paper_2105_11788_amd.profsum pmc    COUNTER_COLLECTION.csv
    python -m paper_2105_11788_amd.profsum traffic --kernel REGEX \\
        --fetch A.csv --write B.csv --copy-fetch C.csv --copy-write D.csv \\
        --copy-bytes N --sources DIR [--source-files a.hip,b.h]

`traffic` scales each counter by what it reads for a plain copy of N bytes
(each byte read once and written once), and prints `key: value` lines that
bench.py reads back, including a digest of the kernel sources so that stale
counters are not reported for changed kernels.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys
from collections import defaultdict


def short(name: str, width: int = 60) -> str:
    name = name.replace("bisim::(anonymous namespace)::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def source_digest(root: str, files: list[str] | None = None) -> str:
    """sha1 over kernel sources (names and contents, sorted): the listed files
    of `root`, else every .hip and .h file there."""
    h = hashlib.sha1()
    names = files if files else [f for f in os.listdir(root) if f.endswith((".hip", ".h"))]
    for f in sorted(names):
        h.update(f.encode())
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_rows(path: str):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def cmd_stats(a) -> None:
    rows = read_rows(a.csv)
    print("| kernel | calls | avg us | total ms | min us | max us | share % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for r in rows[: a.top]:
        print(f"| {short(r['Name'])} | {int(r['Calls'])} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
              f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")


def counter_means(path: str, regex: str | None = None):
    """{(kernel, counter): (dispatches, mean value)} over a counter CSV."""
    acc = defaultdict(lambda: [0, 0.0])
    pat = re.compile(regex) if regex else None
    for r in read_rows(path):
        k = r.get("Kernel_Name", r.get("Kernel-Name", ""))
        if pat and not pat.search(k):
            continue
        c = r.get("Counter_Name", r.get("Counter-Name", ""))
        v = float(r.get("Counter_Value", r.get("Counter-Value", "0")))
        e = acc[(k, c)]
        e[0] += 1
        e[1] += v
    return {key: (e[0], e[1] / e[0]) for key, e in acc.items() if e[0]}


def cmd_pmc(a) -> None:
    print("| kernel | counter | dispatches | mean per dispatch |")
    print("|---|---|---:|---:|")
    for (k, c), (cnt, mean) in sorted(counter_means(a.csv, a.kernel).items()):
        print(f"| {short(k)} | {c} | {cnt} | {mean:.1f} |")


def one_mean(path: str, regex: str, counter: str) -> tuple[int, float]:
    hits = [(cnt, mean) for (k, c), (cnt, mean) in counter_means(path, regex).items()
            if c == counter]
    if not hits:
        sys.exit(f"profsum: no {counter} rows for /{regex}/ in {path}")
    n = sum(h[0] for h in hits)
    return n, sum(h[0] * h[1] for h in hits) / n


def cmd_traffic(a) -> None:
    nf, fetch = one_mean(a.fetch, a.kernel, "FETCH_SIZE")
    nw, write = one_mean(a.write, a.kernel, "WRITE_SIZE")
    _, cf = one_mean(a.copy_fetch, "k_copy16", "FETCH_SIZE")
    _, cw = one_mean(a.copy_write, "k_copy16", "WRITE_SIZE")
    kib = a.copy_bytes / 1024.0
    ff, fw = kib / cf, kib / cw
    traffic = (fetch * ff + write * fw) * 1024.0
    files = [f for f in a.source_files.split(",") if f] if a.source_files else None
    print(f"kernel_regex: {a.kernel}")
    if files:
        print(f"source_files: {','.join(sorted(files))}")
    print(f"source_sha1: {source_digest(a.sources, files)}")
    print(f"fetch_dispatches: {nf}")
    print(f"fetch_kib_per_dispatch: {fetch:.3f}")
    print(f"write_dispatches: {nw}")
    print(f"write_kib_per_dispatch: {write:.3f}")
    print(f"copy_bytes: {a.copy_bytes}")
    print(f"copy_fetch_kib: {cf:.1f}")
    print(f"copy_write_kib: {cw:.1f}")
    print(f"fetch_factor: {ff:.4f}")
    print(f"write_factor: {fw:.4f}")
    print(f"traffic_bytes_per_launch: {traffic:.0f}")


def main(argv=None) -> None:
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = p.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    s.set_defaults(fn=cmd_stats)
    s = sub.add_parser("pmc")
    s.add_argument("csv")
    s.add_argument("--kernel", default=None)
    s.set_defaults(fn=cmd_pmc)
    s = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        s.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    s.add_argument("--kernel", required=True)
    s.add_argument("--copy-bytes", type=int, default=1 << 30)
    s.add_argument("--sources", default=os.path.join(os.path.dirname(__file__), "csrc"))
    s.add_argument("--source-files", default="",
                   help="comma-separated files of --sources that the kernel is built from "
                        "(default: all of them)")
    s.set_defaults(fn=cmd_traffic)
    a = p.parse_args(argv)
    a.fn(a)


if __name__ == "__main__":
    main()
