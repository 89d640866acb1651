"""Summaries of rocprofv3 output for the committed measurement records.

Two commands, both reading the CSV files that ``rocprofv3 --output-format
csv`` writes:

``python -m paper_2504_17615_amd.profiling stats OUT.txt KERNEL_STATS.csv --cmd "..."``
    writes the per-kernel summary (calls, total and average duration, share)
    of a ``--kernel-trace --stats`` run.

``python -m paper_2504_17615_amd.profiling traffic OUT.json FETCH.csv WRITE.csv
--calib-mib N --workload W --source FILE --cmd-fetch "..." --cmd-write "..."``
    turns two counter runs (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``,
    KiB per dispatch) into HBM bytes per launch of every traced kernel.  Each
    counter is scaled by the factor that makes it read the known size of a
    plain float32 copy (``torch.neg`` of N MiB: N MiB read, N MiB written)
    launched in the same run.  The record carries the SHA-256 of the kernel
    source, so that a reader can tell when the kernel changed since.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def short_name(kernel: str) -> str:
    """'void lmgp::(anonymous namespace)::k_rate_big<2>(lmgp::RateArgs)' ->
    'k_rate_big<2>'."""
    k = kernel.strip()
    if k.startswith("void "):
        k = k[5:]
    depth, cut = 0, len(k)
    for i, ch in enumerate(k):  # drop the argument list (first '(' at depth 0
        if ch == "<":           # after the name)
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0 and k[i - 1] not in ": ":
            cut = i
            break
    k = k[:cut]
    lt = k.find("<")
    head, tmpl = (k, "") if lt < 0 else (k[:lt], k[lt:])
    return head.split("::")[-1] + tmpl


def write_stats(out: str, stats_csv: str, cmd: str, top: int = 40) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {cmd}",
             f"# kernels: {len(rows)} distinct, {sum(int(r['Calls']) for r in rows)} dispatches, "
             f"{tot / 1e6:.2f} ms total", "",
             f"{'calls':>7} {'total_ms':>10} {'avg_us':>10} {'share':>6}  kernel"]
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.2f} "
                     f"{float(r['AverageNs']) / 1e3:10.1f} {100 * float(r['TotalDurationNs']) / tot:5.1f}%"
                     f"  {short_name(r['Name'])}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_per_kernel(path: str, counter: str):
    per = defaultdict(lambda: [0, 0.0])  # kernel -> [dispatches, summed KiB]
    seen = set()
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        key = (r.get("Dispatch_Id"), r.get("Correlation_Id"))
        k = short_name(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        if key in seen:  # one row per dimension instance: sum them
            per[k][1] += v
            continue
        seen.add(key)
        per[k][0] += 1
        per[k][1] += v
    return per


def write_traffic(out: str, fetch_csv: str, write_csv: str, calib_mib: int, workload: str,
                  source: str, cmd_fetch: str, cmd_write: str, copy_regex: str = "neg") -> None:
    fetch = _counter_per_kernel(fetch_csv, "FETCH_SIZE")
    write = _counter_per_kernel(write_csv, "WRITE_SIZE")
    rx = re.compile(copy_regex)
    cf = [k for k in fetch if rx.search(k)]
    cw = [k for k in write if rx.search(k)]
    if len(cf) != 1 or len(cw) != 1:
        raise SystemExit(f"expected one copy kernel matching {copy_regex!r}: {cf} {cw}")
    known_kib = calib_mib * 1024.0
    f_fac = known_kib / (fetch[cf[0]][1] / fetch[cf[0]][0])
    w_fac = known_kib / (write[cw[0]][1] / write[cw[0]][0])
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        if rx.search(k):
            continue
        fk = fetch[k][1] / fetch[k][0] * f_fac
        wk = write[k][1] / write[k][0] * w_fac
        kernels[k] = {"dispatches": fetch[k][0], "fetch_kib_per_launch": round(fk, 1),
                      "write_kib_per_launch": round(wk, 1),
                      "hbm_bytes_per_launch": int(round((fk + wk) * 1024))}
    src = os.path.join(ROOT, source)
    rec = {"workload": workload, "source": source,
           "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
           "calibration": {"copy_kernel": cf[0], "copy_mib": calib_mib,
                           "fetch_factor": round(f_fac, 4), "write_factor": round(w_fac, 4)},
           "commands": {"fetch": cmd_fetch, "write": cmd_write}, "kernels": kernels}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("out")
    s.add_argument("stats_csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--top", type=int, default=40)
    t = sub.add_parser("traffic")
    t.add_argument("out")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--calib-mib", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--source", required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    a = ap.parse_args()
    if a.what == "stats":
        write_stats(a.out, a.stats_csv, a.cmd, a.top)
    else:
        write_traffic(a.out, a.fetch_csv, a.write_csv, a.calib_mib, a.workload, a.source,
                      a.cmd_fetch, a.cmd_write)


if __name__ == "__main__":
    main()
