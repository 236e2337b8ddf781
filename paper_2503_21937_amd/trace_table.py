"""Launch sizes against launch times: joins a rocprofv3 kernel trace
(``*_kernel_trace.csv``) with the fused-round launches of the engines'
round logs (``dl_get_round_log``) that ``bench.py --round-log`` writes, and
prints a markdown table per size class of the fused round kernel
(derivations per launch): launches, average duration, algorithmic bytes
(driver rows plus derivations, key and tag each) and the rate they imply.
Given the per-dispatch counter files of ``rocprofv3 --pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE`` runs of the same program (and the factors that scale
each counter to bytes, from a plain copy of known size), it adds the HBM
traffic per launch and its ratio to the algorithmic bytes.

The last launches of the kernel in each file are taken to be those of the
log, in order (the log covers the engines' last runs, which end the traced
program, and the fixpoint's rounds are the same in every run).

    python -m paper_2503_21937_amd.trace_table TRACE.csv ROUND_LOG.jsonl \\
        [FETCH.csv WRITE.csv FETCH_SCALE WRITE_SCALE]
"""
from __future__ import annotations

import csv
import json
import sys

KERNEL = "k_window_round"
CLASSES = [(0, 0, "0 (after the last round)"), (1, 10**5, "1 .. 1e5"), (10**5, 10**6, "1e5 .. 1e6"),
           (10**6, 10**7, "1e6 .. 1e7"), (10**7, 10**12, ">= 1e7")]


def _counter(path: str, name: str) -> list[float]:
    """Per-dispatch values (KiB) of one counter for the kernel, in dispatch order."""
    per: dict[int, float] = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if KERNEL in r["Kernel_Name"] and r["Counter_Name"] == name:
                d = int(r["Dispatch_Id"])
                per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    return [per[d] for d in sorted(per)]


def main(trace: str, log: str, fetch: str | None = None, write: str | None = None, fetch_scale: float = 1.0,
         write_scale: float = 1.0, peak_gbs: float = 8000.0) -> str:
    with open(trace) as f:
        rows = [r for r in csv.DictReader(f) if KERNEL in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
    entries = []
    with open(log) as f:
        for line in f:
            d = json.loads(line)
            for c in d["derivations"]:
                entries.append((int(c), (d["driver_rows"] + int(c)) * d["bytes_per_unit"]))
    n = len(entries)
    if n > len(us):
        raise SystemExit(f"log has {n} launches, trace {len(us)}")
    us = us[len(us) - n:]
    traffic = None
    if fetch and write:
        fk, wk = _counter(fetch, "FETCH_SIZE"), _counter(write, "WRITE_SIZE")
        if min(len(fk), len(wk)) < n:
            raise SystemExit("the counter runs hold fewer launches than the log")
        traffic = [(a * fetch_scale + b * write_scale) * 1024.0 for a, b in zip(fk[len(fk) - n:], wk[len(wk) - n:])]
    head = "| derivations per launch | launches | avg us | total us | share | avg MB | GB/s | of HBM peak |"
    rule = "|---|---|---|---|---|---|---|---|"
    if traffic:
        head += " traffic MB | traffic / algorithmic |"
        rule += "---|---|"
    out = [head, rule]
    total = sum(us)

    def line(name, idx):
        t = sum(us[i] for i in idx)
        b = sum(entries[i][1] for i in idx)
        rate = b / (t * 1e-6) / 1e9 if t > 0 else 0.0
        s = (f"| {name} | {len(idx)} | {t / len(idx):.1f} | {t:.0f} | {t / total:.1%} | "
             f"{b / len(idx) / 1e6:.2f} | {rate:.0f} | {rate / peak_gbs:.3f} |")
        if traffic:
            tr = sum(traffic[i] for i in idx)
            s += f" {tr / len(idx) / 1e6:.2f} | {tr / b:.2f} |"
        return s

    for lo, hi, name in CLASSES:
        idx = [i for i, (c, _) in enumerate(entries) if (c == 0 if hi == 0 else lo <= c < hi)]
        if idx:
            out.append(line(name, idx))
    out.append(line("all", list(range(n))))
    return "\n".join(out)


if __name__ == "__main__":
    a = sys.argv[1:]
    if len(a) >= 6:
        print(main(a[0], a[1], a[2], a[3], float(a[4]), float(a[5])))
    else:
        print(main(a[0], a[1]))
