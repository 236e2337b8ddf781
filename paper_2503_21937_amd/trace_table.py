"""Launch sizes against launch times: joins a rocprofv3 kernel trace
(``*_kernel_trace.csv``) with the fused-round launches of the engines'
round logs (``dl_get_round_log``) that ``bench.py --round-log`` writes, and
prints a markdown table per size class of the fused
round kernel (derivations per launch): launches, average duration,
algorithmic bytes (driver rows plus derivations, key and tag each) and the
rate they imply.

The last launches of the kernel in the trace are taken to be those of the
log, in order (the log covers the engines' last runs, which end the traced
program).

    python -m paper_2503_21937_amd.trace_table TRACE.csv ROUND_LOG.jsonl
"""
from __future__ import annotations

import csv
import json
import sys

KERNEL = "k_window_round"
CLASSES = [(0, 0, "0 (after the last round)"), (1, 10**5, "1 .. 1e5"), (10**5, 10**6, "1e5 .. 1e6"),
           (10**6, 10**7, "1e6 .. 1e7"), (10**7, 10**12, ">= 1e7")]


def main(trace: str, log: str, peak_gbs: float = 8000.0) -> str:
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
    if len(entries) > len(us):
        raise SystemExit(f"log has {len(entries)} launches, trace {len(us)}")
    us = us[len(us) - len(entries):]
    out = ["| derivations per launch | launches | avg us | total us | share | avg MB | GB/s | of HBM peak |",
           "|---|---|---|---|---|---|---|---|"]
    total = sum(us)
    for lo, hi, name in CLASSES:
        sel = [(t, b) for t, (c, b) in zip(us, entries) if (c == 0 if hi == 0 else lo <= c < hi)]
        if not sel:
            continue
        t = sum(x for x, _ in sel)
        b = sum(y for _, y in sel)
        rate = b / (t * 1e-6) / 1e9 if t > 0 else 0.0
        out.append(f"| {name} | {len(sel)} | {t / len(sel):.1f} | {t:.0f} | {t / total:.1%} | "
                   f"{b / len(sel) / 1e6:.2f} | {rate:.0f} | {rate / peak_gbs:.3f} |")
    t = total
    b = sum(y for _, y in entries)
    out.append(f"| all | {len(entries)} | {t / len(entries):.1f} | {t:.0f} | 100% | {b / len(entries) / 1e6:.2f} | "
               f"{b / (t * 1e-6) / 1e9:.0f} | {b / (t * 1e-6) / 1e9 / peak_gbs:.3f} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(main(sys.argv[1], sys.argv[2]))
