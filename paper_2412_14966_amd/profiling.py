"""Summaries of rocprofv3 CSV output for the committed profile records.

``python -m paper_2412_14966_amd.profiling trace DIR``
    per-kernel call count and average / min / max duration from the
    ``*_kernel_stats.csv`` (or ``*_kernel_trace.csv``) files under DIR.
``python -m paper_2412_14966_amd.profiling counters DIR COUNTER``
    per-kernel mean value of one PMC counter per dispatch from the
    ``*_counter_collection.csv`` files under DIR.
``python -m paper_2412_14966_amd.profiling traffic FETCH_DIR WRITE_DIR --copy-mib M --kernel NAME``
    HBM bytes per launch of kernel NAME from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by the factor that makes a plain copy of
    M MiB read and write M MiB; prints the record that bench.py reads.

Only text parsing: nothing here touches the GPU.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys
from collections import defaultdict
from typing import Dict, List


def _rows(root: str, suffix: str) -> List[dict]:
    rows = []
    for path in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _col(row: dict, *names: str):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {list(row)}")


def short_name(name: str) -> str:
    """Kernel name without argument list."""
    return name.split("(")[0].strip()


def kernel_times(root: str) -> Dict[str, dict]:
    """Per-kernel {calls, avg_ns, min_ns, max_ns} from a kernel trace."""
    out: Dict[str, dict] = {}
    trace = _rows(root, "kernel_trace.csv")
    if trace:
        durs = defaultdict(list)
        for r in trace:
            durs[short_name(_col(r, "Kernel_Name"))].append(int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp")))
        for k, d in durs.items():
            out[k] = dict(calls=len(d), avg_ns=sum(d) / len(d), min_ns=min(d), max_ns=max(d))
        return out
    for r in _rows(root, "kernel_stats.csv"):
        out[short_name(_col(r, "Name"))] = dict(calls=int(_col(r, "Calls")), avg_ns=float(_col(r, "AverageNs")),
                                                min_ns=float(_col(r, "MinNs")), max_ns=float(_col(r, "MaxNs")))
    return out


def counter_means(root: str, counter: str) -> Dict[str, dict]:
    """Per-kernel mean of `counter` per dispatch (summed over the counter's
    instances within a dispatch)."""
    per = defaultdict(lambda: defaultdict(float))
    for r in _rows(root, "counter_collection.csv"):
        if _col(r, "Counter_Name") != counter:
            continue
        disp = _col(r, "Dispatch_Id", "Correlation_Id")
        per[short_name(_col(r, "Kernel_Name"))][disp] += float(_col(r, "Counter_Value"))
    return {k: dict(dispatches=len(v), mean=sum(v.values()) / len(v)) for k, v in per.items()}


def _pick(d: Dict[str, dict], key: str) -> str:
    hits = [k for k in d if key in k]
    if not hits:
        raise SystemExit(f"no kernel matching {key!r}: {sorted(d)}")
    return hits[0]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("counter")
    h = sub.add_parser("traffic")
    h.add_argument("fetch_dir")
    h.add_argument("write_dir")
    h.add_argument("--copy-mib", type=float, required=True)
    h.add_argument("--copy-kernel", default="copy", help="substring naming the calibration copy kernel")
    h.add_argument("--kernel", required=True, help="substring naming the profiled kernel")
    h.add_argument("--workload", default="")
    h.add_argument("--kernel-sha", default="")
    a = ap.parse_args(argv)

    if a.cmd == "trace":
        print("| kernel | calls | avg us | min us | max us |\n|---|---|---|---|---|")
        for k, v in sorted(kernel_times(a.dir).items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
            print(f"| `{k}` | {v['calls']} | {v['avg_ns'] / 1e3:.1f} | {v['min_ns'] / 1e3:.1f} | {v['max_ns'] / 1e3:.1f} |")
        return 0
    if a.cmd == "counters":
        print(f"| kernel | dispatches | mean {a.counter} per dispatch |\n|---|---|---|")
        for k, v in sorted(counter_means(a.dir, a.counter).items()):
            print(f"| `{k}` | {v['dispatches']} | {v['mean']:.6g} |")
        return 0
    fetch = counter_means(a.fetch_dir, "FETCH_SIZE")
    write = counter_means(a.write_dir, "WRITE_SIZE")
    copy_kib = a.copy_mib * 1024.0
    kf, kw = _pick(fetch, a.copy_kernel), _pick(write, a.copy_kernel)
    f_scale = copy_kib / fetch[kf]["mean"]
    w_scale = copy_kib / write[kw]["mean"]
    mf, mw = _pick(fetch, a.kernel), _pick(write, a.kernel)
    fetch_b = fetch[mf]["mean"] * f_scale * 1024.0
    write_b = write[mw]["mean"] * w_scale * 1024.0
    rec = dict(workload=a.workload, kernel_sha=a.kernel_sha, kernel=mf,
               fetch_kib_raw=fetch[mf]["mean"], write_kib_raw=write[mw]["mean"],
               copy_kernel=kf, copy_fetch_kib_raw=fetch[kf]["mean"], copy_write_kib_raw=write[kw]["mean"],
               fetch_scale=f_scale, write_scale=w_scale, hbm_bytes_per_launch=fetch_b + write_b)
    json.dump(rec, sys.stdout, indent=1)
    print()
    return 0


if __name__ == "__main__":
    sys.exit(main())
