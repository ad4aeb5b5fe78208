"""Summaries of rocprofv3 CSV output for the committed profile records.

``python -m paper_2412_14966_amd.profiling trace DIR``
    per-(kernel, grid size) call count and average / min / max duration from
    the ``*_kernel_trace.csv`` files under DIR.
``python -m paper_2412_14966_amd.profiling counters DIR COUNTER``
    per-(kernel, grid size) value of one PMC counter per dispatch from the
    ``*_counter_collection.csv`` files under DIR.
``python -m paper_2412_14966_amd.profiling traffic FETCH_DIR WRITE_DIR --copy-mib M --kernel NAME``
    HBM bytes per launch of kernel NAME from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch, largest-grid launches of NAME), each scaled by the factor
    that makes the largest dispatch of a plain copy kernel read and write M MiB;
    prints the record that bench.py reads.

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


def _grid(row: dict) -> int:
    for names in (("Grid_Size",), ("Grid_Size_X",)):
        try:
            return int(_col(row, *names))
        except KeyError:
            pass
    return 0


def kernel_times(root: str) -> Dict[tuple, dict]:
    """Per-(kernel, grid size) {calls, avg_ns, min_ns, max_ns} from a kernel trace."""
    durs = defaultdict(list)
    for r in _rows(root, "kernel_trace.csv"):
        key = (short_name(_col(r, "Kernel_Name")), _grid(r))
        durs[key].append(int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp")))
    return {k: dict(calls=len(d), avg_ns=sum(d) / len(d), min_ns=min(d), max_ns=max(d)) for k, d in durs.items()}


def counter_values(root: str, counter: str) -> Dict[tuple, List[float]]:
    """Per-(kernel, grid size) list of `counter` per dispatch (summed over the
    counter's instances within a dispatch)."""
    per = defaultdict(lambda: defaultdict(float))
    for r in _rows(root, "counter_collection.csv"):
        if _col(r, "Counter_Name") != counter:
            continue
        disp = _col(r, "Dispatch_Id", "Correlation_Id")
        per[(short_name(_col(r, "Kernel_Name")), _grid(r))][disp] += float(_col(r, "Counter_Value"))
    return {k: list(v.values()) for k, v in per.items()}


def _largest(d: Dict[tuple, object], key: str) -> tuple:
    """(kernel, grid) entry of the kernel matching `key` with the largest grid."""
    hits = [k for k in d if key in k[0]]
    if not hits:
        raise SystemExit(f"no kernel matching {key!r}: {sorted(set(k[0] for k in d))}")
    return max(hits, key=lambda k: k[1])


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
    h.add_argument("--schedule", type=lambda t: [int(x) for x in t.split(",")], default=None,
                   help="waves,capacity,persistent of the profiled launches")
    a = ap.parse_args(argv)

    if a.cmd == "trace":
        print("| kernel | grid (work-items) | calls | avg us | min us | max us |\n|---|---|---|---|---|---|")
        for (k, g), v in sorted(kernel_times(a.dir).items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
            print(f"| `{k}` | {g} | {v['calls']} | {v['avg_ns'] / 1e3:.2f} | {v['min_ns'] / 1e3:.2f} | "
                  f"{v['max_ns'] / 1e3:.2f} |")
        return 0
    if a.cmd == "counters":
        print(f"| kernel | grid (work-items) | dispatches | mean {a.counter} | min | max |\n|---|---|---|---|---|---|")
        for (k, g), v in sorted(counter_values(a.dir, a.counter).items()):
            print(f"| `{k}` | {g} | {len(v)} | {sum(v) / len(v):.6g} | {min(v):.6g} | {max(v):.6g} |")
        return 0
    fetch = counter_values(a.fetch_dir, "FETCH_SIZE")
    write = counter_values(a.write_dir, "WRITE_SIZE")
    copy_kib = a.copy_mib * 1024.0
    # the calibration copy is the largest dispatch of the copy kernel
    cf = max(max(v) for k, v in fetch.items() if a.copy_kernel in k[0])
    cw = max(max(v) for k, v in write.items() if a.copy_kernel in k[0])
    f_scale, w_scale = copy_kib / cf, copy_kib / cw
    kf, kw = _largest(fetch, a.kernel), _largest(write, a.kernel)
    mf = sum(fetch[kf]) / len(fetch[kf])
    mw = sum(write[kw]) / len(write[kw])
    rec = dict(workload=a.workload, kernel_sha=a.kernel_sha, schedule=a.schedule, kernel=kf[0], grid=kf[1],
               dispatches=len(fetch[kf]), fetch_kib_raw=mf, write_kib_raw=mw,
               copy_mib=a.copy_mib, copy_fetch_kib_raw=cf, copy_write_kib_raw=cw,
               fetch_scale=f_scale, write_scale=w_scale,
               hbm_bytes_per_launch=(mf * f_scale + mw * w_scale) * 1024.0)
    json.dump(rec, sys.stdout, indent=1)
    print()
    return 0


if __name__ == "__main__":
    sys.exit(main())
