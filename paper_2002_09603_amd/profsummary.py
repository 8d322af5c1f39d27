"""Summaries of rocprofv3 CSV output for the kernels of this library.

rocprofv3's own ``--stats`` table averages a kernel over every launch of the
same instantiation, but the V-cycle kernels run once per AMG level with very
different sizes.  These summaries group dispatches by (kernel, grid size), so
the finest-level launches can be compared with the per-launch figures that
``bench.py`` measures with HIP events.

    python -m paper_2002_09603_amd.profsummary trace DIR [--top 25]
    python -m paper_2002_09603_amd.profsummary pmc DIR --copy-regex neg_kernel \
        --copy-bytes 1073741824 [--match k_cheb_step]

``counters`` tabulates any counters of a ``--pmc`` run per kernel and grid.
``trace`` reads ``*kernel_trace.csv`` (from ``--kernel-trace``), ``pmc`` reads
``*counter_collection.csv`` (from ``--pmc FETCH_SIZE`` or ``--pmc
WRITE_SIZE``).  For ``pmc`` the counter of the largest dispatch matching
``--copy-regex`` (a plain elementwise copy that reads and writes
``--copy-bytes`` each) calibrates KiB-per-dispatch readings to bytes; the
scale factor is printed with the result.  ``sources`` prints the SHA-256 of
the HIP sources, which ties a counter reading to the kernels it was taken on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def sources_sha256() -> str:
    """SHA-256 over the HIP sources and headers of the library, in name order."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    s = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("pm::", "")
    depth, out = 0, []
    for ch in s:                      # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _files(d, suffix):
    fs = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not fs:
        raise SystemExit(f"no *{suffix} under {d}")
    return fs


def trace(d, top, match=None):
    agg = defaultdict(lambda: [0, 0])
    n_all, t_all = 0, 0
    for fn in _files(d, "kernel_trace.csv"):
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                key = (short_name(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"])
                       * int(r["Grid_Size_Z"]))
                agg[key][0] += 1
                agg[key][1] += dt
                n_all += 1
                t_all += dt
    rows = sorted(agg.items(), key=lambda kv: -kv[1][1])
    if match:
        rows = [kv for kv in rows if re.search(match, kv[0][0])]
    print(f"{n_all} dispatches, {t_all / 1e6:.2f} ms of kernel time\n")
    print("| kernel | grid (work-items) | launches | avg us | total ms | share |")
    print("|---|---:|---:|---:|---:|---:|")
    for (name, grid), (n, t) in rows[:top]:
        print(f"| `{name}` | {grid} | {n} | {t / n / 1e3:.1f} | {t / 1e6:.2f} | {100 * t / t_all:.1f}% |")


def pmc(d, copy_regex, copy_bytes, match=None):
    per = defaultdict(lambda: defaultdict(float))     # (name, grid) -> dispatch -> value
    counter = None
    for fn in _files(d, "counter_collection.csv"):
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                counter = r["Counter_Name"]
                key = (short_name(r["Kernel_Name"]), int(r["Grid_Size"]))
                per[key][(fn, r["Dispatch_Id"])] += float(r["Counter_Value"])
    copies = [(k, v) for k, v in per.items() if re.search(copy_regex, k[0])]
    if not copies:
        raise SystemExit(f"no dispatch matching {copy_regex!r}")
    (ck, cv) = max(copies, key=lambda kv: kv[0][1])
    c_kib = sum(cv.values()) / len(cv)
    scale = (copy_bytes / 1024.0) / c_kib
    print(f"counter {counter}; calibration: `{ck[0]}` grid {ck[1]} moves {copy_bytes} B each way, "
          f"reads {c_kib:.1f} KiB per dispatch -> scale {scale:.4f} (bytes = KiB x 1024 x scale)\n")
    print("| kernel | grid (work-items) | dispatches | avg KiB | calibrated bytes per dispatch |")
    print("|---|---:|---:|---:|---:|")
    rows = sorted(per.items(), key=lambda kv: -sum(kv[1].values()))
    if match:
        rows = [kv for kv in rows if re.search(match, kv[0][0])]
    for (name, grid), v in rows:
        a = sum(v.values()) / len(v)
        print(f"| `{name}` | {grid} | {len(v)} | {a:.1f} | {a * 1024 * scale:.0f} |")
    print(f"\nsources_sha256 {sources_sha256()}")


def counters(d, match=None):
    """Per (kernel, grid): the average of every collected counter per
    dispatch, and the ratios used for the stencil kernels: VALU instructions
    and issue cycles per wave, the share of a wave's lifetime spent issuing
    VALU instructions, and the mean number of resident waves per busy CU."""
    per = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))  # key -> counter -> dispatch -> value
    for fn in _files(d, "counter_collection.csv"):
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                key = (short_name(r["Kernel_Name"]), int(r["Grid_Size"]))
                per[key][r["Counter_Name"]][(fn, r["Dispatch_Id"])] += float(r["Counter_Value"])
    rows = sorted(per.items(), key=lambda kv: kv[0])
    if match:
        rows = [kv for kv in rows if re.search(match, kv[0][0])]
    names = sorted({c for _, cs in rows for c in cs})
    print("| kernel | grid | " + " | ".join(names) + " |")
    print("|---|---:|" + "---:|" * len(names))
    avg = {}
    for key, cs in rows:
        a = {c: sum(v.values()) / len(v) for c, v in cs.items()}
        avg[key] = a
        print(f"| `{key[0]}` | {key[1]} | " + " | ".join(f"{a.get(c, float('nan')):.4g}" for c in names) + " |")
    print()
    for key, a in avg.items():
        w = a.get("SQ_WAVES")
        out = []
        if w:
            if "SQ_INSTS_VALU" in a:
                out.append(f"VALU instructions per wave {a['SQ_INSTS_VALU'] / w:.0f}")
            if "SQ_ACTIVE_INST_VALU" in a and "SQ_WAVE_CYCLES" in a and a["SQ_WAVE_CYCLES"] > 0:
                out.append(f"VALU issue share of wave lifetime {a['SQ_ACTIVE_INST_VALU'] / a['SQ_WAVE_CYCLES']:.3f}")
            if "SQ_WAVE_CYCLES" in a:
                out.append(f"wave lifetime {a['SQ_WAVE_CYCLES'] / w:.0f} cycles")
        if "SQ_LEVEL_WAVES" in a and a.get("SQ_BUSY_CU_CYCLES"):
            out.append(f"resident waves per busy CU {a['SQ_LEVEL_WAVES'] / a['SQ_BUSY_CU_CYCLES']:.1f}")
        if out:
            print(f"* `{key[0]}` grid {key[1]}: " + "; ".join(out))
    print(f"\nsources_sha256 {sources_sha256()}")


def main(argv=None):
    ap = argparse.ArgumentParser(description="group rocprofv3 CSV output by kernel and grid size")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--top", type=int, default=25)
    t.add_argument("--match")
    p = sub.add_parser("pmc")
    p.add_argument("dir")
    p.add_argument("--copy-regex", required=True)
    p.add_argument("--copy-bytes", type=int, required=True)
    p.add_argument("--match")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--match")
    sub.add_parser("sources")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        trace(a.dir, a.top, a.match)
    elif a.cmd == "pmc":
        pmc(a.dir, a.copy_regex, a.copy_bytes, a.match)
    elif a.cmd == "counters":
        counters(a.dir, a.match)
    else:
        print(sources_sha256())


if __name__ == "__main__":
    sys.exit(main())
