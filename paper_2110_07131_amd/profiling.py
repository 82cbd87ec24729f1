"""HBM traffic of a kernel from rocprofv3 counter runs.

Two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of the same
benchmark command (which also performs plain device copies of a known size,
`bench.py --calib-copy-mb N`) give per-dispatch KiB for every kernel.  The
copy dispatches calibrate each counter (bytes the copy must move / counter
reading); the kernel's average reading times that factor is its HBM traffic
per launch.  The result is stamped with a hash of the kernel's sources, so
a later change to that kernel invalidates it (the benchmark then reports
traffic as null).

    python -m paper_2110_07131_amd.profiling --fetch DIR1 --write DIR2 \\
        --kernel k_bfilter --copy-mb 1024 --key plain/fp32/exact --out profiles/traffic.json

A phase of several kernels (the bounded table's scan: the block pass, the
group passes and k_bdecide, launched once per query chunk) is measured with
--match (all its dispatches) and --per (the dispatch that counts phases):
the traffic per phase is the sum over the matching dispatches divided by the
number of phases.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


# The sources a kernel is compiled from (its file and the headers it includes).
KERNEL_SOURCES = {
    "k_bfilter": ["batch_kernels.hip", "batch_device.h", "rk_batch.h", "rk_common.h", "host_rules.h",
                  "rkmips.h"],
    "k_bscan": ["scan_kernels.hip", "batch_device.h", "rk_batch.h", "rk_common.h", "host_rules.h",
                "rkmips.h"],
    "k_filter": ["query_kernels.hip", "batch_device.h", "rk_batch.h", "rk_kernels.h", "rk_common.h",
                 "host_rules.h", "rkmips.h"],
}


def strip_comments(src: str) -> str:
    """C/C++ source without its comments and blank-line runs: a change to a
    comment leaves the compiled kernel, and so its hash, as it was."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":  # string or character literal, copied whole
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    lines = [ln.rstrip() for ln in "".join(out).splitlines()]
    return "\n".join(ln for ln in lines if ln)


def source_hash(kernel: str) -> str:
    """sha256 over the sources of a kernel (csrc/ and include/), comments
    left out."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        path = os.path.join(CSRC, f)
        if not os.path.exists(path):
            path = os.path.join(os.path.dirname(HERE), "include", f)
        h.update(f.encode())
        with open(path, encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def _col(row: dict, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(names)


def read_counter(run_dir: str, counter: str) -> list[tuple[str, float]]:
    """(kernel name, value) per dispatch for one counter of a rocprofv3 run."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    per = {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if _col(row, "Counter_Name") != counter:
                    continue
                key = (f, _col(row, "Dispatch_Id", "Correlation_Id"))
                name = _col(row, "Kernel_Name")
                v = float(_col(row, "Counter_Value"))
                if key in per:
                    per[key] = (name, per[key][1] + v)  # summed over dimensions
                else:
                    per[key] = (name, v)
    return list(per.values())


def kernel_average(rows, pattern: str, per: str | None = None) -> tuple[float, int]:
    """Average reading per dispatch of `pattern`; with `per`, the sum over the
    dispatches of `pattern` per dispatch of `per` (a phase of several kernels)."""
    vals = [v for n, v in rows if re.search(pattern, n)]
    if not vals:
        raise ValueError(f"no dispatch of {pattern}")
    if per is None:
        return sum(vals) / len(vals), len(vals)
    count = sum(1 for n, _ in rows if re.search(per, n))
    if count == 0:
        raise ValueError(f"no dispatch of {per}")
    return sum(vals) / count, count


def copy_factor(rows, copy_bytes: int) -> tuple[float, float]:
    """Factor = expected KiB / measured KiB over the calibration copies: the
    copy-kernel dispatches whose reading is at least a quarter of the expected size."""
    want = copy_bytes / 1024.0
    vals = [v for n, v in rows if "copyBuffer" in n and v >= 0.25 * want]
    if not vals:
        raise ValueError("no calibration copy found")
    meas = sum(vals) / len(vals)
    return want / meas, meas


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True, help="label (and default dispatch pattern)")
    ap.add_argument("--match", default=None, help="regex of the dispatches summed (default: --kernel)")
    ap.add_argument("--per", default=None, help="regex of the dispatch counting phases")
    ap.add_argument("--copy-mb", type=int, required=True)
    ap.add_argument("--key", required=True, help="workload/precision/table, e.g. plain/fp32/exact")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    nbytes = a.copy_mb << 20
    fr, wr = read_counter(a.fetch, "FETCH_SIZE"), read_counter(a.write, "WRITE_SIZE")
    ff, fmeas = copy_factor(fr, nbytes)
    wf, wmeas = copy_factor(wr, nbytes)
    pat = a.match or a.kernel
    fk, nf = kernel_average(fr, pat, a.per)
    wk, nw = kernel_average(wr, pat, a.per)
    entry = {
        "kernel": a.kernel, "key": a.key, "source_hash": source_hash(a.kernel),
        "match": pat, "per": a.per or pat,
        "fetch_kib_per_launch": fk, "write_kib_per_launch": wk, "launches": [nf, nw],
        "copy_mb": a.copy_mb, "copy_fetch_kib": fmeas, "copy_write_kib": wmeas,
        "fetch_factor": ff, "write_factor": wf,
        "traffic_bytes_per_launch": (fk * ff + wk * wf) * 1024.0,
        "command": a.command,
    }
    db = {}
    if os.path.exists(a.out):
        with open(a.out) as fh:
            db = json.load(fh)
    db[f"{a.kernel}:{a.key}"] = entry
    with open(a.out, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    print(json.dumps(entry))


if __name__ == "__main__":
    main()
