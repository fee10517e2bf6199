"""Summarize rocprofv3 output databases (SQLite) into the short text summaries kept under
profiles/.

  python -m paper_2306_10379_amd.profsum trace  <results.db> <command-line> > profiles/<name>.md
  python -m paper_2306_10379_amd.profsum traffic <fetch.db> <write.db> <command-line> <out.json>

`trace` lists per-kernel launch counts and durations (launches shorter than 8 us, i.e.
iteration kernels that returned at once because the solve was done or the step did not
need them, are reported separately). `traffic` reads one FETCH_SIZE run and one WRITE_SIZE
run, scales each counter by what it reads for the 1 GiB device-to-device copy that the
profiling run performs (the calibration), and records bytes per dispatch for each kernel
together with a hash of the kernel sources, so that a reader can tell when the numbers
are stale.
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/gsi_kernels.hip", "csrc/gsi_device.h", "csrc/gsi_small.hip", "csrc/gsi_small_dev.h"]


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def trace(db: str, command: str) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels").fetchall()
    live = collections.defaultdict(list)
    idle = collections.Counter()
    for name, s, e in rows:
        d = (e - s) / 1e3
        if d < 8.0:
            idle[short(name)] += 1
        else:
            live[short(name)].append(d)
    out = [f"# rocprofv3 kernel trace summary", "", f"command: `{command}`", "",
           "Launches under 8 us are counted as short (a pass that returned at once). A kernel with "
           "launch sites of different sizes (the iteration's SpMM and the explicit A X product, which "
           "most iterations skip after dispatching its grid) has a mean over all its launches; the "
           "last two columns are the count and mean of its full launches (at least half its longest).",
           "",
           "| kernel | launches (>= 8 us) | total ms | avg us | min us | max us | short launches | full launches "
           "| full avg us |",
           "|---|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(live.items(), key=lambda kv: -sum(kv[1])):
        full = [x for x in v if x >= 0.5 * max(v)]
        out.append(f"| {k} | {len(v)} | {sum(v) / 1e3:.1f} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
                   f"{idle.get(k, 0)} | {len(full)} | {sum(full) / len(full):.1f} |")
    for k, c in idle.items():
        if k not in live:
            out.append(f"| {k} | 0 | 0 | - | - | - | {c} | 0 | - |")
    return "\n".join(out) + "\n"


def _counter(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value, grid_size from counters_collection order by dispatch_id").fetchall()
    per = collections.defaultdict(list)
    for name, val, grid in rows:
        per[short(name)].append(float(val))
    return per


def traffic(fetch_db: str, write_db: str, command: str, out_json: str) -> dict:
    f, w = _counter(fetch_db), _counter(write_db)
    gib_kib = 1024.0 * 1024.0
    # calibration: the largest device-to-device copy is the 1 GiB copy of the profiling run
    copy_f = max(f.get("__amd_rocclr_copyBuffer", [0.0]))
    copy_w = max(w.get("__amd_rocclr_copyBuffer", [0.0]))
    fs = gib_kib / copy_f if copy_f > 0 else None
    ws = gib_kib / copy_w if copy_w > 0 else None
    res = {"command": command, "source_hash": source_hash(), "fetch_scale": fs, "write_scale": ws,
           "calibration": "1 GiB device copy: FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB" % (copy_f, copy_w),
           "kernels": {}}
    for k in sorted(set(f) | set(w)):
        fv = [x for x in f.get(k, []) if x > 64.0]  # skip launches that returned at once
        wv = [x for x in w.get(k, []) if x > 64.0]
        if not fv and not wv:
            continue
        fk = max(fv) if fv else 0.0
        wk = max(wv) if wv else 0.0
        res["kernels"][k] = {"fetch_kib": fk, "write_kib": wk,
                             "bytes": (fk * (fs or 1.0) + wk * (ws or 1.0)) * 1024.0}
    with open(out_json, "w") as fo:
        json.dump(res, fo, indent=1)
    return res


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        sys.stdout.write(trace(sys.argv[2], sys.argv[3]))
    elif sys.argv[1] == "traffic":
        r = traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
        print(json.dumps(r, indent=1))
