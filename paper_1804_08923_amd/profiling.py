"""Summaries of rocprofv3 result databases (kernel traces and counter runs).

    python -m paper_1804_08923_amd.profiling trace <results.db>
    python -m paper_1804_08923_amd.profiling pmc <results.db>
    python -m paper_1804_08923_amd.profiling traffic <fetch.db> <write.db> <key> <kernel> <out.json>

``trace`` prints per-kernel call counts and durations; ``pmc`` prints the
per-dispatch average and maximum of every collected counter per kernel.
``traffic`` turns a FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch) of a
command that also made a 1 GiB device copy into HBM bytes per launch of
<kernel>: each counter is scaled by 1 GiB over what it read for the copy's
largest dispatch, and the result is stored under <key> (workload/storage) in
<out.json> together with a hash of the kernel sources it was measured on.
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import re
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = ("lbm_kernels.h", "lbm_lattice.h")
Q19_SOURCES = ("lbm_q19.h", "lbm_lattice.h")  # the D3Q19 kernels (k19_*)
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30


def sources_of(kernel: str):
    """The source files a kernel is built from (D3Q19 kernels are k19_*)."""
    return Q19_SOURCES if "k19_" in kernel else KERNEL_SOURCES


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    """Hash of the kernel sources; counter figures are valid only for it."""
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    return re.sub(r"\(.*", "", name)


def trace_summary(db: str) -> str:
    c = sqlite3.connect(db)
    rows = c.execute(
        "select name, count(*), avg(duration), min(duration), max(duration), sum(duration), max(vgpr_count) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    tot = sum(r[5] for r in rows) or 1
    out = [f"{'kernel':64s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'total_ms':>9s} {'%':>5s}"]
    for r in rows:
        out.append(f"{_short(r[0])[:64]:64s} {r[1]:6d} {r[2] / 1e3:9.2f} {r[3] / 1e3:9.2f} {r[4] / 1e3:9.2f} "
                   f"{r[5] / 1e6:9.3f} {100 * r[5] / tot:5.1f}")
    return "\n".join(out)


def pmc_summary(db: str) -> str:
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, cn, v in rows:
        agg[_short(name)][cn].append(v)
    out = []
    for name, d in agg.items():
        parts = " ".join(f"{k}(avg)={sum(v) / len(v):.6g} {k}(max)={max(v):.6g}" for k, v in sorted(d.items()))
        n = max(len(v) for v in d.values())
        out.append(f"{name[:64]:64s} dispatches={n:4d} {parts}")
    return "\n".join(out)


def _counter_values(db: str, counter: str):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, value from counters_collection where counter_name = ?",
                     (counter,)).fetchall()
    out = collections.defaultdict(list)
    for name, v in rows:
        out[_short(name)].append(v)
    return out


def traffic(fetch_db: str, write_db: str, kernel: str) -> dict:
    """Calibrated HBM bytes per launch of `kernel` (counters are KiB per dispatch)."""
    res = {}
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        vals = _counter_values(db, counter)
        copy = [v for k, v in vals.items() if COPY_KERNEL in k]
        if not copy:
            raise SystemExit(f"{db}: no {COPY_KERNEL} dispatch to calibrate against")
        scale = COPY_BYTES / (max(max(v) for v in copy) * 1024.0)
        kv = [v for k, v in vals.items() if k.endswith(kernel) or k == kernel]
        if len(kv) != 1:
            raise SystemExit(f"{db}: kernel {kernel!r} matched {len(kv)} names")
        per = sum(kv[0]) / len(kv[0]) * 1024.0 * scale
        res[counter] = {"kib_per_dispatch": sum(kv[0]) / len(kv[0]), "scale": round(scale, 4),
                        "bytes_per_launch": per, "dispatches": len(kv[0])}
    res["bytes_per_launch"] = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    return res


def main(argv):
    if len(argv) == 3 and argv[1] in ("trace", "pmc"):
        print(trace_summary(argv[2]) if argv[1] == "trace" else pmc_summary(argv[2]))
        return 0
    if len(argv) == 7 and argv[1] == "traffic":
        _, _, fdb, wdb, key, kernel, out = argv
        t = traffic(fdb, wdb, kernel)
        t["kernel"] = kernel
        t["kernel_hash"] = kernel_source_hash(sources_of(kernel))
        allt = {}
        if os.path.exists(out):
            with open(out) as fh:
                allt = json.load(fh)
        allt[key] = t
        with open(out, "w") as fh:
            json.dump(allt, fh, indent=1)
        print(json.dumps(t, indent=1))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv))
