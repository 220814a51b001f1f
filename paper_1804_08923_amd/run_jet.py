"""Run a jet workload on one GPU and report the Sec. IV C diagnostics as it goes.

    python -m paper_1804_08923_amd.run_jet --workload jet-ut1-240x240x1200 --steps 20000 --every 1000

One JSON line per report: step, elapsed seconds, throughput since the last
report (MLUPS), the leading edge, the jet-phase node count, the column volume,
the fragment count and the fragments' mass-median equivalent diameter
d = (6 V / pi)^(1/3) (the diameter at which the cumulative fragment volume,
in ascending order, reaches half of the total), and whether the FP64 audit
totals are finite.  Everything runs in the library; this script only
schedules the calls and formats the numbers.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time


def mass_median(volumes) -> float:
    v = sorted(int(x) for x in volumes)
    if not v:
        return float("nan")
    half, acc = 0.5 * sum(v), 0
    for x in v:
        acc += x
        if acc >= half:
            return (6.0 * x / math.pi) ** (1.0 / 3.0)
    return float("nan")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="jet-ut1-240x240x1200")
    ap.add_argument("--steps", type=int, default=None, help="default: the workload's step count")
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--storage", default="fp32")
    args = ap.parse_args(argv)

    import torch

    from .lbm import LBM
    from .workloads import WORKLOADS
    prob = WORKLOADS[args.workload]().replace(storage=args.storage)
    steps = prob.steps if args.steps is None else args.steps
    sim = LBM(prob)
    print(json.dumps({"workload": prob.name, "nodes": prob.n_nodes, "storage": prob.storage, "steps": steps,
                      "meta": prob.meta}), flush=True)
    t_start = time.perf_counter()
    done = 0
    while done < steps:
        k = min(args.every, steps - done)
        t0 = time.perf_counter()
        sim.step(k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        done += k
        stats, vol = sim.jet_diagnostics()
        try:
            a = sim.macroscopic(audit=True)["audit"]
            finite = all(math.isfinite(x) for x in a)
        except RuntimeError:
            finite = False
        rec = dict(step=done, elapsed_s=round(time.perf_counter() - t_start, 2),
                   mlups=round(prob.n_nodes * k / dt / 1e6, 1), **stats,
                   mass_median_d=round(mass_median(vol), 3), finite=finite)
        print(json.dumps(rec), flush=True)
        if not finite:
            break
    sim.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
