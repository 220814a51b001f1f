#!/usr/bin/env python3
"""Throughput of the colour-gradient D3Q27 central-moment LBM step on one MI355X.

Workload: the 128x128x512 liquid-liquid jet (D = 16, u = 0.04, gamma = 2,
eta = 1, Re = 1e3, We = 50, Fr = 10, 1 % seeded radial inlet noise), synthetic,
populations resident in HBM.  A step is one full time step of the method
(density pass + fused collide-perturb-recolour-stream kernel with the jet
boundaries).  Prints ONE JSON line on stdout; progress goes to stderr.

value = MLUPS of the FP32-storage step (nodes x steps / s / 1e6).
roofline = the fused kernel's algorithmic bytes per launch / its average
duration (HIP events recorded by the library around every launch in the timed
region) against the 8 TB/s HBM peak.
cpu_baseline = the FP64 oracle on the host cores, on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Reference model of a step: both colour sets (2 x 27 populations) read once and
# written once per node update.
STEP_BYTES = {"fp32": 432, "bf16": 216, "fp16": 216, "bf16eq": 216, "fp16eq": 216}
# Bytes this implementation must move per node update.  Fused kernel: 27
# colour-blind deviations read, (phi, rho - rho_b0) and rho_r/rho read, 27
# deviations and the float4 (rho_r/rho, V) of the recolouring written.  Density
# pass: 27 deviations and the source-node float4 read, 3 floats written.
# Equilibrium-referenced 16-bit forms: the rest population in two 16-bit
# planes and a 16-byte reference record per node, read and written.
FUSED_BYTES = {"fp32": 27 * 4 + 12 + 27 * 4 + 16, "bf16": 27 * 2 + 12 + 27 * 2 + 16,
               "fp16": 27 * 2 + 12 + 27 * 2 + 16, "bf16eq": 28 * 2 + 16 + 12 + 28 * 2 + 16 + 16,
               "fp16eq": 28 * 2 + 16 + 12 + 28 * 2 + 16 + 16}
DENSITY_BYTES = {"fp32": 27 * 4 + 16 + 12, "bf16": 27 * 2 + 16 + 12, "fp16": 27 * 2 + 16 + 12,
                 "bf16eq": 28 * 2 + 16 + 16 + 12, "fp16eq": 28 * 2 + 16 + 16 + 12}
PAPER_CONTEXT = {"mlups": [1.2, 12.0], "hardware": "unspecified cluster (COMA / Earth Simulator named)",
                 "workload": "240x240x1200 UT jet, 20000 iterations in ~32 h"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(storage):
    """HBM bytes per fused-kernel launch from committed rocprofv3 counter runs,
    used only while the kernel source is unchanged since they were taken."""
    from paper_1804_08923_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    ent = t.get(storage)
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def run_leg(prob, steps, warmup, diagnostics=False):
    import torch

    from paper_1804_08923_amd.lbm import LBM
    sim = LBM(prob, device="cuda:0")
    N = prob.n_nodes
    sim.profile(True)
    done = 0
    while done < warmup:
        k = min(50, warmup - done)
        sim.step(k)
        done += k
    torch.cuda.synchronize()
    sim.profile_read()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    done = 0
    while done < steps:
        k = min(100, steps - done)
        sim.step(k)
        done += k
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    kms, launches = sim.profile_read()
    bnd = kms[2] / launches[2]
    sim.profile(False)
    m = sim.macroscopic(audit=True)
    audit = m["audit"]
    umax = float(m["u"].norm(dim=1).max().item())
    finite = bool(torch.isfinite(m["u"]).all().item())
    del m
    diag = None
    if diagnostics:
        # jet diagnostics (leading edge, fragments) of the final state, timed
        # on the host clock around the synchronising call
        sim.jet_diagnostics()
        reps = 5
        t1 = time.perf_counter()
        for _ in range(reps):
            stats, vol = sim.jet_diagnostics()
        diag = dict(ms=round((time.perf_counter() - t1) / reps * 1e3, 3), step=warmup + steps, **stats)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    st = prob.storage
    mlups = N * steps / (ms * 1e-3) / 1e6
    avg_fused = kms[1] / launches[1]
    avg_dens = kms[0] / launches[0]
    achieved = FUSED_BYTES[st] * N / (avg_fused * 1e-3) / 1e9
    return dict(mlups=mlups, ms_per_step=ms / steps, wall_s=wall, umax=umax, finite=finite, audit=audit, diag=diag,
                fused_ms=avg_fused, density_ms=avg_dens, boundary_ms=bnd, fused_gbs=achieved,
                step_roofline_frac=mlups / (HBM_PEAK_GBS * 1e9 / STEP_BYTES[st] / 1e6))


def adjoint_leg(prob, nadj=10):
    """Cost of one adjoint step (lbm_adjoint_step) at a developed state, and of
    recomputing one forward state from a checkpoint (set_state + step +
    get_state), both timed with events on the library's stream."""
    import torch

    from paper_1804_08923_amd.lbm import LBM
    sim = LBM(prob, device="cuda:0", adjoint=True)
    sim.step(50)
    st = sim.get_state()
    t = sim.time
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5)
    lam = [torch.randn(st.shape, generator=g, device="cuda:0", dtype=torch.float32), torch.empty_like(st)]
    dA = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    du = torch.zeros(prob.nx * prob.ny, dtype=torch.float32, device="cuda:0")
    for i in range(2):
        sim.adjoint_step(st, t, lam[i % 2], lam[1 - i % 2], dA, du)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(nadj):
        sim.adjoint_step(st, t, lam[i % 2], lam[1 - i % 2], dA, du)
    e1.record()
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / nadj
    finite = bool(torch.isfinite(lam[nadj % 2]).all().item()) and bool(torch.isfinite(dA).all().item())
    e0.record()
    for _ in range(nadj):
        sim.set_state(st, t)
        sim.step(1)
        sim.get_state()
    e1.record()
    torch.cuda.synchronize()
    rec_ms = e0.elapsed_time(e1) / nadj
    sim.close()
    del sim, st, lam
    torch.cuda.empty_cache()
    return dict(adjoint_ms=adj_ms, recompute_ms=rec_ms, finite=finite)


def cpu_baseline(prob, nz_sample=64, steps=32):
    """The FP64 oracle on a slab of the same jet (full cross-section, nz_sample planes)."""
    from oracle import Oracle
    from oracle import make_params as or_params
    import numpy as np
    sp = prob.replace(nz=nz_sample)
    orc = Oracle("f64")
    p = or_params(sp)
    N = sp.n_nodes
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, sp.rho_b0))
    t0 = time.perf_counter()
    orc.step(p, sp.A, fr, fb, h, 0, steps)
    dt = time.perf_counter() - t0
    return {"value": N * steps / dt / 1e6, "unit": "MLUPS", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{sp.nx}x{sp.ny}x{sp.nz} slab of the jet (same inlet, walls, outlet), {steps} steps "
                      f"from the initial state, FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="jet-128x128x512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the BF16/FP16 storage legs")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-step timing")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (calibrates hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the step is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1804_08923_amd.workloads import WORKLOADS
    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    prob = WORKLOADS[args.workload]().replace(storage="fp32")
    log(f"bench: {prob.name} ({prob.n_nodes} nodes) fp32, warmup {args.warmup}, steps {args.steps}")

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
        log("bench: copy probe (1 GiB read + 1 GiB write) done")

    main_leg = run_leg(prob, args.steps, args.warmup, diagnostics=True)
    log(f"bench: fp32 {main_leg['mlups']:.0f} MLUPS, fused kernel {main_leg['fused_ms']:.3f} ms "
        f"({main_leg['fused_gbs']:.0f} GB/s), density {main_leg['density_ms']:.3f} ms, "
        f"boundary {main_leg['boundary_ms']:.3f} ms")
    log(f"bench: jet diagnostics {main_leg['diag']}")
    legs = {}
    if not args.no_legs:
        for st in ("bf16", "fp16", "bf16eq", "fp16eq"):
            r = run_leg(prob.replace(storage=st), args.steps, args.warmup)
            legs[st] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                        "x_fp32": round(r["mlups"] / main_leg["mlups"], 3),
                        "step_roofline_frac": round(r["step_roofline_frac"], 4),
                        "fused_kernel_ms": round(r["fused_ms"], 4), "fused_kernel_gbs": round(r["fused_gbs"], 1),
                        "finite": r["finite"]}
            log(f"bench: {st} {r['mlups']:.0f} MLUPS ({r['mlups'] / main_leg['mlups']:.2f}x fp32)")
    adj = None
    if not args.no_adjoint:
        a = adjoint_leg(prob)
        adj = {"adjoint_step_ms": round(a["adjoint_ms"], 4), "forward_step_ms": round(main_leg["ms_per_step"], 4),
               "ratio": round(a["adjoint_ms"] / main_leg["ms_per_step"], 3),
               "recompute_step_ms": round(a["recompute_ms"], 4), "finite": a["finite"],
               "note": "adjoint step alone; recompute = set_state + step + get_state of one checkpointed state"}
        log(f"bench: adjoint step {a['adjoint_ms']:.3f} ms = {adj['ratio']:.2f}x forward, "
            f"recompute {a['recompute_ms']:.3f} ms")
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        cpu = cpu_baseline(prob)
        log(f"bench: oracle {cpu['value']:.3f} MLUPS on {cpu['cores']} threads")

    traffic = measured_traffic("fp32")
    line = {
        "metric": "MLUPS and % HBM roofline: FP32 vs BF16-storage fused step; adjoint/forward cost",
        "value": round(main_leg["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_leg["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": prob.name, "nodes": prob.n_nodes, "lattice": "D3Q27 two-colour",
                   "storage": "fp32", "bc": prob.bc, "gamma": prob.gamma, "Re": prob.meta.get("Re"),
                   "We": prob.meta.get("We"), "Fr": prob.meta.get("Fr")},
        "roofline": {"bound": "hbm", "achieved": round(main_leg["fused_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(main_leg["fused_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_collide<jet, fp32> (fused collide-recolour-stream)",
                     "bytes_per_node": FUSED_BYTES["fp32"], "avg_launch_ms": round(main_leg["fused_ms"], 4)},
        "step_roofline_frac": round(main_leg["step_roofline_frac"], 4),
        "step_bytes_per_node": STEP_BYTES["fp32"],
        "impl_bytes_per_node": FUSED_BYTES["fp32"] + DENSITY_BYTES["fp32"],
        "density_kernel_ms": round(main_leg["density_ms"], 4),
        "boundary_kernels_ms": round(main_leg["boundary_ms"], 4),
        "jet_diagnostics": main_leg["diag"],
        "cpu_baseline": cpu,
        "storage_legs": legs,
        "adjoint_forward_ratio": adj["ratio"] if adj else None,
        "adjoint": adj,
        "finite": main_leg["finite"],
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
