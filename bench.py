#!/usr/bin/env python3
"""Throughput of the colour-gradient D3Q27 central-moment LBM step on one MI355X.

Workload: the 256x256x1024 high-Re liquid-liquid jet (67.1 M nodes; D = 24,
u = 0.05, gamma = 2, eta = 0.01, Re = 1e6, We = 1e3, Fr = 10, 1 % seeded radial
inlet noise), synthetic, populations resident in HBM.  A step is one full time
step of the method (density pass + fused collide-perturb-recolour-stream kernel
with the jet boundaries).  The jet is first developed for `--warmup` steps
(default 2000, outside the timed region); then `--steps` steps (default 2000)
are timed with HIP events on the library's stream, with no instrumentation
inside the timed region.  A separate profiled pass right after it (the
library's per-kernel events) gives the per-kernel durations.  Prints ONE JSON
line on stdout; progress goes to stderr.

value = MLUPS of the FP32-storage step (nodes x steps / s / 1e6).
roofline = the fused kernel's algorithmic bytes per launch / its average
duration in the profiled pass, against the 8 TB/s HBM peak.
cpu_baseline = the FP64 oracle on the host cores, on a bounded slab sample of
the same jet, on all threads and on one.
lattices = the reduced D3Q19 lattice (Sec. II's suggested cost cut) against
D3Q27: on the same jet (developed and timed like the headline leg) and on a
periodic droplet box of the same size, each with its own kernel timings and
roofline.
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
PROFILE_STEPS = 50
# D3Q19 (lattice = 19), bytes per node update.  Collision kernel: 19 pulled
# deviations read, the float4 (phi, rho - rho_b0, rho_r, rho_b) read, 19
# deviations and the float4 recolouring record written.  Density pass: 19
# deviations and the source-node record read, the float4 written.  Reference
# model: both colour sets (2 x 19 populations) read once and written once.
Q19_FUSED_BYTES = 19 * 4 + 16 + 19 * 4 + 16
Q19_DENSITY_BYTES = 19 * 4 + 16 + 16
Q19_STEP_BYTES = 2 * 2 * 19 * 4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(storage, workload, kernel="k_collide"):
    """HBM bytes per fused-kernel launch from committed rocprofv3 counter runs,
    used only while the kernel source is unchanged since they were taken and
    only for the workload they were taken on."""
    from paper_1804_08923_amd.profiling import kernel_source_hash, sources_of
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    ent = t.get(f"{workload}/{storage}")
    if not ent or ent.get("kernel_hash") != kernel_source_hash(sources_of(kernel)):
        return None
    return ent.get("bytes_per_launch")


def _advance(sim, n, chunk=100):
    done = 0
    while done < n:
        k = min(chunk, n - done)
        sim.step(k)
        done += k


def run_leg(prob, steps, warmup, diagnostics=False, keep=False):
    """Develop the jet for `warmup` steps, time `steps` steps (no
    instrumentation), then profile PROFILE_STEPS more steps per kernel."""
    import torch

    from paper_1804_08923_amd.lbm import LBM
    sim = LBM(prob, device="cuda:0")
    N = prob.n_nodes
    t_dev = time.perf_counter()
    _advance(sim, warmup)
    torch.cuda.synchronize()
    dev_s = time.perf_counter() - t_dev
    stream = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    _advance(sim, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # profiled pass: the library records events around its kernel groups
    sim.profile(True)
    _advance(sim, PROFILE_STEPS)
    kms, launches = sim.profile_read()
    sim.profile(False)
    m = sim.macroscopic(audit=True)
    audit = m["audit"]
    umax = float(m["u"].norm(dim=1).max().item())
    finite = bool(torch.isfinite(m["u"]).all().item())
    del m
    diag = None
    if diagnostics and prob.bc == "jet":
        sim.jet_diagnostics()
        reps = 3
        t1 = time.perf_counter()
        for _ in range(reps):
            stats, vol = sim.jet_diagnostics()
        diag = dict(ms=round((time.perf_counter() - t1) / reps * 1e3, 3), step=sim.time, **stats)
    if not keep:
        sim.close()
        del sim
        sim = None
        torch.cuda.empty_cache()
    st = prob.storage
    mlups = N * steps / (ms * 1e-3) / 1e6
    avg_fused = kms[1] / launches[1]
    avg_dens = kms[0] / launches[0]
    achieved = FUSED_BYTES[st] * N / (avg_fused * 1e-3) / 1e9
    return dict(mlups=mlups, ms_per_step=ms / steps, wall_s=wall, develop_s=dev_s, umax=umax, finite=finite,
                audit=audit, diag=diag, fused_ms=avg_fused, density_ms=avg_dens, boundary_ms=kms[2] / launches[2],
                profiled_step_ms=sum(kms) / launches[1], fused_gbs=achieved,
                step_roofline_frac=mlups / (HBM_PEAK_GBS * 1e9 / STEP_BYTES[st] / 1e6), sim=sim)


def adjoint_leg(prob, fwd_ms, nadj=10):
    """Cost of one reverse step at a developed state: the adjoint step
    (lbm_adjoint_step) and the recompute of the forward state it needs from the
    previous one (a forward step into a caller-held snapshot), both timed with
    events on the library's stream; their sum with the forward step is the
    full cost of one step of a checkpointed gradient."""
    import torch

    from paper_1804_08923_amd.lbm import LBM
    sim = LBM(prob, device="cuda:0", adjoint=True)
    _advance(sim, 50)
    snap = [sim.new_snapshot(), sim.new_snapshot()]
    sim.save_snapshot(snap[0])
    t = sim.time
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5)
    lam = [torch.randn((2 * 27, prob.n_nodes), generator=g, device="cuda:0", dtype=torch.float32), None]
    lam[1] = torch.empty_like(lam[0])
    dA = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    du = torch.zeros(prob.nx * prob.ny, dtype=torch.float32, device="cuda:0")
    stream = sim.stream
    for i in range(2):
        sim.adjoint_step_snapshot(snap[0], t, lam[i % 2], lam[1 - i % 2], dA, du)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(nadj):
        sim.adjoint_step_snapshot(snap[0], t, lam[i % 2], lam[1 - i % 2], dA, du)
    e1.record(stream)
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / nadj
    finite = bool(torch.isfinite(lam[nadj % 2]).all().item()) and bool(torch.isfinite(dA).all().item())
    # recompute: restore the checkpointed state once, then step into snapshots
    sim.load_snapshot(snap[0], t)
    sim.step_to_snapshot(snap[1])
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(nadj):
        sim.step_to_snapshot(snap[i % 2])
    e1.record(stream)
    torch.cuda.synchronize()
    rec_ms = e0.elapsed_time(e1) / nadj
    e0.record(stream)
    for _ in range(nadj):
        sim.load_snapshot(snap[0], t)
    e1.record(stream)
    torch.cuda.synchronize()
    load_ms = e0.elapsed_time(e1) / nadj
    sim.close()
    del sim, snap, lam
    torch.cuda.empty_cache()
    return dict(adjoint_ms=adj_ms, recompute_ms=rec_ms, load_ms=load_ms, finite=finite,
                gradient_step_ms=fwd_ms + rec_ms + adj_ms)


def lattice_legs(jet, steps, warmup):
    """D3Q19 against D3Q27 at equal lattice size and boundaries: a periodic box
    of the jet's size holding one droplet (R = nx/4, W = 4) at the jet's
    density ratio, with the Table I viscosity (tau = 1) and A = 1e-3 (a static
    droplet at the jet's tau ~ 0.5 is not a stable test case; the work per node
    does not depend on them); alpha_b gives the blue phase c_s^2 = 1/3 on each
    lattice.  Returns per-lattice MLUPS and kernel timings."""
    from paper_1804_08923_amd.workloads import Problem
    base = Problem(name=f"droplet-{jet.nx}x{jet.ny}x{jet.nz}", nx=jet.nx, ny=jet.ny, nz=jet.nz, bc="periodic",
                   rho_r0=jet.rho_r0, rho_b0=jet.rho_b0, nu_r=1.0 / 6.0, nu_b=1.0 / 6.0, A=1e-3, beta=jet.beta,
                   drop_R=jet.nx / 4.0, drop_W=4.0, init="droplet", storage="fp32")
    out = {}
    for q in (27, 19):
        prob = base.replace(lattice=q, alpha_b=1.0 / 3.0 if q == 19 else 8.0 / 27.0)
        r = run_leg(prob, steps, warmup)
        fb = Q19_FUSED_BYTES if q == 19 else FUSED_BYTES["fp32"]
        db = Q19_DENSITY_BYTES if q == 19 else DENSITY_BYTES["fp32"]
        sb = Q19_STEP_BYTES if q == 19 else STEP_BYTES["fp32"]
        N = prob.n_nodes
        out[f"d3q{q}"] = {
            "mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
            "fused_kernel_ms": round(r["fused_ms"], 4), "density_kernel_ms": round(r["density_ms"], 4),
            "fused_bytes_per_node": fb, "density_bytes_per_node": db,
            "fused_kernel_gbs": round(fb * N / (r["fused_ms"] * 1e-3) / 1e9, 1),
            "density_kernel_gbs": round(db * N / (r["density_ms"] * 1e-3) / 1e9, 1),
            "step_bytes_per_node": sb,
            "step_roofline_frac": round(r["mlups"] / (HBM_PEAK_GBS * 1e9 / sb / 1e6), 4),
            "impl_roofline_frac": round(r["mlups"] / (HBM_PEAK_GBS * 1e9 / (fb + db) / 1e6), 4),
            "finite": r["finite"]}
        if q == 19:
            out["d3q19"]["fused_traffic"] = measured_traffic("d3q19", base.name, kernel="k19_collide")
        log(f"bench: {prob.name} D3Q{q}: {r['mlups']:.0f} MLUPS, fused {r['fused_ms']:.3f} ms, density "
            f"{r['density_ms']:.3f} ms")
    out["workload"] = base.name
    out["d3q19_x_d3q27"] = round(out["d3q19"]["mlups"] / out["d3q27"]["mlups"], 3)
    return out


def q19_jet_leg(jet, steps, warmup, main_leg, chunk=250):
    """D3Q19 on the headline jet itself (alpha_b = 1/3 gives the coolant
    c_s^2 = 1/3), run for the headline leg's warmup + steps in chunks of
    `chunk` steps, each timed with events, with the FP64 audit between them
    (outside the timed region): the rate is taken over every chunk run while
    the state was finite, and the first step at which it was not is reported."""
    import torch

    from paper_1804_08923_amd.lbm import LBM, LbmError
    prob = jet.replace(lattice=19, alpha_b=1.0 / 3.0)
    sim = LBM(prob, device="cuda:0")
    N = prob.n_nodes
    stream = sim.stream
    nonfinite_at = None
    timed_ms, timed_steps = 0.0, 0
    done = 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    while done < warmup + steps:
        k = min(chunk, warmup + steps - done)
        e0.record(stream)
        sim.step(k)
        e1.record(stream)
        torch.cuda.synchronize()
        try:
            sim.macroscopic(audit=True)
        except LbmError as err:
            if err.code != -4:
                raise
            nonfinite_at = done + k
            break
        timed_ms += e0.elapsed_time(e1)
        timed_steps += k
        done += k
    kms = [0.0, 0.0]
    if nonfinite_at is None:
        sim.profile(True)
        sim.step(PROFILE_STEPS)
        ms, launches = sim.profile_read()
        sim.profile(False)
        kms = [ms[0] / launches[0], ms[1] / launches[1]]
    sim.close()
    del sim
    torch.cuda.empty_cache()
    fb, db = Q19_FUSED_BYTES, Q19_DENSITY_BYTES
    mlups = N * timed_steps / (timed_ms * 1e-3) / 1e6 if timed_steps else None
    out = {"workload": prob.name, "timed_steps": timed_steps, "mlups": round(mlups, 1) if mlups else None,
           "x_d3q27": round(mlups / main_leg["mlups"], 3) if mlups else None,
           "nonfinite_at_step": nonfinite_at, "finite": nonfinite_at is None}
    if nonfinite_at is None:
        out.update({"fused_kernel_ms": round(kms[1], 4), "density_kernel_ms": round(kms[0], 4),
                    "fused_kernel_gbs": round(fb * N / (kms[1] * 1e-3) / 1e9, 1),
                    "step_roofline_frac": round(mlups / (HBM_PEAK_GBS * 1e9 / Q19_STEP_BYTES / 1e6), 4)})
    log(f"bench: {prob.name} D3Q19: {out['mlups']} MLUPS over {timed_steps} timed steps "
        f"({out['x_d3q27']}x D3Q27); non-finite at step {nonfinite_at}")
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, nz_sample=8, budget_s=10.0):
    """The FP64 oracle on a slab of the same jet (full cross-section, nz_sample
    planes, from the initial state), on all threads and on one, each for about
    budget_s seconds."""
    from oracle import Oracle
    from oracle import make_params as or_params
    import numpy as np
    sp = prob.replace(nz=nz_sample)
    orc = Oracle("f64")
    p = or_params(sp)
    N = sp.n_nodes
    res = {}
    n_all = orc.num_threads()
    for label, threads in (("all", n_all), ("one", 1)):
        orc.set_num_threads(threads)
        fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, sp.rho_b0))
        steps, t_used = 0, 0.0
        while t_used < budget_s:
            t0 = time.perf_counter()
            orc.step(p, sp.A, fr, fb, h, steps, 1)
            t_used += time.perf_counter() - t0
            steps += 1
        res[label] = (N * steps / t_used / 1e6, steps, t_used, threads)
        del fr, fb, h
    orc.set_num_threads(n_all)
    v, s, t, c = res["all"]
    v1, s1, t1, _ = res["one"]
    return {"value": round(v, 4), "unit": "MLUPS", "cores": c, "kind": "oracle",
            "sample": f"{sp.nx}x{sp.ny}x{sp.nz} slab of the jet (same inlet, walls, outlet), FP64, from the initial "
                      f"state: {s} steps in {t:.1f} s on {c} threads; {s1} steps in {t1:.1f} s on 1 thread",
            "single_core_mlups": round(v1, 4), "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="jet-256x256x1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the BF16/FP16 storage legs")
    ap.add_argument("--legs", default="bf16,fp16,bf16eq,fp16eq", help="storage legs to run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-step timing")
    ap.add_argument("--no-lattices", action="store_true", help="skip the D3Q19 / D3Q27 periodic comparison")
    ap.add_argument("--lattice-steps", type=int, default=1000, help="timed steps of each lattice leg")
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
    log(f"bench: {prob.name} ({prob.n_nodes} nodes) fp32, develop {args.warmup} steps, time {args.steps} steps")

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
    log(f"bench: fp32 {main_leg['mlups']:.0f} MLUPS ({main_leg['ms_per_step']:.3f} ms/step); profiled: fused "
        f"{main_leg['fused_ms']:.3f} ms ({main_leg['fused_gbs']:.0f} GB/s), density {main_leg['density_ms']:.3f} ms, "
        f"boundary {main_leg['boundary_ms']:.3f} ms")
    log(f"bench: jet after {main_leg['diag']['step'] if main_leg['diag'] else '?'} steps: {main_leg['diag']}")
    legs = {}
    if not args.no_legs:
        for st in [s for s in args.legs.split(",") if s]:
            r = run_leg(prob.replace(storage=st), args.steps, args.warmup)
            legs[st] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                        "x_fp32": round(r["mlups"] / main_leg["mlups"], 3),
                        "step_roofline_frac": round(r["step_roofline_frac"], 4),
                        "fused_kernel_ms": round(r["fused_ms"], 4), "fused_kernel_gbs": round(r["fused_gbs"], 1),
                        "density_kernel_ms": round(r["density_ms"], 4), "finite": r["finite"]}
            log(f"bench: {st} {r['mlups']:.0f} MLUPS ({r['mlups'] / main_leg['mlups']:.2f}x fp32), fused "
                f"{r['fused_ms']:.3f} ms, density {r['density_ms']:.3f} ms")
    adj = None
    if not args.no_adjoint:
        a = adjoint_leg(prob, main_leg["ms_per_step"])
        fwd = main_leg["ms_per_step"]
        adj = {"adjoint_step_ms": round(a["adjoint_ms"], 4), "forward_step_ms": round(fwd, 4),
               "ratio": round(a["adjoint_ms"] / fwd, 3),
               "recompute_step_ms": round(a["recompute_ms"], 4), "recompute_ratio": round(a["recompute_ms"] / fwd, 3),
               "checkpoint_load_ms": round(a["load_ms"], 4),
               "gradient_step_ms": round(a["gradient_step_ms"], 4),
               "gradient_step_ratio": round(a["gradient_step_ms"] / fwd, 3), "finite": a["finite"],
               "note": "per step of a checkpointed gradient: forward step + recompute (a step into a snapshot) + "
                       "adjoint step; the checkpoint load is paid once per segment"}
        log(f"bench: adjoint step {a['adjoint_ms']:.3f} ms = {adj['ratio']:.2f}x forward, recompute "
            f"{a['recompute_ms']:.3f} ms = {adj['recompute_ratio']:.2f}x, gradient step {adj['gradient_step_ratio']:.2f}x")
    lat = None
    if not args.no_lattices:
        lat = lattice_legs(prob, args.lattice_steps, 200)
        log(f"bench: D3Q19 / D3Q27 on {lat['workload']}: {lat['d3q19_x_d3q27']:.2f}x")
        lat["jet"] = q19_jet_leg(prob, args.steps, args.warmup, main_leg)
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        cpu = cpu_baseline(prob)
        log(f"bench: oracle {cpu['value']:.3f} MLUPS on {cpu['cores']} threads, {cpu['single_core_mlups']:.4f} on one "
            f"({cpu['cpu_model']})")

    traffic = measured_traffic("fp32", prob.name)
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
                   "storage": "fp32", "bc": prob.bc, "gamma": prob.gamma, "eta": prob.meta.get("eta"),
                   "Re": prob.meta.get("Re"), "We": prob.meta.get("We"), "Fr": prob.meta.get("Fr"),
                   "developed_steps": args.warmup},
        "roofline": {"bound": "hbm", "achieved": round(main_leg["fused_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(main_leg["fused_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_collide<jet, fp32> (fused collide-recolour-stream)",
                     "bytes_per_node": FUSED_BYTES["fp32"], "avg_launch_ms": round(main_leg["fused_ms"], 4),
                     "timing": f"library events around each launch, {PROFILE_STEPS} steps right after the timed region"},
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
        "lattices": lat,
        "finite": main_leg["finite"],
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
