"""Write the FP64 oracle's macroscopic fields of a jet workload at given steps.

Test infrastructure: calls only the oracle (``oracle/``) on the seeded,
synthetic jet set-up of Sec. IV A (all-blue domain at rest, circular inlet
with radial noise, free-slip walls, convective outlet, buoyancy).  The fields
are the reference of the per-field error table of the 16-bit storage forms
(rho, u, phi at the listed steps).  They are large, so they are cached under
``tests/golden/cache/`` (not in version control):

    python tests/golden/make_jet_oracle_fields.py --workload jet-128x128x512 \
        --steps 100,1000

Each output ``<workload>_oracle_t<step>.npz`` holds FP32 copies of rho_r,
rho_b, u (N x 3) and phi in node order (x fastest), plus the FP64 totals
sum rho_r, sum rho_b and sum rho u of the FP64 state.  Progress goes to
stdout.  Thread count: OMP_NUM_THREADS.

    python tests/golden/make_jet_oracle_fields.py --sample jet-128x128x512 --steps 100,1000

writes the sample the GPU comparison reads, tests/golden/jet_sample/
<workload>_oracle_sample.npz: the fields rho, u, phi (FP32) per step at the
nodes listed in ``idx`` (node order), with the maxima of |rho|, |u|, |phi|
over the whole lattice (the denominators of the relative errors) and the
FP64 totals.  The sample: every node with x and y multiples of 8 (all z),
plus, around the jet column (|x - cx|, |y - cy| <= 24, z < 160, where the
interface is during the first 1000 steps), every node with even x and y.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle, make_params  # noqa: E402
from paper_1804_08923_amd.workloads import WORKLOADS  # noqa: E402

CACHE = os.path.join(HERE, "cache")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="jet-128x128x512")
    ap.add_argument("--steps", default="100,1000")
    ap.add_argument("--chunk", type=int, default=10)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--sample", metavar="WORKLOAD", help="write the shipped sample of cached fields")
    a = ap.parse_args()
    if a.sample:
        return write_sample(a.sample, sorted(int(s) for s in a.steps.split(",")), a.out)
    prob = WORKLOADS[a.workload]()
    assert prob.bc == "jet" and prob.init == "jet"
    marks = sorted(int(s) for s in a.steps.split(","))
    os.makedirs(a.out, exist_ok=True)
    orc = Oracle("f64")
    p = make_params(prob)
    N = prob.n_nodes
    fr, fb, hist = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    t, t_start = 0, time.time()
    print(f"oracle {a.workload}: {N} nodes, {orc.num_threads()} threads, marks {marks}", flush=True)
    for m in marks:
        while t < m:
            k = min(a.chunk, m - t)
            orc.step(p, prob.A, fr, fb, hist, t, k)
            t += k
            el = time.time() - t_start
            print(f"step {t}  {el:.0f} s  {t * N / el / 1e6:.3f} MLUPS", flush=True)
        rr, rb, u, ph = orc.macroscopic(p, fr, fb)
        rho = rr + rb
        f = fr + fb
        c, _ = orc.lattice()
        mom = np.array([float((f * c[:, k][:, None]).sum()) for k in range(3)])
        path = os.path.join(a.out, f"{a.workload}_oracle_t{m}.npz")
        np.savez(path + ".tmp.npz", rho_r=rr.astype(np.float32), rho_b=rb.astype(np.float32),
                 u=u.astype(np.float32), phi=ph.astype(np.float32),
                 totals=np.array([rr.sum(), rb.sum(), *mom]), step=np.int64(m),
                 max_u=np.float64(np.linalg.norm(u, axis=1).max()), max_rho=np.float64(rho.max()))
        os.replace(path + ".tmp.npz", path)
        print(f"wrote {path}", flush=True)
    return 0


def write_sample(workload: str, marks, cache: str) -> int:
    prob = WORKLOADS[workload]()
    idx = sample_nodes(prob)
    out = {"idx": idx.astype(np.int32), "steps": np.array(marks, np.int64)}
    for m in marks:
        with np.load(os.path.join(cache, f"{workload}_oracle_t{m}.npz")) as f:
            rho = (f["rho_r"].astype(np.float64) + f["rho_b"].astype(np.float64))
            u = f["u"]
            phi = f["phi"]
            out[f"rho_{m}"] = rho[idx].astype(np.float32)
            out[f"u_{m}"] = u[idx]
            out[f"phi_{m}"] = phi[idx]
            out[f"max_{m}"] = np.array([np.abs(rho).max(), np.linalg.norm(u.astype(np.float64), axis=1).max(),
                                        np.abs(phi).max()])
            out[f"totals_{m}"] = f["totals"]
    ship = os.path.join(HERE, "jet_sample")
    os.makedirs(ship, exist_ok=True)
    path = os.path.join(ship, f"{workload}_oracle_sample.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path} ({idx.size} nodes)", flush=True)
    return 0


def sample_nodes(prob) -> np.ndarray:
    """Node indices of the shipped sample (see the module docstring)."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coarse = (x % 8 == 0) & (y % 8 == 0)
    near = ((np.abs(x - prob.inlet_cx) <= 24) & (np.abs(y - prob.inlet_cy) <= 24) & (z < 160)
            & (x % 2 == 0) & (y % 2 == 0))
    return np.flatnonzero((coarse | near).ravel()).astype(np.int64)


if __name__ == "__main__":
    sys.exit(main())
