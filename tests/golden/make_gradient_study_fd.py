"""Central differences of the FP64 oracle for the 64x64x256 gradient study.

Test infrastructure: calls only the oracle (``oracle/``).  The differentiation
workload is the jet of Sec. IV A on a 64x64x256 lattice (D = 12, u = 0.03,
gamma = 2, eta = 1, Re = 500, We = 30, Fr = 10, no inlet noise), started all
blue at rest and run for 2000 steps; the objective is the red volume
J = sum (1 + phi)/2 over the planes z in [32, 96) of the final state.  Its
derivatives with respect to the perturbation strength A and, along a seeded
direction e over the 112 inlet columns, the inlet axial velocity profile are
taken by central differences with relative steps 1e-4 (h_A = 1e-4 A,
h_u = 1e-4 u), in FP64, so truncation (O(h^2), ~1e-8 relative) and rounding
(~1e-12 relative) stay far below the 1e-4 bar the GPU adjoint is held to.

One oracle run per call (each takes ~15 min on 16 host threads):

    python tests/golden/make_gradient_study_fd.py --run A+ --out <file.json>

with --run one of A+, A-, u+, u-; ``--combine a.json b.json ...`` merges the
four runs into tests/golden/gradient_study_jet64_fd.json.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle, make_params  # noqa: E402
from paper_1804_08923_amd.workloads import jet_64  # noqa: E402

NSTEPS = 2000
WIN = (32, 96)
REL_H = 1e-4
E_SEED = 2018
OUT = os.path.join(HERE, "gradient_study_jet64_fd.json")


def inlet_direction(prob):
    """The direction e over the inlet columns (x fastest; zero outside the
    circle), the same draw the GPU test makes."""
    nx, ny = prob.nx, prob.ny
    xx, yy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    inside = ((xx - prob.inlet_cx) ** 2 + (yy - prob.inlet_cy) ** 2 < (prob.inlet_D / 2) ** 2).ravel()
    rng = np.random.default_rng(E_SEED)
    return np.where(inside, rng.standard_normal(nx * ny), 0.0), inside


def objective(prob, fr, fb):
    a = fr.sum(axis=0) / prob.rho_r0
    b = fb.sum(axis=0) / prob.rho_b0
    phi = (a - b) / (a + b)
    nxy = prob.nx * prob.ny
    return float((0.5 * (1.0 + phi))[WIN[0] * nxy:WIN[1] * nxy].sum())


def run(which: str) -> dict:
    prob = jet_64()
    e, inside = inlet_direction(prob)
    hA = REL_H * prob.A
    hu = REL_H * prob.inlet_u
    sgn = 1.0 if which.endswith("+") else -1.0
    A = prob.A + (sgn * hA if which.startswith("A") else 0.0)
    inlet = np.full(prob.nx * prob.ny, prob.inlet_u, np.float64)
    if which.startswith("u"):
        inlet = inlet + sgn * hu * e
    orc = Oracle("f64")
    p = make_params(prob)
    N = prob.n_nodes
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    t0 = time.time()
    done = 0
    while done < NSTEPS:
        k = min(50, NSTEPS - done)
        orc.step(p, A, fr, fb, h, done, k, inlet_uz=inlet)
        done += k
        print(f"{which}: step {done} of {NSTEPS}, {time.time() - t0:.0f} s", flush=True)
    J = objective(prob, fr, fb)
    return {"run": which, "J": J, "A": A, "hA": hA, "hu": hu, "threads": orc.num_threads(),
            "seconds": round(time.time() - t0, 1), "n_inlet": int(inside.sum())}


def combine(paths):
    runs = {}
    for pth in paths:
        with open(pth) as fh:
            r = json.load(fh)
        runs[r["run"]] = r
    assert set(runs) == {"A+", "A-", "u+", "u-"}, sorted(runs)
    prob = jet_64()
    hA, hu = runs["A+"]["hA"], runs["u+"]["hu"]
    out = {
        "workload": prob.name, "steps": NSTEPS, "window_z": list(WIN), "relative_step": REL_H,
        "e_seed": E_SEED, "n_inlet": runs["A+"]["n_inlet"],
        "J": {k: v["J"] for k, v in runs.items()},
        "dJ_dA": (runs["A+"]["J"] - runs["A-"]["J"]) / (2 * hA),
        "dJ_du_dot_e": (runs["u+"]["J"] - runs["u-"]["J"]) / (2 * hu),
        "note": "FP64 oracle, central differences, all blue at rest at t = 0, no inlet noise",
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--run", choices=["A+", "A-", "u+", "u-"])
    ap.add_argument("--out")
    ap.add_argument("--combine", nargs="+")
    a = ap.parse_args()
    if a.combine:
        combine(a.combine)
        return 0
    r = run(a.run)
    with open(a.out, "w") as fh:
        json.dump(r, fh, indent=1)
    print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
