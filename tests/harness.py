"""Helpers shared by the GPU parity tests: run the same seeded problem through
the oracle and through the HIP library, and compare fields."""
from __future__ import annotations

import sys

import numpy as np

from oracle import Oracle, make_params as or_params
from paper_1804_08923_amd.workloads import Problem

Q = 27

# Velocity errors (rel L-inf) after 200 steps of the droplet-32-cm case,
# measured by tests/test_oracle_storage_floor.py: the FP64 oracle with its
# state rounded to the FP32 storage form after every step (the floor of FP32
# storage with exact arithmetic), and the oracle's plain FP32 build (the
# paper's scheme evaluated and stored in single precision).
DROPLET_CM_U_FLOOR = 2.8e-6
DROPLET_CM_U_PLAIN_FP32 = 1.9e-4


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_linf(a, b):
    """max |a - b| / max |b| (vector fields compared by magnitude per node)."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if a.ndim == 2:
        return float(np.linalg.norm(a - b, axis=1).max() / max(np.linalg.norm(b, axis=1).max(), 1e-300))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_init(orc: Oracle, prob: Problem):
    p = or_params(prob)
    if prob.init == "droplet":
        fr, fb, h = orc.init_droplet(p, prob.center, prob.drop_R, prob.drop_W)
    elif prob.init == "jet":
        N = prob.n_nodes
        fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    else:
        raise ValueError(prob.init)
    return p, fr, fb, h


def oracle_fields(orc, p, fr, fb):
    rr, rb, u, ph = orc.macroscopic(p, fr, fb)
    return dict(rho_r=rr, rho_b=rb, rho=rr + rb, u=u, phi=ph)


def gpu_fields(sim):
    m = sim.macroscopic()
    out = {k: v.detach().cpu().numpy().astype(np.float64) for k, v in m.items() if k != "audit"}
    out["rho"] = out["rho_r"] + out["rho_b"]
    return out


def random_state(orc: Oracle, prob: Problem, seed: int, noise=2e-4):
    """Random but physical populations (fr, fb) in FP64 built by the oracle's
    initialiser from seeded fields plus small population noise."""
    from synth import population_noise, random_state_fields
    p = or_params(prob)
    rr, rb, u = random_state_fields(prob, seed)
    fr, fb, h = orc.init_fields(p, rr, rb, u)
    nz = population_noise(prob.n_nodes, seed, amp=noise)
    fr += np.where(fr > 1e-3, nz[0], 0.0)
    fb += np.where(fb > 1e-3, nz[1], 0.0)
    return p, fr, fb, h


def state_to_f32(fr, fb):
    """The FP32 state both sides start from (the oracle gets it back in FP64)."""
    st = np.concatenate([fr, fb], axis=0).astype(np.float32)
    return st, st[:Q].astype(np.float64), st[Q:].astype(np.float64)


def hist_from(p, fr, fb):
    P = p.nx * p.ny
    h = np.zeros((2 * Q, P))
    h[:Q] = fr[:, -P:]
    h[Q:] = fb[:, -P:]
    return h
