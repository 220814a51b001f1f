"""The FP32 floors of the droplet with central-moment relaxation.

The GPU keeps its state in FP32 -- the colour-blind deviation d_i = f_i - w_i
rho_b0 and, per node, the minority colour -- and computes in FP32.  Two
floors bracket what an FP32 implementation of this run can reach, both
measured here on the CPU against the FP64 oracle after 200 steps of the
droplet with tau != 1, gamma = 2 and gravity:

* storage floor: the FP64 oracle with its state rounded to that FP32 form
  after every step (exact arithmetic otherwise);
* plain FP32 scheme: the oracle's FP32 build, which evaluates the paper's
  scheme literally in single precision and stores f itself.

The GPU parity test of the same case takes its velocity bar between them.
"""
import numpy as np

from harness import DROPLET_CM_U_FLOOR, DROPLET_CM_U_PLAIN_FP32, Q, oracle_fields, oracle_init, rel_linf
from paper_1804_08923_amd.workloads import droplet_cm


def _round_to_fp32_storage(prob, w, fr, fb):
    """(fr, fb) as the FP32 (d, minority colour) form holds them."""
    d = ((fr + fb) - w[:, None] * prob.rho_b0).astype(np.float32).astype(np.float64)
    red_minor = fr.sum(axis=0) <= fb.sum(axis=0)
    keep = np.where(red_minor, fr, fb).astype(np.float32).astype(np.float64)
    other = (d + w[:, None] * prob.rho_b0) - keep
    fr[:] = np.where(red_minor, keep, other)
    fb[:] = np.where(red_minor, other, keep)


def test_droplet_cm_fp32_storage_floor(orc):
    prob = droplet_cm()
    w = np.asarray(orc.lattice()[1], np.float64)
    p, fr, fb, h = oracle_init(orc, prob)
    p2, gr, gb, h2 = oracle_init(orc, prob)
    _round_to_fp32_storage(prob, w, gr, gb)
    for t in range(prob.steps):
        orc.step(p2, prob.A, gr, gb, h2, t, 1)
        _round_to_fp32_storage(prob, w, gr, gb)
    orc.step(p, prob.A, fr, fb, h, 0, prob.steps)
    exact = oracle_fields(orc, p, fr, fb)
    rounded = oracle_fields(orc, p2, gr, gb)
    e = {k: rel_linf(rounded[k], exact[k]) for k in ("rho", "u", "phi", "rho_r")}
    print("FP32 storage floor after", prob.steps, "steps:", e)
    # the recorded floor the GPU bar is built on
    assert 0.5 * DROPLET_CM_U_FLOOR <= e["u"] <= 2.0 * DROPLET_CM_U_FLOOR, e
    for k in ("rho", "phi", "rho_r"):
        assert e[k] < 1e-6, (k, e)


def test_droplet_cm_plain_fp32_scheme():
    from oracle import Oracle
    prob = droplet_cm()
    o64, o32 = Oracle("f64"), Oracle("f32")
    p, fr, fb, h = oracle_init(o64, prob)
    p2, gr, gb, h2 = oracle_init(o32, prob)
    o64.step(p, prob.A, fr, fb, h, 0, prob.steps)
    o32.step(p2, prob.A, gr, gb, h2, 0, prob.steps)
    exact = oracle_fields(o64, p, fr, fb)
    single = oracle_fields(o32, p2, gr, gb)
    e = {k: rel_linf(single[k], exact[k]) for k in ("rho", "u", "phi", "rho_r")}
    print("plain FP32 scheme after", prob.steps, "steps:", e)
    assert 0.5 * DROPLET_CM_U_PLAIN_FP32 <= e["u"] <= 2.0 * DROPLET_CM_U_PLAIN_FP32, e
