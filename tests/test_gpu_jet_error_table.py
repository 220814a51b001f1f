"""Per-field error of every storage form against the FP64 oracle on the
128x128x512 jet (D = 16, u = 0.04, gamma = 2, eta = 1, Re = 1e3, We = 50,
Fr = 10, 1 % inlet noise) at the steps the oracle's cached run reached.

The FP64 oracle's run of the whole lattice takes hours on the host, so its
fields are made once by tests/golden/make_jet_oracle_fields.py (oracle only)
and shipped as a sample (tests/golden/jet_sample/): every node with x and y
multiples of 8, plus every node with even x and y around the jet column for
z < 160, with the maxima of |rho|, |u| and |phi| over the whole lattice as
the denominators.  The GPU runs the same jet from the same all-blue start in
each storage form; the table of relative L-inf errors (over the sample) is
printed.

Bars (FP32): step 100, rho 1e-6, u 1e-5, phi 2e-6 (measured 1.7e-7, 1.1e-6,
3.8e-7); step 1000, 1e-4 on each field (measured 1.1e-5, 1.5e-5, 4.1e-5).
The FP32 trajectory parts from the FP64 one as the jet amplifies rounding
(a factor of about 60 between steps 100 and 1000); the step-1000 bar is a
regression bound, since the oracle's own FP32 floor at that step would take
another six hours of host time.  The equilibrium-referenced FP16 form is held
to the 1e-3 u_max velocity bound at both steps; the other 16-bit forms miss
it and are reported (test_gpu_storage holds them to it as strict expected
failures at small size).  Skipped when the sample is absent.
"""
import os

import numpy as np
import pytest

from harness import say

pytestmark = pytest.mark.gpu

SAMPLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "jet_sample",
                      "jet-128x128x512_oracle_sample.npz")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible ROCm device"
    return t


@pytest.mark.skipif(not os.path.exists(SAMPLE), reason="cached FP64 oracle sample of the 128x128x512 jet is absent")
def test_jet128_error_table(torch):
    from paper_1804_08923_amd.lbm import LBM
    from paper_1804_08923_amd.workloads import jet_128
    ref = dict(np.load(SAMPLE))
    marks = [int(s) for s in ref["steps"]]
    prob = jet_128()
    idx = torch.from_numpy(ref["idx"].astype(np.int64)).cuda()
    table = {}
    for storage in ("fp32", "bf16", "fp16", "bf16eq", "fp16eq"):
        sim = LBM(prob.replace(storage=storage))
        done = 0
        for m in marks:
            sim.step(m - done)
            done = m
            f = sim.macroscopic(audit=True)
            rho = (f["rho_r"].double() + f["rho_b"].double())[idx]
            u = f["u"][idx]
            phi = f["phi"][idx]
            g = {"rho": rho.double().cpu().numpy(), "u": u.double().cpu().numpy(), "phi": phi.double().cpu().numpy()}
            mx = ref[f"max_{m}"]
            e = {"rho": np.abs(g["rho"] - ref[f"rho_{m}"]).max() / mx[0],
                 "u": np.linalg.norm(g["u"] - ref[f"u_{m}"], axis=1).max() / mx[1],
                 "phi": np.abs(g["phi"] - ref[f"phi_{m}"]).max() / mx[2]}
            tot = np.array(f["audit"])
            rt = ref[f"totals_{m}"]
            e["mass_r"] = abs(tot[0] - rt[0]) / rt[0]
            table[(storage, m)] = e
            say(f"  {storage:7s} step {m:5d}: rho {e['rho']:.2e}  u {e['u']:.2e}  phi {e['phi']:.2e}  "
                f"red mass {e['mass_r']:.2e}  (u_max {mx[1]:.3e})")
        sim.close()
        torch.cuda.empty_cache()
    bars = {100: (1e-6, 1e-5, 2e-6), 1000: (1e-4, 1e-4, 1e-4)}
    for m in marks:
        e = table[("fp32", m)]
        b = bars[m]
        assert e["rho"] <= b[0] and e["u"] <= b[1] and e["phi"] <= b[2], (m, e)
        assert table[("fp16eq", m)]["u"] <= 1e-3, (m, table[("fp16eq", m)])
