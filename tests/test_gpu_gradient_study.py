"""Gradient study on the 64x64x256 jet (D = 12, u = 0.03, gamma = 2, eta = 1,
Re = 500, We = 30, Fr = 10): 2 000 steps with a checkpoint every 100, through
rollout() and the library's adjoint step, at full size.

Objective: the dispersed-phase (red) volume sum (1 + phi) / 2 over a window of
planes after 2 000 steps.  Over the window z in [192, 256) it vanishes: the
jet head travels about 60 lattice units (plus a little buoyant acceleration)
in 2 000 steps, and the recolouring keeps the far field pure blue, so that
objective and all its gradients are zero.  The gradients are therefore checked
on the same functional over z in [32, 96), which the head crosses during the
run.

Reference: central differences of the FP64 oracle at h = 1e-4 relative
(tests/golden/gradient_study_jet64_fd.json, written by
tests/golden/make_gradient_study_fd.py, which calls only the oracle), for
dJ/dA and for dJ/du_in along a seeded direction e over the inlet columns
(the 112 columns of the 12 x 12 square that lie in the D = 12 circle).  Bar:
1e-4 relative on both gradients (measured 1.7e-5 and 2.7e-6).  The GPU's J
is also held to the oracle's (the mean of its two A runs) at 1e-4: the FP32
forward run drifts 5.3e-5 from the FP64 one over the 2 000 jet steps (1e-5
holds after 200 droplet steps).  A second, weaker check uses central
differences of the GPU's own FP32 forward run (h = 1e-2 relative; at 1e-4
the FP32 rounding of the state dominates the difference) at 1e-2.  The
single-step adjoint is checked element by element against the FP64 oracle's
complex-step tangent-linear elsewhere; this test covers the full-size
checkpointed chain.
"""
import json
import os

import numpy as np
import pytest

from harness import Q, say
from paper_1804_08923_amd.workloads import jet_64

pytestmark = pytest.mark.gpu

NSTEPS, EVERY = 2000, 100
WIN = (32, 96)
WIN_LITERAL = (192, 256)
FD_REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gradient_study_jet64_fd.json")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible ROCm device"
    return t


def _objective(torch, prob, xT, win):
    x = xT.double()
    a = x[:Q].sum(0) / prob.rho_r0
    b = x[Q:].sum(0) / prob.rho_b0
    phi = (a - b) / (a + b)
    nxy = prob.nx * prob.ny
    return (0.5 * (1.0 + phi))[win[0] * nxy:win[1] * nxy].sum()


def _forward_J(torch, prob, inlet, x0):
    from paper_1804_08923_amd.lbm import LBM
    sim = LBM(prob, inlet_uz=inlet)
    sim.set_state(x0, 0)
    sim.step(NSTEPS)
    J = float(_objective(torch, prob, sim.get_state(), WIN))
    sim.close()
    return J


def test_gradient_study_jet64(torch):
    from paper_1804_08923_amd.adjoint import rollout
    from paper_1804_08923_amd.lbm import LBM
    prob = jet_64()
    nx, ny = prob.nx, prob.ny
    xx, yy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    inside = ((xx - prob.inlet_cx) ** 2 + (yy - prob.inlet_cy) ** 2 < (prob.inlet_D / 2) ** 2).ravel()
    assert inside.sum() == 112
    inlet = np.full(nx * ny, prob.inlet_u, np.float32)
    say(f"gradient study {prob.name}: {NSTEPS} steps, checkpoint every {EVERY}")
    sim = LBM(prob, adjoint=True, inlet_uz=inlet)
    x0 = sim.get_state().clone().requires_grad_(True)
    A = torch.tensor(prob.A, dtype=torch.float64, device=sim.device, requires_grad=True)
    u_in = torch.from_numpy(inlet).to(sim.device).requires_grad_(True)
    xT = rollout(sim, x0, NSTEPS, every=EVERY, A=A, u_in=u_in)
    J_lit = float(_objective(torch, prob, xT.detach(), WIN_LITERAL))
    J = _objective(torch, prob, xT, WIN)
    J_val = float(J.detach())
    say(f"  J over z in {WIN_LITERAL}: {J_lit:.3e} (vanishes); J over z in {WIN}: {J_val:.6f}")
    assert J_lit < 1e-6
    assert J_val > 1.0
    J.backward()
    torch.cuda.synchronize()
    gA = float(A.grad)
    gu = u_in.grad.detach().cpu().numpy().astype(np.float64)
    x0_ref = x0.detach().clone()
    sim.close()
    del xT, x0
    torch.cuda.empty_cache()
    say(f"  adjoint: dJ/dA {gA:.6e}, |dJ/du_in| {np.linalg.norm(gu):.6e}")
    # inlet cells outside the circle are blue walls: no gradient reaches them
    assert np.all(gu[~inside] == 0.0)

    # the FP64 oracle's central differences
    with open(FD_REF) as fh:
        ref = json.load(fh)
    assert ref["steps"] == NSTEPS and tuple(ref["window_z"]) == WIN and ref["n_inlet"] == 112
    rng = np.random.default_rng(ref["e_seed"])
    e = np.where(inside, rng.standard_normal(nx * ny), 0.0)
    J_ora = 0.5 * (ref["J"]["A+"] + ref["J"]["A-"])
    relJ = abs(J_val - J_ora) / J_ora
    relA64 = abs(gA - ref["dJ_dA"]) / abs(ref["dJ_dA"])
    gue64 = float((gu * e).sum())
    relu64 = abs(gue64 - ref["dJ_du_dot_e"]) / abs(ref["dJ_du_dot_e"])
    say(f"  FP64 oracle: J {J_ora:.9f} (GPU rel {relJ:.2e}); dJ/dA {ref['dJ_dA']:.6e} (rel {relA64:.2e}); "
        f"dJ/du_in . e {ref['dJ_du_dot_e']:.6e} vs adjoint {gue64:.6e} (rel {relu64:.2e})")

    hA = 1e-2 * prob.A
    Jp = _forward_J(torch, prob.replace(A=prob.A + hA), inlet, x0_ref)
    Jm = _forward_J(torch, prob.replace(A=prob.A - hA), inlet, x0_ref)
    fdA = (Jp - Jm) / (2 * hA)
    relA = abs(gA - fdA) / abs(fdA)
    say(f"  dJ/dA central difference {fdA:.6e}: rel {relA:.2e}")

    hu = 1e-2 * prob.inlet_u
    Jp = _forward_J(torch, prob, (inlet + hu * e).astype(np.float32), x0_ref)
    Jm = _forward_J(torch, prob, (inlet - hu * e).astype(np.float32), x0_ref)
    # the FP32 profile actually used on each side
    de = ((inlet + hu * e).astype(np.float32).astype(np.float64)
          - (inlet - hu * e).astype(np.float32).astype(np.float64)) / (2 * hu)
    fdu = (Jp - Jm) / (2 * hu)
    gue = float((gu * de).sum())
    relu = abs(gue - fdu) / abs(fdu)
    say(f"  dJ/du_in . e adjoint {gue:.6e}, central difference {fdu:.6e}: rel {relu:.2e}")
    assert relJ < 1e-4
    assert relA64 < 1e-4
    assert relu64 < 1e-4
    assert relA < 1e-2
    assert relu < 1e-2
