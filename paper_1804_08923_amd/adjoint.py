"""Gradients of a multi-step run through the library's adjoint step.

``rollout(sim, x0, nsteps, every=K, A=..., u_in=...)`` returns the state after
``nsteps`` steps of ``sim`` (an ``LBM`` created with ``adjoint=True``) started
from ``x0`` (lbm_get_state layout) as a differentiable torch tensor.  Its
backward pass runs the library's adjoint step backwards in time and yields the
gradients with respect to ``x0``, the perturbation strength ``A`` and the
inlet axial-velocity profile ``u_in``.

Checkpointing: the forward pass writes the state that ends every K-step
segment straight into a snapshot (lbm_step_into: the library's own layout,
no conversion).  The backward pass takes one segment at a time: it loads the
segment's checkpoint, recomputes the segment's states by stepping into
snapshot buffers (one forward step each), and reverses the segment with
lbm_adjoint_step_snapshot (lbm_adjoint_step for x0 itself).  Memory:
nsteps/K checkpoints plus K - 1 segment snapshots of snap_bytes each.  All
arithmetic runs in the library.
"""
from __future__ import annotations

import torch

from .lbm import LBM, Q


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, A, u_in, sim: LBM, t0: int, nsteps: int, every: int):
        sim.set_state(x0, t0)
        ckpts = [x0.detach().clone().contiguous()]
        for s in range(nsteps):
            if (s + 1) % every == 0 and s + 1 < nsteps:
                snap = sim.new_snapshot()
                sim.step_to_snapshot(snap)
                ckpts.append(snap)
            else:
                sim.step(1)
        xT = sim.get_state()
        ctx.sim, ctx.t0, ctx.nsteps, ctx.every, ctx.ckpts = sim, t0, nsteps, every, ckpts
        ctx.has_u = u_in is not None
        ctx.u_shape = u_in.shape if u_in is not None else None
        return xT

    @staticmethod
    def backward(ctx, gT):
        sim: LBM = ctx.sim
        dev = sim.device
        lam = gT.detach().to(torch.float32).contiguous().clone()
        lam_out = torch.empty_like(lam)
        dA = torch.zeros(1, dtype=torch.float64, device=dev)
        du = torch.zeros(sim.prob.nx * sim.prob.ny, dtype=torch.float32, device=dev) if ctx.has_u else None
        K, n, t0 = ctx.every, ctx.nsteps, ctx.t0
        seg_snaps = [sim.new_snapshot() for _ in range(min(K, n) - 1)]
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * K
            s1 = min(n, s0 + K)
            ck = ctx.ckpts[seg]
            if seg == 0:
                sim.set_state(ck, t0)
            else:
                sim.load_snapshot(ck, t0 + s0)
            for j in range(s1 - s0 - 1):
                sim.step_to_snapshot(seg_snaps[j])  # the state at t0 + s0 + 1 + j
            for s in reversed(range(s0, s1)):
                if s > s0:
                    sim.adjoint_step_snapshot(seg_snaps[s - s0 - 1], t0 + s, lam, lam_out, dA, du)
                elif seg == 0:
                    sim.adjoint_step(ck, t0 + s, lam, lam_out, dA, du)
                else:
                    sim.adjoint_step_snapshot(ck, t0 + s, lam, lam_out, dA, du)
                lam, lam_out = lam_out, lam
        del seg_snaps
        ctx.ckpts = None
        if du is not None:
            du = du.reshape(ctx.u_shape)
        return lam, dA.reshape(()), du, None, None, None, None


def rollout(sim: LBM, x0: torch.Tensor, nsteps: int, every: int = 100, t0: int = 0,
            A: torch.Tensor | None = None, u_in: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable ``nsteps``-step run of ``sim`` from ``x0`` at time ``t0``.

    ``A`` (0-d float64) and ``u_in`` (nx*ny float32) must hold the values the
    handle was built with; they are inputs only so that autograd can return
    their gradients."""
    if sim.adjoint is None:
        raise ValueError("the LBM handle was created without the adjoint work buffer (adjoint=True)")
    if nsteps < 1 or every < 1:
        raise ValueError("nsteps and every must be >= 1")
    if A is None:
        A = torch.tensor(float(sim.prob.A), dtype=torch.float64, device=sim.device)
    if abs(float(A.detach()) - float(sim.prob.A)) > 1e-12 * max(1.0, abs(float(sim.prob.A))):
        raise ValueError("A differs from the value the handle was created with")
    if u_in is not None:
        if sim.inlet is None or not torch.equal(u_in.detach().to(sim.device, torch.float32).reshape(-1), sim.inlet):
            raise ValueError("u_in differs from the inlet profile the handle was created with")
    x0 = x0.to(sim.device, torch.float32).contiguous()
    assert x0.numel() == 2 * Q * sim.sizes.n_nodes
    return _Rollout.apply(x0, A, u_in, sim, int(t0), int(nsteps), int(every))
