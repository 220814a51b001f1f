"""Adjoint step through the C ABI against the oracle's complex-step tangent-linear.

The oracle's complex-step build gives J v = Im(S(x + i h v))/h exactly up to
rounding (J the Jacobian of one FP64 oracle step S).  The adjoint step must
satisfy the dot-product identity <w, J v> = <J^T w, v> and return the
parameter gradients <w, dS/dA> and <w, dS/du_in>.  Checked:
  * every element of J^T w on tiny periodic and jet lattices (all nodes are
    near a wall, the inlet or the outlet there);
  * dot products with random and boundary-supported directions, dJ/dA and
    dJ/du_in on lattices of several 256-node blocks;
  * the same reverse step with the forward state given as a snapshot (the
    library's own layout, lbm_adjoint_step_snapshot), element by element;
  * snapshots: stepping into snapshots, saving and loading them reproduce
    plain stepping bit for bit;
  * a checkpointed multi-step gradient through the torch.autograd binding
    (checkpoints and recomputed states as snapshots) against complex step and
    central differences of the FP64 oracle.
Tolerances: the adjoint's node arithmetic is FP32 (FP64 only for the dJ/dA
and dJ/du_in accumulations), so single-step results agree to ~1e-6 relative;
the target bar for gradients is 1e-4 relative.
"""
import numpy as np
import pytest

from harness import Q, random_state, say
from oracle import make_params as or_params
from paper_1804_08923_amd.workloads import Problem

pytestmark = pytest.mark.gpu

H = 1e-20  # complex-step size


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible ROCm device"
    return t


def _jet(nx, ny, nz, D, noise=0.01, **kw):
    base = dict(name="adj-jet", nx=nx, ny=ny, nz=nz, bc="jet", rho_r0=1.0, rho_b0=0.5, nu_r=0.02, nu_b=0.035,
                A=3e-3, g=(0.0, 0.0, 2e-5), inlet_cx=(nx - 1) / 2.0, inlet_cy=(ny - 1) / 2.0, inlet_D=D,
                inlet_u=0.03, noise_amp=noise, noise_seed=11, init="jet")
    base.update(kw)
    return Problem(**base)


def _periodic(nx, ny, nz, **kw):
    base = dict(name="adj-per", nx=nx, ny=ny, nz=nz, bc="periodic", rho_r0=1.0, rho_b0=0.5, nu_r=0.02,
                nu_b=0.05, A=2e-3, g=(1e-4, -2e-4, 3e-4), init="jet")
    base.update(kw)
    return Problem(**base)


def _inlet_profile(prob, seed):
    """A nonuniform axial inlet profile (FP32 values)."""
    rng = np.random.default_rng(seed)
    return (prob.inlet_u * (1.0 + 0.2 * rng.standard_normal(prob.nx * prob.ny))).astype(np.float32)


def _state(orc, prob, seed):
    """Random FP32 state (54, N) with its exact FP64 copy."""
    _, fr, fb, _ = random_state(orc, prob, seed=seed, noise=2e-3)
    st = np.concatenate([fr, fb]).astype(np.float32)
    return st, st.astype(np.float64)


def _cs_step(orc_cs, prob, st64, t, v=None, dA=0.0, inlet=None, du=None):
    """Tangent of one oracle step: (J v + dS/dA dA + dS/du du), shape (54, N)."""
    p = or_params(prob)
    x = st64.astype(np.complex128)
    if v is not None:
        x = x + 1j * H * v
    fr, fb = np.ascontiguousarray(x[:Q]), np.ascontiguousarray(x[Q:])
    P = prob.nx * prob.ny
    hist = np.ascontiguousarray(np.concatenate([fr[:, -P:], fb[:, -P:]]))
    iu = None
    if inlet is not None:
        iu = inlet.astype(np.complex128)
        if du is not None:
            iu = iu + 1j * H * du
    orc_cs.step(p, prob.A + 1j * H * dA, fr, fb, hist, t, 1, inlet_uz=iu)
    return np.concatenate([fr.imag, fb.imag]) / H


def _gpu_adjoint(torch, prob, st32, t, w32, inlet=None):
    from paper_1804_08923_amd.lbm import LBM
    sim = LBM(prob, adjoint=True, inlet_uz=inlet)
    dev = sim.device
    st = torch.from_numpy(st32).to(dev)
    lam_in = torch.from_numpy(w32).to(dev)
    lam_out = torch.empty_like(lam_in)
    dA = torch.zeros(1, dtype=torch.float64, device=dev)
    du = torch.zeros(prob.nx * prob.ny, dtype=torch.float32, device=dev)
    sim.adjoint_step(st, t, lam_in, lam_out, dA, du)
    torch.cuda.synchronize()
    out = lam_out.cpu().numpy().astype(np.float64), float(dA.item()), du.cpu().numpy().astype(np.float64)
    sim.close()
    return out


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _dot_check(name, gpu, w, d, tol=2e-6):
    """gpu ~ <w, d> within tol times the condition scale sum |w_i d_i| of the
    dot product (random cotangents make <w, d> cancel, and the GPU evaluates
    the forward fields in FP32)."""
    ref = float((w * d).sum())
    scale = float(np.abs(w * d).sum())
    say(f"  {name}: gpu {gpu:.9e} oracle {ref:.9e} rel {_rel(gpu, ref):.2e} "
        f"err/sum|w d| {abs(gpu - ref) / scale:.2e}")
    assert abs(gpu - ref) <= tol * scale


@pytest.mark.parametrize("case", ["periodic-4x3x3", "jet-5x5x4", "jet-6x5x3"])
def test_adjoint_every_element(torch, orc, orc_cs, case):
    """J^T w element by element on tiny lattices: column k of J from one complex
    step per (population, node)."""
    prob = {"periodic-4x3x3": _periodic(4, 3, 3), "jet-5x5x4": _jet(5, 5, 4, D=3.2),
            "jet-6x5x3": _jet(6, 5, 3, D=3.0, g=(0.0, 0.0, -3e-5))}[case]
    say(f"adjoint every element {case}")
    st32, st64 = _state(orc, prob, seed=3)
    rng = np.random.default_rng(4)
    w32 = rng.standard_normal(st32.shape).astype(np.float32)
    t = 5
    inlet = _inlet_profile(prob, 9) if prob.bc == "jet" else None
    lam, dA, du = _gpu_adjoint(torch, prob, st32, t, w32, inlet)
    N = prob.n_nodes
    ref = np.zeros_like(lam)
    w64 = w32.astype(np.float64)
    for k in range(2 * Q):
        for n in range(N):
            v = np.zeros_like(st64)
            v[k, n] = 1.0
            ref[k, n] = (w64 * _cs_step(orc_cs, prob, st64, t, v=v, inlet=inlet)).sum()
    err = np.abs(lam - ref).max() / np.abs(ref).max()
    say(f"  max |J^T w - ref| / max |ref| = {err:.2e} (max |ref| = {np.abs(ref).max():.3e})")
    assert err < 2e-6
    _dot_check("dJ/dA", dA, w64, _cs_step(orc_cs, prob, st64, t, dA=1.0, inlet=inlet))
    if prob.bc == "jet":
        P = prob.nx * prob.ny
        for q in range(P):
            e = np.zeros(P)
            e[q] = 1.0
            rq = (w64 * _cs_step(orc_cs, prob, st64, t, inlet=inlet, du=e)).sum()
            assert abs(du[q] - rq) <= 1e-5 * max(abs(rq), 1e-3 * np.abs(du).max()), (q, du[q], rq)
        say(f"  dJ/du_in: {np.count_nonzero(du)} inlet columns, max |.| = {np.abs(du).max():.3e}")


@pytest.mark.parametrize("case", ["periodic-16x12x10", "jet-14x12x10", "jet-20x18x12"])
def test_adjoint_dot_products(torch, orc, orc_cs, case):
    """<w, J v> = <J^T w, v> for random v, for v supported on the boundary
    planes, and the parameter gradients, on lattices of several blocks."""
    prob = {"periodic-16x12x10": _periodic(16, 12, 10), "jet-14x12x10": _jet(14, 12, 10, D=6),
            "jet-20x18x12": _jet(20, 18, 12, D=9, noise=0.0)}[case]
    say(f"adjoint dot products {case}")
    st32, st64 = _state(orc, prob, seed=7)
    rng = np.random.default_rng(8)
    w32 = rng.standard_normal(st32.shape).astype(np.float32)
    w64 = w32.astype(np.float64)
    t = 17
    inlet = _inlet_profile(prob, 2) if prob.bc == "jet" else None
    lam, dA, du = _gpu_adjoint(torch, prob, st32, t, w32, inlet)
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    edge = ((x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z <= 1) | (z >= nz - 3)).ravel()
    for kind in ("random", "boundary"):
        v = rng.standard_normal(st64.shape)
        if kind == "boundary":
            v[:, ~edge] = 0.0
        lhs = (w64 * _cs_step(orc_cs, prob, st64, t, v=v, inlet=inlet)).sum()
        rhs = (lam * v).sum()
        say(f"  {kind}: <w, Jv> = {lhs:.9e}, <J^T w, v> = {rhs:.9e}, rel {_rel(rhs, lhs):.2e}")
        assert _rel(rhs, lhs) < 1e-5
        assert abs(rhs - lhs) <= 2e-6 * float(np.abs(lam * v).sum())
    _dot_check("dJ/dA", dA, w64, _cs_step(orc_cs, prob, st64, t, dA=1.0, inlet=inlet))
    if prob.bc == "jet":
        e = rng.standard_normal(nx * ny)
        _dot_check("dJ/du_in . e", float((du * e).sum()), w64, _cs_step(orc_cs, prob, st64, t, inlet=inlet, du=e))


def _gpu_snapshot_case(torch, prob, st32, t_start, nsteps, w32, inlet=None):
    """From st32 at time t_start, step nsteps - 1 times and once more into a
    snapshot; return the FP32 state there (lbm_get_state) and the reverse
    step from the snapshot."""
    from paper_1804_08923_amd.lbm import LBM
    sim = LBM(prob, adjoint=True, inlet_uz=inlet)
    dev = sim.device
    sim.set_state(torch.from_numpy(st32).to(dev), t_start)
    sim.step(nsteps - 1)
    snap = sim.new_snapshot()
    sim.step_to_snapshot(snap)
    t = sim.time
    x_t = sim.get_state().cpu().numpy()
    lam_in = torch.from_numpy(w32).to(dev)
    lam_out = torch.empty_like(lam_in)
    dA = torch.zeros(1, dtype=torch.float64, device=dev)
    du = torch.zeros(prob.nx * prob.ny, dtype=torch.float32, device=dev)
    sim.adjoint_step_snapshot(snap, t, lam_in, lam_out, dA, du)
    torch.cuda.synchronize()
    out = lam_out.cpu().numpy().astype(np.float64), float(dA.item()), du.cpu().numpy().astype(np.float64)
    sim.close()
    return t, x_t, out


@pytest.mark.parametrize("case", ["periodic-4x3x3", "jet-5x5x4", "jet-6x5x3"])
def test_adjoint_from_snapshot_every_element(torch, orc, orc_cs, case):
    """The reverse step with x_t given as a snapshot: J^T w element by element
    against complex step of the oracle at the same state (its FP32 copy from
    lbm_get_state), and dJ/dA, dJ/du_in by dot products."""
    prob = {"periodic-4x3x3": _periodic(4, 3, 3), "jet-5x5x4": _jet(5, 5, 4, D=3.2),
            "jet-6x5x3": _jet(6, 5, 3, D=3.0, g=(0.0, 0.0, -3e-5))}[case]
    say(f"adjoint from a snapshot, every element {case}")
    st32, _ = _state(orc, prob, seed=13)
    rng = np.random.default_rng(14)
    w32 = rng.standard_normal(st32.shape).astype(np.float32)
    inlet = _inlet_profile(prob, 6) if prob.bc == "jet" else None
    t, x_t, (lam, dA, du) = _gpu_snapshot_case(torch, prob, st32, 4, 3, w32, inlet)
    assert t == 7
    st64 = x_t.astype(np.float64)
    N = prob.n_nodes
    ref = np.zeros_like(lam)
    w64 = w32.astype(np.float64)
    for k in range(2 * Q):
        for n in range(N):
            v = np.zeros_like(st64)
            v[k, n] = 1.0
            ref[k, n] = (w64 * _cs_step(orc_cs, prob, st64, t, v=v, inlet=inlet)).sum()
    err = np.abs(lam - ref).max() / np.abs(ref).max()
    say(f"  max |J^T w - ref| / max |ref| = {err:.2e}")
    # the snapshot holds the state the FP32 copy rounds: the Jacobians differ at that level
    assert err < 1e-5
    _dot_check("dJ/dA", dA, w64, _cs_step(orc_cs, prob, st64, t, dA=1.0, inlet=inlet), tol=1e-5)
    if prob.bc == "jet":
        e = rng.standard_normal(prob.nx * prob.ny)
        _dot_check("dJ/du_in . e", float((du * e).sum()), w64, _cs_step(orc_cs, prob, st64, t, inlet=inlet, du=e),
                   tol=1e-5)


@pytest.mark.parametrize("case,storage", [("periodic-16x12x10", "fp32"), ("jet-14x12x10", "fp32"),
                                          ("jet-14x12x10", "bf16"), ("jet-14x12x10", "fp16eq")])
def test_snapshots_reproduce_plain_steps(torch, orc, case, storage):
    """lbm_step_into, lbm_snapshot_save and lbm_snapshot_load change nothing
    about the run: the states agree bit for bit with plain stepping."""
    from paper_1804_08923_amd.lbm import LBM
    prob = {"periodic-16x12x10": _periodic(16, 12, 10), "jet-14x12x10": _jet(14, 12, 10, D=6)}[case]
    prob = prob.replace(storage=storage)
    say(f"snapshots {case} {storage}")
    st32, _ = _state(orc, prob, seed=5)
    dev = torch.device("cuda:0")
    x0 = torch.from_numpy(st32).to(dev)

    def run(plan):
        sim = LBM(prob, adjoint=True)
        sim.set_state(x0, 2)
        snaps = []
        for op in plan:
            if op == "s":
                sim.step(1)
            elif op == "i":
                snaps.append(sim.new_snapshot())
                sim.step_to_snapshot(snaps[-1])
            elif op == "v":
                snaps.append(sim.new_snapshot())
                sim.save_snapshot(snaps[-1])
                saved_t = sim.time
            elif op == "l":
                sim.load_snapshot(snaps[-1], saved_t)
        out = sim.get_state().cpu().numpy(), sim.time
        sim.close()
        return out

    ref, tr = run("sssssss")
    for plan in ("ssiisss", "iiiiiii", "ssvsssl" + "sssss"):
        got, tg = run(plan)
        assert tg == tr, (plan, tg, tr)
        assert np.array_equal(got, ref), plan


def _objective_np(prob, fr, fb, z_lo):
    """J = sum over z >= z_lo of (1 + phi)/2 (red volume), any dtype."""
    a = fr.sum(axis=0) / prob.rho_r0
    b = fb.sum(axis=0) / prob.rho_b0
    phi = (a - b) / (a + b)
    zz = np.arange(prob.n_nodes) // (prob.nx * prob.ny)
    return (0.5 * (1.0 + phi))[zz >= z_lo].sum()


def test_rollout_gradients_checkpointed(torch, orc, orc_cs):
    """Gradients of J = red volume in a window after 23 steps, through
    rollout() with a checkpoint every 5 steps (ragged last segment), against
    complex step of the oracle through all 23 steps, and central differences of
    the FP64 oracle for dJ/dA (step 1e-4 A)."""
    from paper_1804_08923_amd.adjoint import rollout
    from paper_1804_08923_amd.lbm import LBM
    prob = _jet(12, 12, 16, D=5, noise=0.01)
    nsteps, every, z_lo = 23, 5, 6
    say("rollout gradients 12x12x16 jet, 23 steps, checkpoint every 5")
    st32, st64 = _state(orc, prob, seed=21)
    inlet = _inlet_profile(prob, 5)
    sim = LBM(prob, adjoint=True, inlet_uz=inlet)
    dev = sim.device
    x0 = torch.from_numpy(st32).to(dev).requires_grad_(True)
    A = torch.tensor(prob.A, dtype=torch.float64, device=dev, requires_grad=True)
    u_in = torch.from_numpy(inlet).to(dev).requires_grad_(True)
    xT = rollout(sim, x0, nsteps, every=every, A=A, u_in=u_in)
    nxy = prob.nx * prob.ny
    a = xT[:Q].sum(0) / prob.rho_r0
    b = xT[Q:].sum(0) / prob.rho_b0
    phi = (a - b) / (a + b)
    J = (0.5 * (1.0 + phi))[z_lo * nxy:].sum()
    J.backward()
    gx0 = x0.grad.cpu().numpy().astype(np.float64)
    gA = float(A.grad.item())
    gu = u_in.grad.cpu().numpy().astype(np.float64)
    sim.close()

    p = or_params(prob)

    def cs_run(v=None, dA=0.0, du=None):
        x = st64.astype(np.complex128) + (1j * H * v if v is not None else 0.0)
        fr, fb = np.ascontiguousarray(x[:Q]), np.ascontiguousarray(x[Q:])
        hist = np.ascontiguousarray(np.concatenate([fr[:, -nxy:], fb[:, -nxy:]]))
        iu = inlet.astype(np.complex128) + (1j * H * du if du is not None else 0.0)
        orc_cs.step(p, prob.A + 1j * H * dA, fr, fb, hist, 0, nsteps, inlet_uz=iu)
        return _objective_np(prob, fr, fb, z_lo).imag / H

    rA = cs_run(dA=1.0)
    say(f"  dJ/dA adjoint {gA:.9e} complex step {rA:.9e} rel {_rel(gA, rA):.2e}")
    assert _rel(gA, rA) < 1e-4
    # central differences of the FP64 oracle, h = 1e-4 A
    hA = 1e-4 * prob.A
    Js = []
    for sgn in (1.0, -1.0):
        x = st64.copy()
        fr, fb = np.ascontiguousarray(x[:Q]), np.ascontiguousarray(x[Q:])
        hist = np.ascontiguousarray(np.concatenate([fr[:, -nxy:], fb[:, -nxy:]]))
        orc.step(p, prob.A + sgn * hA, fr, fb, hist, 0, nsteps, inlet_uz=inlet.astype(np.float64))
        Js.append(_objective_np(prob, fr, fb, z_lo))
    fd = (Js[0] - Js[1]) / (2 * hA)
    say(f"  dJ/dA central difference {fd:.9e} rel {_rel(gA, fd):.2e}")
    assert _rel(gA, fd) < 1e-4
    rng = np.random.default_rng(31)
    e = rng.standard_normal(nxy)
    ru = cs_run(du=e)
    gu_e = (gu * e).sum()
    say(f"  dJ/du_in . e adjoint {gu_e:.9e} complex step {ru:.9e} rel {_rel(gu_e, ru):.2e}")
    assert _rel(gu_e, ru) < 1e-4
    v = rng.standard_normal(st64.shape)
    rx = cs_run(v=v)
    gx = (gx0 * v).sum()
    say(f"  dJ/dx0 . v adjoint {gx:.9e} complex step {rx:.9e} rel {_rel(gx, rx):.2e}")
    assert _rel(gx, rx) < 1e-4
