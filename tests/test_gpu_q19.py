"""Parity of the D3Q19 path (lbm_params.lattice = 19, through the C ABI) with
the D3Q19 build of the FP64 oracle (the reduced lattice of Sec. II, whose
coefficients the oracle's CPU pins tie to the D3Q27 moments).

Element-by-element comparisons of every population on seeded random states
(one step from the general form the state is handed over in, a second step
from the library's shifted form, ten steps), lattices of several 256-node
blocks with a ragged tail and lattices one node thick, the droplet of
Sec. III after 200 steps, Laplace's law on the 100^3 droplet of Table I at
gamma = 1, and the entry points D3Q19 does not implement.
"""
import numpy as np
import pytest

from harness import gpu_fields, rel_linf, say
from oracle import Oracle, make_params as or_params
from paper_1804_08923_amd.workloads import Problem

pytestmark = pytest.mark.gpu
Q19 = 19


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible ROCm device"
    return t


@pytest.fixture(scope="module")
def o19():
    return Oracle("q19")


def _prob(nx, ny, nz, **kw):
    base = dict(name="q19-rand", nx=nx, ny=ny, nz=nz, bc="periodic", rho_r0=1.0, rho_b0=0.5,
                nu_r=0.02, nu_b=0.05, A=2e-3, g=(1e-4, -2e-4, 3e-4), init="droplet", lattice=19,
                alpha_b=1.0 / 3.0)
    base.update(kw)
    return Problem(**base)


def _random_state(o19, prob, seed, noise=2e-4):
    """Random physical populations (FP64) from seeded fields plus noise, and
    the FP32 copy both sides start from."""
    from synth import population_noise, random_state_fields
    p = or_params(prob)
    rr, rb, u = random_state_fields(prob, seed)
    fr, fb, _ = o19.init_fields(p, rr, rb, u)
    nz = population_noise(prob.n_nodes, seed, amp=noise, q=Q19)
    fr += np.where(fr > 1e-3, nz[0], 0.0)
    fb += np.where(fb > 1e-3, nz[1], 0.0)
    st = np.concatenate([fr, fb], axis=0).astype(np.float32)
    return p, st


def _sim(prob, **kw):
    from paper_1804_08923_amd.lbm import LBM
    return LBM(prob, **kw)


def _gpu_state(sim):
    st = sim.get_state().cpu().numpy().astype(np.float64)
    return st[:Q19], st[Q19:]


@pytest.mark.parametrize("shape", [(16, 12, 10), (13, 7, 5), (300, 2, 3), (64, 32, 3), (43, 44, 2), (256, 3, 2),
                                   (512, 4, 3), (256, 8, 2), (256, 1, 1), (1, 1, 1), (1, 6, 4), (5, 1, 3), (3, 4, 1)])
def test_q19_steps_from_a_random_state(torch, o19, shape):
    """Steps 1, 2 and 10 from a random state (tau != 1, gamma = 2, eta != 1,
    g != 0), every population of both colours against the oracle: step 1
    reads the general form set_state writes, the later steps the shifted form
    the step writes.  300 x 2 planes are three 256-node blocks with a ragged
    tail; 64 x 32 and 43 x 44 planes are 8 blocks (the second with a ragged
    last one), which the kernels hand out in XCD bands, as 512 x 4 x 3 and
    256 x 8 x 2; rows of 256 and 512 nodes are the bench's row shape
    (256 x 1 x 1 with every neighbour row the same); one-node-thick axes make
    a node its own periodic neighbour.  (The random state of 512 x 4 x 2 is
    ill-conditioned: there the FP32 rounding of the stored state alone, with
    exact arithmetic, moves u by 4.5e-5 in 10 steps.)"""
    prob = _prob(*shape)
    say(f"D3Q19 random state {shape}")
    p, st = _random_state(o19, prob, seed=7 + sum(shape))
    fr64, fb64 = st[:Q19].astype(np.float64), st[Q19:].astype(np.float64)
    sim = _sim(prob)
    sim.set_state(torch.from_numpy(st).cuda(), t=0)
    # the state is taken over up to the FP32 rounding of d = f - w rho_b0: each
    # node keeps its minority colour exactly, the other is (d + w rho_b0) - f^k
    g0 = sim.get_state().cpu().numpy().astype(np.float64)
    scale = np.abs(fr64 + fb64).max()
    blue = fr64.sum(0) > fb64.sum(0)
    ek = np.where(blue, g0[Q19:] - fb64, g0[:Q19] - fr64)
    eo = np.where(blue, g0[:Q19] - fr64, g0[Q19:] - fb64)
    assert np.abs(ek).max() == 0.0
    assert np.abs(eo).max() <= 4 * 2.0 ** -23 * scale
    done = 0
    for upto, bar in ((1, 2e-6), (2, 3e-6), (10, 1e-5)):
        sim.step(upto - done)
        o19.step(p, prob.A, fr64, fb64, np.zeros((2 * Q19, p.nx * p.ny)), done, upto - done)
        done = upto
        gr, gb = _gpu_state(sim)
        err = max(np.abs(gr - fr64).max(), np.abs(gb - fb64).max()) / scale
        say(f"  step {upto}: max pop err {err:.2e}")
        assert err < bar, upto
    f = gpu_fields(sim)
    rr, rb, u, ph = o19.macroscopic(p, fr64, fb64)
    errs = {"rho": rel_linf(f["rho"], rr + rb), "u": rel_linf(f["u"], u), "phi": rel_linf(f["phi"], ph)}
    say(f"  step 10 fields rel Linf {errs}")
    # u sums 18 populations, each within ~1e-7 of the population scale, and
    # divides by a density near 0.5: up to ~1e-6 absolute against |u| of a few
    # 1e-2 on these small lattices (3 x 4 x 1 measures 1.04e-5)
    for k, e in errs.items():
        assert e < (5e-5 if k == "u" else 1e-5), k
    sim.close()


def _droplet(**kw):
    base = dict(name="q19-droplet-32", nx=32, ny=32, nz=32, bc="periodic", nu_r=1 / 6, nu_b=1 / 6, A=1e-3,
                drop_R=8.0, drop_W=2.0, steps=200, lattice=19, alpha_b=1.0 / 3.0)
    base.update(kw)
    return Problem(**base)


@pytest.mark.parametrize("kind", ["tau1", "cm"])
def test_q19_droplet_200_steps(torch, o19, kind):
    """The 32^3 droplet of Sec. III on D3Q19 (tau = 1, gamma = 1), and its
    tau != 1, gamma = 2, gravity variant, after 200 steps against the oracle:
    the initial state to 1e-6, then rho, u, phi and rho_r to the bars of the
    D3Q27 droplet parity (rel L-inf 1e-5; 5e-5 on u at tau ~ 0.53)."""
    prob = _droplet() if kind == "tau1" else _droplet(name="q19-droplet-32-cm", rho_b0=0.5, nu_r=0.01,
                                                       nu_b=0.03, g=(0.0, 0.0, 1e-5))
    say(f"D3Q19 droplet {prob.name}")
    sim = _sim(prob)
    p = or_params(prob)
    fr, fb, h = o19.init_droplet(p, prob.center, prob.drop_R, prob.drop_W)
    gr, gb = _gpu_state(sim)
    assert np.abs(gr - fr).max() < 1e-6 and np.abs(gb - fb).max() < 1e-6
    sim.step(prob.steps)
    fg = gpu_fields(sim)
    a0 = sim.macroscopic(audit=True)["audit"]
    sim.close()
    o19.step(p, prob.A, fr, fb, h, 0, prob.steps)
    rr, rb, u, ph = o19.macroscopic(p, fr, fb)
    fo = dict(rho=rr + rb, u=u, phi=ph, rho_r=rr)
    errs = {k: rel_linf(fg[k], fo[k]) for k in fo}
    say(f"  rel Linf {errs}")
    bars = {"rho": 1e-5, "u": 1e-5 if kind == "tau1" else 5e-5, "phi": 1e-5, "rho_r": 1e-5}
    for k, e in errs.items():
        assert e <= bars[k], k
    # the FP64 audit of the state against the oracle's colour masses
    assert abs(a0[0] / rr.sum() - 1) < 1e-6 and abs(a0[1] / rb.sum() - 1) < 1e-6


def test_q19_laplace_table1_gamma1(torch):
    """Laplace's law on D3Q19 for the Table I droplet (100^3, R = 25, W = 4,
    gamma = 1, tau = 1, A = 0.0008): dp = 2 sigma / R within 2 % of
    sigma = (4/9) A tau (Eq. sigma), pressure rho (1 - alpha_bar)/2 (the
    D3Q19 sound speed), after 100 000 steps; spurious currents below 1e-4."""
    from paper_1804_08923_amd.lbm import LBM
    prob = Problem(name="q19-table1-g1", nx=100, ny=100, nz=100, bc="periodic", rho_r0=1.0, rho_b0=1.0,
                   nu_r=1 / 6, nu_b=1 / 6, A=8e-4, drop_R=25.0, drop_W=4.0, init="droplet", lattice=19,
                   alpha_b=1.0 / 3.0)
    sim = LBM(prob)
    for s in range(0, 100_000, 25_000):
        sim.step(25_000)
        say(f"  {prob.name}: step {s + 25_000}")
    m = {k: v.detach().cpu().numpy().astype(np.float64) for k, v in sim.macroscopic().items()}
    sim.close()
    n = prob.nx
    phi = m["phi"]
    ab = (1 + phi) / 2 * prob.alpha_r + (1 - phi) / 2 * prob.alpha_b
    pres = (m["rho_r"] + m["rho_b"]) * (1 - ab) / 2
    Reff = (3.0 * ((1 + phi) / 2).sum() / (4.0 * np.pi)) ** (1.0 / 3.0)
    c = prob.center
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = [np.abs(a.ravel() - ci) for a, ci in ((x, c[0]), (y, c[1]), (z, c[2]))]
    r = np.sqrt(sum(np.minimum(di, n - di) ** 2 for di in d))
    dp = pres[r <= Reff - 5].mean() - pres[r >= Reff + 8].mean()
    sig, sig_th = dp * Reff / 2.0, 4.0 / 9.0 * prob.A * (3 * prob.nu_r + 0.5)
    umax = np.linalg.norm(m["u"], axis=1).max()
    E = abs(sig - sig_th) / sig_th
    say(f"  sigma {sig:.5e} vs {sig_th:.5e}: E {100 * E:.2f} %, R_eff {Reff:.2f}, |u|max {umax:.2e}")
    assert E < 0.02
    assert umax < 1e-4


def _q19_jet(name, nx, ny, nz, D, Re, We, steps, seed):
    from paper_1804_08923_amd.workloads import jet_problem
    return jet_problem(name, nx, ny, nz, D=D, u=0.04, gamma=2.0, eta=1.0, Re=Re, We=We, Fr=2.0, steps=steps,
                       noise_amp=0.01, noise_seed=seed).replace(lattice=19, alpha_b=1.0 / 3.0)


@pytest.mark.parametrize("steps", [1, 150])
def test_q19_small_jet(torch, o19, steps):
    """The jet boundaries on D3Q19 (inflow ghost with seeded noise, free-slip
    walls, convective outflow) and buoyancy on a 20x18x40 lattice from the
    all-blue start: fields to 1e-5 (rel L-inf), every population of both
    colours to 1e-5 of the population scale, and the FP64 audit against the
    oracle's colour masses.  Then the oracle's state at step s is handed over
    with lbm_set_state at time level s and both sides take 10 more steps (the
    inlet noise depends on the time level)."""
    prob = _q19_jet("q19-jet-small", 20, 18, 40, 8, 40.0, 20.0, 150, 7)
    say(f"D3Q19 small jet {steps} steps")
    sim = _sim(prob)
    sim.step(steps)
    fg = gpu_fields(sim)
    a0 = sim.macroscopic(audit=True)["audit"]
    p = or_params(prob)
    N = prob.n_nodes
    fr, fb, h = o19.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    o19.step(p, prob.A, fr, fb, h, 0, steps)
    rr, rb, u, ph = o19.macroscopic(p, fr, fb)
    fo = dict(rho=rr + rb, u=u, phi=ph, rho_r=rr)
    errs = {k: rel_linf(fg[k], fo[k]) for k in fo}
    say(f"  rel Linf {errs}")
    for k, e in errs.items():
        assert e <= 1e-5, k
    assert abs(a0[0] / rr.sum() - 1) < 1e-5 and abs(a0[1] / rb.sum() - 1) < 1e-6
    gr, gb = _gpu_state(sim)
    scale = np.abs(fr + fb).max()
    err = max(np.abs(gr - fr).max(), np.abs(gb - fb).max()) / scale
    say(f"  max pop err {err:.2e}")
    assert err < 1e-5
    # hand-over at time level `steps`
    st = np.concatenate([fr, fb], axis=0).astype(np.float32)
    fr, fb = st[:Q19].astype(np.float64), st[Q19:].astype(np.float64)
    sim.set_state(torch.from_numpy(st).cuda(), t=steps)
    sim.step(10)
    h = np.concatenate([fr, fb], axis=0)[:, (prob.nz - 1) * prob.nx * prob.ny:].copy()
    o19.step(p, prob.A, fr, fb, h, steps, 10)
    gr, gb = _gpu_state(sim)
    sim.close()
    err = max(np.abs(gr - fr).max(), np.abs(gb - fb).max()) / scale
    say(f"  after set_state at t = {steps} and 10 steps: max pop err {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("shape,D", [((3, 3, 3), 2.0), ((20, 5, 4), 3.0), ((64, 32, 6), 5.0)])
def test_q19_tiny_jets(torch, o19, shape, D):
    """The D3Q19 jet where almost every node is next to a wall, the inlet or
    the outlet (the 3x3x3 minimum), and on a 64x32 plane (8 blocks, in XCD
    bands): 30 steps against the oracle, every population."""
    prob = _q19_jet("q19-jet-tiny", *shape, D, 20.0, 10.0, 30, 5)
    say(f"D3Q19 tiny jet {shape} D={D}")
    sim = _sim(prob)
    sim.step(prob.steps)
    gr, gb = _gpu_state(sim)
    sim.close()
    p = or_params(prob)
    N = prob.n_nodes
    fr, fb, h = o19.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    o19.step(p, prob.A, fr, fb, h, 0, prob.steps)
    scale = np.abs(fr + fb).max()
    err = max(np.abs(gr - fr).max(), np.abs(gb - fb).max()) / scale
    say(f"  max pop err {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("case", ["blobs", "jet"])
def test_q19_jet_diagnostics(torch, case):
    """The jet diagnostics of Sec. IV C on D3Q19 handles against the CPU
    reference on the same order-parameter field (the GPU's own phi from
    lbm_macroscopic), exactly: seeded random blobs in the general form the
    fields preset writes (periodic, 33 x 65 x 17), and a D3Q19 jet after 300
    steps in the shifted form; the static-workspace entry point agrees."""
    from oracle.diagnostics import jet_diagnostics
    from synth import sphere_blobs

    from paper_1804_08923_amd.lbm import LBM
    if case == "blobs":
        nx, ny, nz = 33, 65, 17
        phi = sphere_blobs(nx, ny, nz, 3, 150)
        prob = _prob(nx, ny, nz, init="fields", inlet_cx=(nx - 1) / 2, inlet_cy=(ny - 1) / 2, inlet_D=4.0)
        rr = (prob.rho_r0 * (1 + phi) / 2).astype(np.float32)
        rb = (prob.rho_b0 * (1 - phi) / 2).astype(np.float32)
        sim = LBM(prob, rho_r=torch.from_numpy(rr), rho_b=torch.from_numpy(rb))
    else:
        prob = _q19_jet("q19-jet-diag", 32, 30, 64, 10, 200.0, 20.0, 300, 9)
        sim = LBM(prob)
        sim.step(300)
    stats, vol = sim.jet_diagnostics()
    phi = sim.macroscopic()["phi"].cpu().numpy()
    ref, rvol = jet_diagnostics(phi, prob.nx, prob.ny, prob.nz)
    say(f"  D3Q19 {case}: {stats}, {len(vol)} fragments")
    assert stats == ref and np.array_equal(vol, rvol)
    assert stats["jet_nodes"] > 100
    s2, v2 = sim.jet_diagnostics_static(len(vol) + 1)
    assert s2 == stats and np.array_equal(v2, vol)
    sim.close()


def test_q19_unsupported_entry_points(torch):
    """Snapshots and the adjoint step need the D3Q27 lattice: each returns
    LBM_ERR_UNSUPPORTED on a D3Q19 handle and leaves it usable."""
    from paper_1804_08923_amd.lbm import LbmError
    prob = _prob(8, 8, 8)
    sim = _sim(prob)
    snap = torch.empty(256, dtype=torch.uint8, device="cuda")
    for call in (lambda: sim.step_to_snapshot(snap), lambda: sim.save_snapshot(snap),
                 lambda: sim.load_snapshot(snap, 0)):
        with pytest.raises(LbmError) as ei:
            call()
        assert ei.value.code == -2
    st = sim.get_state()
    lam = torch.zeros_like(st)
    dA = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(LbmError) as ei:
        sim.adjoint_step(st, 0, lam, torch.empty_like(st), dA)
    assert ei.value.code == -2
    sim.step(3)
    assert sim.time == 3
    sim.close()
