"""Static droplet tests of Sec. III (Table I) on the HIP path.

100^3 periodic box, a red droplet of radius R = 25 with a tanh interface of
width W = 4 in blue fluid, nu = 1/6 in both phases (tau = 1), no gravity,
100 000 steps, density ratios gamma = 1, 10, 100, 1000.  The pressure of each
phase is Eq. press, p = rho 9 (1 - alpha_bar) / 19, averaged inside and
outside the droplet away from the interface; Laplace's law in three
dimensions, Eq. lap, gives sigma_Lap = dp R / 2, compared with Eq. sigma,
sigma_th = (4/9) A tau.

The perturbation strength: Table I prints sigma_th = 3.5556e-4 for every row,
which with tau = 1 is Eq. sigma at A = 8e-4; the text of Sec. III states
A = 0.01, which would give 4.44e-3.  The sweep runs at A = 8e-4 so that the
printed sigma_th and spurious velocities are comparable; one case runs at the
stated A = 0.01.  Bars: |E| <= 2 % (the paper reaches 0.40 %) and a maximum
spurious velocity within 4x of the value Table I prints.

The rows gamma = 100 and 1000 start from a different state (a reading):
with alpha_bar linear in phi (Sec. II) the printed tanh densities put a
pressure of order gamma/4 times the bulk value into the interface, and the
method as printed does not survive the resulting transient -- the FP64
oracle itself turns non-finite within 20 steps (40^3, R = 10, gamma = 100).
Those rows keep the tanh order parameter but scale both colour densities so
that the pressure of Eq. press is the bulk value everywhere
(rho_k = rho_k0 s (1 +- phi)/2, s = 1 in the pure phases); the oracle's
behaviour from that start is pinned on the CPU (test_oracle_laplace), and
the GPU path is checked against the oracle from it below.  The printed
start at those ratios stays here as a strict expected failure.
"""
import numpy as np
import pytest

from golden_io import laplace_table
from harness import say
from paper_1804_08923_amd.workloads import Problem

pytestmark = pytest.mark.gpu

STEPS = 100_000
CHUNK = 20_000


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible ROCm device"
    return t


def _droplet(gamma, A):
    return Problem(name=f"table1-g{gamma:g}", nx=100, ny=100, nz=100, bc="periodic", rho_r0=1.0,
                   rho_b0=1.0 / gamma, nu_r=1 / 6, nu_b=1 / 6, A=A, drop_R=25.0, drop_W=4.0, init="droplet",
                   steps=STEPS)


def _balanced_fields(prob):
    """The pressure-balanced start of the droplet prob describes (host FP64,
    handed to the library as FP32 fields)."""
    from synth import droplet_profile
    from test_oracle_laplace import balanced_densities
    phi = droplet_profile(prob.nx, prob.drop_R, prob.drop_W, center=prob.center[0])
    rr, rb = balanced_densities(prob, phi)
    return rr.astype(np.float32), rb.astype(np.float32)


def _laplace(prob, f):
    """sigma_Lap, effective radius and max |u| from GPU fields (FP64 host math)."""
    n = prob.nx
    phi = f["phi"].astype(np.float64)
    rho = f["rho_r"].astype(np.float64) + f["rho_b"].astype(np.float64)
    ab = (1 + phi) / 2 * prob.alpha_r + (1 - phi) / 2 * prob.alpha_b
    pres = rho * 9.0 * (1.0 - ab) / 19.0                       # Eq. press
    Reff = (3.0 * ((1 + phi) / 2).sum() / (4.0 * np.pi)) ** (1.0 / 3.0)
    c = prob.center
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = [np.abs(a.ravel() - ci) for a, ci in ((x, c[0]), (y, c[1]), (z, c[2]))]
    r = np.sqrt(sum(np.minimum(di, n - di) ** 2 for di in d))  # periodic images
    dp = pres[r <= Reff - 5].mean() - pres[r >= Reff + 8].mean()
    un = np.linalg.norm(f["u"].astype(np.float64), axis=1)
    umax = un.max()
    say(f"  |u|max by region: red (phi > 0.9) {un[phi > 0.9].max():.3e}, interface {un[np.abs(phi) <= 0.9].max():.3e}, "
        f"blue (phi < -0.9) {un[phi < -0.9].max():.3e}")
    return dp * Reff / 2.0, Reff, umax


def _run(torch, prob, balanced=False):
    from paper_1804_08923_amd.lbm import LBM
    if balanced:
        rr, rb = _balanced_fields(prob)
        sim = LBM(prob.replace(init="fields"), rho_r=rr, rho_b=rb)
    else:
        sim = LBM(prob)
    for s in range(0, STEPS, CHUNK):
        sim.step(CHUNK)
        m = sim.macroscopic()
        f = {k: v.detach().cpu().numpy() for k, v in m.items()}
        finite = bool(np.isfinite(f["phi"]).all() and np.isfinite(f["u"]).all())
        say(f"  {prob.name}: step {s + CHUNK}{'' if finite else ': non-finite'}")
        if not finite:
            sim.close()
            raise AssertionError(f"{prob.name}: non-finite fields by step {s + CHUNK}")
    sim.close()
    return f


_ROWS = {}


def _table_row(torch, row, balanced):
    """Run Table I row `row` once per process (cached): sigma_Lap, E, |u|max."""
    key = (row, balanced)
    if key in _ROWS:
        return _ROWS[key]
    gamma, sig_tab, sig_lap_tab, e_tab, umax_tab = laplace_table()[row]
    tau = 3 * (1 / 6) + 0.5
    A = 8e-4
    sig_th = 4.0 / 9.0 * A * tau
    assert abs(sig_th - sig_tab) < 1e-8                          # the row's sigma_th
    prob = _droplet(gamma, A)
    say(f"Table I droplet gamma = {gamma:g}: 100^3, R = 25, W = 4, A = {A}, {STEPS} steps, "
        f"{'pressure-balanced' if balanced else 'tanh'} start")
    f = _run(torch, prob, balanced)
    sig, Reff, umax = _laplace(prob, f)
    E = 100.0 * abs(sig - sig_th) / sig_th
    say(f"  sigma_Lap {sig:.5e} (paper {sig_lap_tab:.5e}), sigma_th {sig_th:.5e}, E {E:.2f} % "
        f"(paper {e_tab:.2f} %), R_eff {Reff:.2f}, |u|max {umax:.3e} (paper {umax_tab:.2e})")
    _ROWS[key] = (E, umax, umax_tab)
    return _ROWS[key]


@pytest.mark.parametrize("row,balanced", [(0, False), (1, False), (2, True), (3, True)])
def test_table1_droplet(torch, row, balanced):
    """sigma_Lap within 2 % of Eq. sigma for every row; for gamma = 1 and 10
    also the spurious velocity within 4x of the printed value."""
    E, umax, umax_tab = _table_row(torch, row, balanced)
    assert E <= 2.0
    if row < 2:
        assert umax <= 4.0 * umax_tab


@pytest.mark.xfail(reason="at gamma >= 100 the interface carries spurious currents 20-130x the printed ones",
                   strict=True)
@pytest.mark.parametrize("row", [2, 3])
def test_table1_spurious_velocity_high_gamma(torch, row):
    E, umax, umax_tab = _table_row(torch, row, True)
    assert umax <= 4.0 * umax_tab


@pytest.mark.xfail(reason="the method as printed diverges from the tanh start at gamma = 100 "
                          "(so does the FP64 oracle)", strict=True)
def test_table1_tanh_start_gamma_100(torch):
    _table_row(torch, 2, False)


def test_droplet_stated_A(torch):
    """gamma = 1 at the A = 0.01 of the text: sigma_th = 4.44e-3."""
    A = 0.01
    prob = _droplet(1.0, A)
    sig_th = 4.0 / 9.0 * A * 1.0
    say(f"droplet gamma = 1, A = {A}: {STEPS} steps")
    f = _run(torch, prob)
    sig, Reff, umax = _laplace(prob, f)
    E = 100.0 * abs(sig - sig_th) / sig_th
    say(f"  sigma_Lap {sig:.5e}, sigma_th {sig_th:.5e}, E {E:.2f} %, R_eff {Reff:.2f}, |u|max {umax:.3e}")
    assert E <= 2.0


@pytest.mark.parametrize("gamma,balanced", [(30.0, False), (100.0, False), (100.0, True), (1000.0, True)])
def test_high_density_ratio_parity(torch, orc, gamma, balanced):
    """The start-up transient of a high-density-ratio droplet (24^3, R = 6,
    W = 4, A = 8e-4), 100 steps, against the FP64 oracle, from the tanh
    start (where the oracle survives it) and from the pressure-balanced start
    the Table I rows at gamma >= 100 use: the GPU path follows the method.  Bar 2e-5: the FP32 instantiation of the
    plain scheme itself moves u by 7.5e-6 and rho by 1e-6 on the gamma = 100
    case.  Where the dense colour dominates, the blue fraction is kept to its
    own relative precision; keeping the red fraction instead gave 2e-4."""
    from harness import gpu_fields, oracle_fields, oracle_init, rel_linf
    from oracle import make_params as or_params
    from paper_1804_08923_amd.lbm import LBM
    prob = Problem(name=f"drop24-g{gamma:g}", nx=24, ny=24, nz=24, bc="periodic", rho_r0=1.0,
                   rho_b0=1.0 / gamma, nu_r=1 / 6, nu_b=1 / 6, A=8e-4, drop_R=6.0, drop_W=4.0, init="droplet",
                   steps=100)
    if balanced:
        rr, rb = _balanced_fields(prob)
        prob = prob.replace(init="fields")
        sim = LBM(prob, rho_r=rr, rho_b=rb)
        p = or_params(prob)
        fr, fb, h = orc.init_fields(p, rr.astype(np.float64), rb.astype(np.float64))
    else:
        sim = LBM(prob)
        p, fr, fb, h = oracle_init(orc, prob)
    sim.step(prob.steps)
    fg = gpu_fields(sim)
    sim.close()
    orc.step(p, prob.A, fr, fb, h, 0, prob.steps)
    fo = oracle_fields(orc, p, fr, fb)
    errs = {k: rel_linf(fg[k], fo[k]) for k in ("rho", "u", "phi", "rho_r", "rho_b")}
    umax = np.linalg.norm(fo["u"], axis=1).max()
    say(f"  gamma {gamma:g} ({'balanced' if balanced else 'tanh'} start): |u|max {umax:.3e}, rel Linf {errs}")
    for k, e in errs.items():
        assert e <= 2e-5, k
