"""Pins of the oracle's jet boundaries (Sec. IV A) on the CPU.

The paper describes the jet boundaries in words only: a circular inlet with
uniform inflow and the corresponding equilibria, free-slip side walls and
bottom, and the convective outflow of Lou et al. at the top, with U_c the
axial velocity of the plane below the outlet.  The oracle's discrete reading
(half-way specular reflection, an inlet ghost plane holding the red
equilibrium, the convective rule applied to all populations after streaming)
is checked here against consequences that do not come from the oracle's own
code:

* free slip: by the method of images.  A half-way specular wall is equivalent
  to a periodic lattice twice as long holding the mirror image of the state,
  so the jet lattice with a closed inlet must evolve exactly like that
  periodic lattice (which the periodic pins cover) wherever the outlet has
  not yet had an influence.  A reflection that reverses the wrong components,
  drops the tangential shift, or mirrors the wrong ghost field fails this.
* inlet: closed forms of the inflow.  Over one step from an all-blue start the
  only red populations are the ones streamed out of the inlet ghost cells, so
  the red mass and momentum equal lattice sums of the inlet equilibrium
  (derived below from the D3Q27 moments), including the radial noise at the
  given time level and a per-cell inflow profile.
* the inlet face: over the same step the blue mass falls by exactly the
  post-collision blue populations that stream from the nodes above inlet
  cells into the inlet, with the gradient the ghost field phi = +1 of the
  inlet cells drives.
* fixed points: red fluid at rest with an inlet at rest is steady (the inlet
  ghosts then equal the mirror image: red equilibrium at rho_r0 with
  alpha_r, ghost fields phi = 1 and rho = rho_r0); a blue lattice at rest
  under gravity with a closed inlet is steady.
* the outlet: the new outlet plane is the convex combination of its previous
  value and the freshly streamed plane below, weighted by lambda = max(0, u_z)
  of that streamed plane at the new time level.
* symmetry: a noise-free jet on a square cross-section keeps the symmetries of
  the square (x -> nx-1-x, y -> ny-1-y, x <-> y), which fixes the inlet centre.

Every pin runs on the D3Q27 oracle and on its D3Q19 build (the boundary code
is the same; the closed forms take each lattice's sums).
"""
import numpy as np
import pytest

from oracle import Oracle, make_params
from paper_1804_08923_amd.workloads import Problem


@pytest.fixture(scope="module", params=["f64", "q19"])
def orc(request):
    return Oracle(request.param)


@pytest.fixture(scope="module")
def lat(orc):
    c, w = orc.lattice()
    return c.astype(np.int64), w


def _mirror_table(c):
    """mirror[i, m]: direction i with the components in mask m (bit 0 x, 1 y, 2 z) reversed."""
    Q = len(c)
    idx = {tuple(v): i for i, v in enumerate(c)}
    out = np.zeros((Q, 8), np.int64)
    for i in range(Q):
        for m in range(8):
            s = np.array([-1 if (m >> a) & 1 else 1 for a in range(3)])
            out[i, m] = idx[tuple(c[i] * s)]
    return out


def _jet(nx, ny, nz, **kw):
    base = dict(name="jetbc", nx=nx, ny=ny, nz=nz, bc="jet", rho_r0=1.0, rho_b0=0.5,
                nu_r=0.02, nu_b=0.03, A=2e-3, g=(0.0, 0.0, 0.0), inlet_cx=(nx - 1) / 2, inlet_cy=(ny - 1) / 2,
                inlet_D=0.0, inlet_u=0.05, noise_amp=0.0, noise_seed=0, init="jet")
    base.update(kw)
    return Problem(**base)


def _grid(p):
    z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def _kappa(alpha, w0):
    """varphi_i(alpha) = w_i kappa(alpha) for |c_i| >= 1 (Eq. varphi_ik):
    kappa = (1 - alpha)/(1 - w_0), 27 (1 - alpha)/19 on D3Q27."""
    return (1.0 - alpha) / (1.0 - w0)


# ---------------------------------------------------------------- free slip
def _smooth_state(orc, prob, seed):
    """A two-colour state with interfaces and a flow, concentrated near the
    bottom corner (x, y, z small) so that the walls there carry traffic."""
    p = make_params(prob)
    x, y, z = _grid(prob)
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(0.5, 2.5, 3)
    r = np.sqrt((x - c0[0]) ** 2 + (y - c0[1]) ** 2 + (z - c0[2]) ** 2)
    phi = -np.tanh((r - 3.0) / 1.2)
    rho_r = prob.rho_r0 * (1 + phi) / 2 * (1 + 0.01 * rng.standard_normal(x.size))
    rho_b = prob.rho_b0 * (1 - phi) / 2 * (1 + 0.01 * rng.standard_normal(x.size))
    k = rng.uniform(0.3, 0.9, (3, 3))
    u = np.stack([0.03 * np.cos(k[a, 0] * x + 0.7 * a) * np.sin(k[a, 1] * y + 0.3) * np.cos(k[a, 2] * z - 0.2 * a)
                  for a in range(3)], axis=1)
    fr, fb, h = orc.init_fields(p, rho_r, rho_b, u)
    return p, fr, fb, h


@pytest.mark.parametrize("dims,seed", [((6, 5, 20), 1), ((5, 7, 20), 2)])
def test_free_slip_equals_mirror_image(orc, lat, dims, seed):
    """Free-slip walls (x = -1/2, x = nx - 1/2, the same in y, z = -1/2 with no
    inlet) by the method of images: the jet lattice evolves like the periodic
    lattice of 2nx x 2ny x 2nz holding the mirrored state, up to the planes
    the convective outlet has reached (two planes per step)."""
    c, _ = lat
    Q = len(c)
    mir = _mirror_table(c)
    nx, ny, nz = dims
    prob = _jet(nx, ny, nz)
    p, fr, fb, h = _smooth_state(orc, prob, seed)
    per = prob.replace(nx=2 * nx, ny=2 * ny, nz=2 * nz, bc="periodic")
    pp = make_params(per)
    X, Y, Z = _grid(per)
    mx, my, mz = X >= nx, Y >= ny, Z >= nz
    xs = np.where(mx, 2 * nx - 1 - X, X)
    ys = np.where(my, 2 * ny - 1 - Y, Y)
    zs = np.where(mz, 2 * nz - 1 - Z, Z)
    src = (zs * ny + ys) * nx + xs
    m = mx.astype(int) | (my.astype(int) << 1) | (mz.astype(int) << 2)
    Fr = np.empty((Q, X.size))
    Fb = np.empty((Q, X.size))
    for i in range(Q):
        Fr[i] = fr[mir[i, m], src]
        Fb[i] = fb[mir[i, m], src]
    Hp = np.zeros((2 * Q, (2 * nx) * (2 * ny)))
    fr0 = fr.copy()
    T = 5
    orc.step(p, prob.A, fr, fb, h, 0, T)
    orc.step(pp, prob.A, Fr, Fb, Hp, 0, T)
    keep = Z <= nz - 2 * T
    inside = keep & ~mx & ~my & ~mz
    jet_idx = (Z[inside] * ny + Y[inside]) * nx + X[inside]
    scale = np.abs(fr).max() + np.abs(fb).max()
    assert np.abs(fr[:, jet_idx] - Fr[:, inside]).max() < 1e-13 * scale
    assert np.abs(fb[:, jet_idx] - Fb[:, inside]).max() < 1e-13 * scale
    # and the state moved: the comparison is not between two untouched states
    assert np.abs(fr[:, jet_idx] - fr0[:, jet_idx]).max() > 1e-4


def test_closed_inlet_rest_is_fixed_point_under_gravity(orc):
    """All-blue lattice at rest with no inlet cell: the body force
    (rho - rho_b0) g vanishes, the walls reflect a symmetric state and the
    outlet sees lambda = 0, so nothing changes."""
    prob = _jet(7, 6, 9, g=(0.0, 0.0, 1e-5))
    p = make_params(prob)
    N = prob.n_nodes
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    f0 = fb.copy()
    orc.step(p, prob.A, fr, fb, h, 0, 20)
    assert np.abs(fr).max() == 0.0
    assert np.abs(fb - f0).max() < 1e-15


# ---------------------------------------------------------------- inlet
def test_red_rest_with_resting_inlet_is_fixed_point(orc):
    """Red fluid at rest everywhere and an inlet at rest (u_in = 0, no noise):
    the inlet ghosts then hold the mirror image of the red rest state (red
    equilibrium at rho_r0 with alpha_r, ghost fields phi = 1, rho = rho_r0), so
    nothing changes.  A blue ghost, the blue alpha or the blue density fails."""
    prob = _jet(9, 8, 7, inlet_D=5.0, inlet_u=0.0)
    p = make_params(prob)
    N = prob.n_nodes
    fr, fb, h = orc.init_fields(p, np.full(N, prob.rho_r0), np.zeros(N))
    f0 = fr.copy()
    orc.step(p, prob.A, fr, fb, h, 0, 10)
    assert np.abs(fb).max() == 0.0
    assert np.abs(fr - f0).max() < 1e-15


def test_first_step_blue_loss_through_inlet_face(orc, lat):
    """Mass budget of the first step from an all-blue lattice at rest: the
    walls and the quiescent outlet conserve mass, so the blue mass falls by
    exactly the post-collision blue populations that stream from the nodes
    above inlet cells into the inlet (each ghost cell below such a node holds
    inlet fluid, not the node's mirror image).  Those populations are the
    blue rest equilibrium plus the perturbation (Eq. perturb) driven by the
    gradient of phi at z = 0, where the ghost cells of the inlet carry
    phi = +1 and every other ghost cell mirrors phi = -1:
        grad phi = 3 sum_i w_i phi(x + c_i) c_i = 6 sum_{i: c_z = -1, x + c_i in inlet} w_i c_i."""
    c, w = lat
    Q = len(c)
    prob = _jet(12, 11, 8, inlet_D=6.0, inlet_u=0.05, noise_amp=0.2, noise_seed=5, A=5e-3)
    p = make_params(prob)
    N = prob.n_nodes
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    mb0 = fb.sum()
    orc.step(p, prob.A, fr, fb, h, 0, 1)

    def inside(x, y):
        if not (0 <= x < prob.nx and 0 <= y < prob.ny):
            return False
        dx, dy = x - prob.inlet_cx, y - prob.inlet_cy
        return dx * dx + dy * dy < 0.25 * prob.inlet_D ** 2

    down = [i for i in range(Q) if c[i, 2] == -1]
    ph_b = orc.phi_coeffs(prob.alpha_b)
    lost = 0.0
    n_in = 0
    for y in range(prob.ny):
        for x in range(prob.nx):
            if not inside(x, y):
                continue
            n_in += 1
            g = 6.0 * sum(w[i] * c[i] for i in down if inside(x + c[i, 0], y + c[i, 1]))
            post = prob.rho_b0 * ph_b + orc.perturb(p, prob.A, g)
            lost += post[down].sum()
    assert n_in > 20
    assert abs((mb0 - fb.sum()) - lost) < 1e-14 * mb0
    # the perturbation part of the loss is visible at this tolerance
    rest_only = n_in * prob.rho_b0 * ph_b[down].sum()
    assert abs(lost - rest_only) > 1e-6


def _inflow_closed_forms(prob, orc, t, lat, inlet_uz=None):
    """Red mass and momentum streamed out of the inlet ghost plane in one step.

    Each ghost cell holds f^e_i = rho_r0 [varphi_i(alpha_r) + w_i P_i(u)] and
    sends its c_z = +1 populations (nine on D3Q27, five on D3Q19) to z = 0.
    With the indicator [c_z = 1] = (c_z + c_z^2)/2 and the lattice sums
    sum w c_a^2 = sum w c_a^4 = 1/3, sum w c_a^2 c_b^2 = sum w c_a^4 c_b^2 = 1/9
    (both lattices) and s = sum w c_x^2 c_y^2 c_z^2 (1/27 on D3Q27, 0 on D3Q19),
    the moments of the equilibrium give per cell
        mass = z-momentum = (rho_r0/2) (kappa_r/3 + u_z + u_z^2),
        x-momentum = (rho_r0 u_x/2) (1/3 + u_z + u_z^2 + 13.5 (s - 1/27) u_y^2)
        (y alike with u_x^2), kappa_r = (1 - alpha_r)/(1 - w_0), independent of
    the radial part of u except through u_x, u_y themselves."""
    nx, ny = prob.nx, prob.ny
    c, w = lat
    kap = _kappa(prob.alpha_r, w[0])
    s = float((w * c[:, 0] ** 2 * c[:, 1] ** 2 * c[:, 2] ** 2).sum())
    mass = 0.0
    mom = np.zeros(3)
    for y in range(ny):
        for x in range(nx):
            dx, dy = x - prob.inlet_cx, y - prob.inlet_cy
            if not dx * dx + dy * dy < 0.25 * prob.inlet_D ** 2:
                continue
            r = np.hypot(dx, dy)
            ur = prob.noise_amp * prob.inlet_u * orc.noise(prob.noise_seed, t, x, y, nx, ny)
            ux = ur * dx / r if r > 0 else 0.0
            uy = ur * dy / r if r > 0 else 0.0
            uz = prob.inlet_u if inlet_uz is None else inlet_uz[y * nx + x]
            m = 0.5 * prob.rho_r0 * (kap / 3 + uz + uz * uz)
            mass += m
            mom += [0.5 * prob.rho_r0 * ux * (1 / 3 + uz + uz * uz + 13.5 * (s - 1 / 27) * uy * uy),
                    0.5 * prob.rho_r0 * uy * (1 / 3 + uz + uz * uz + 13.5 * (s - 1 / 27) * ux * ux), m]
    return mass, mom


@pytest.mark.parametrize("t0,profile", [(0, False), (7, False), (3, True)])
def test_first_step_red_inflow_matches_closed_forms(orc, lat, t0, profile):
    """All-blue start: after one step every red population came out of an inlet
    ghost cell, so the red mass and momentum equal the closed forms, with the
    radial noise of time level t0 (and a per-cell axial profile when given)."""
    c, _ = lat
    prob = _jet(14, 13, 6, inlet_D=7.0, inlet_u=0.05, noise_amp=0.3, noise_seed=99, g=(0.0, 0.0, 1e-5))
    p = make_params(prob)
    N = prob.n_nodes
    iu = None
    if profile:
        iu = np.random.default_rng(4).uniform(0.02, 0.08, prob.nx * prob.ny)
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    orc.step(p, prob.A, fr, fb, h, t0, 1, inlet_uz=iu)
    m_exp, mom_exp = _inflow_closed_forms(prob, orc, t0, lat, iu)
    assert m_exp > 0 and np.abs(mom_exp[:2]).max() > 1e-4 * m_exp
    assert abs(fr.sum() - m_exp) < 1e-13 * m_exp
    mom = np.array([(fr * c[:, a][:, None]).sum() for a in range(3)])
    assert np.abs(mom - mom_exp).max() < 1e-13 * m_exp
    # the red is all in plane z = 0
    x, y, z = _grid(prob)
    assert np.abs(fr[:, z > 0]).max() == 0.0
    # another time level draws other noise
    m2, mom2 = _inflow_closed_forms(prob, orc, t0 + 1, lat, iu)
    assert np.abs(mom2[:2] - mom_exp[:2]).max() > 1e-3 * np.abs(mom_exp[:2]).max()


# ---------------------------------------------------------------- outlet
def test_outlet_convective_rule_at_new_time_level(orc, lat):
    """Top plane after a step = [its previous value + lam f(nz-2, t+1)]/(1 + lam)
    for both colours, lam = max(0, u_z) of the freshly streamed plane below
    (u_z with the half-force term, Eq. Momentum).  The state is chosen so that
    u_z below the outlet changes sign and size between t and t + 1, so the
    time level matters."""
    c, _ = lat
    nx, ny, nz = 6, 5, 6
    prob = _jet(nx, ny, nz, g=(0.0, 0.0, 2e-4), rho_b0=0.5)
    p = make_params(prob)
    x, y, z = _grid(prob)
    rng = np.random.default_rng(11)
    phi = np.tanh(2.0 * np.sin(0.9 * x + 0.4 * y) * np.cos(0.7 * z))
    rho_r = prob.rho_r0 * (1 + phi) / 2
    rho_b = prob.rho_b0 * (1 - phi) / 2
    u = np.zeros((x.size, 3))
    u[:, 2] = 0.04 * np.sin(1.3 * z + 0.5 * x) + 0.01 * rng.standard_normal(x.size)
    u[:, 0] = 0.02 * np.cos(0.8 * y)
    fr, fb, h = orc.init_fields(p, rho_r, rho_b, u)
    P = nx * ny
    top = slice((nz - 1) * P, nz * P)
    below = slice((nz - 2) * P, (nz - 1) * P)
    hr0, hb0 = fr[:, top].copy(), fb[:, top].copy()

    def uz_of(fr_, fb_):
        f = fr_[:, below] + fb_[:, below]
        rho = f.sum(axis=0)
        return ((f * c[:, 2][:, None]).sum(axis=0) + 0.5 * (rho - prob.rho_b0) * prob.g[2]) / rho

    uz_t = uz_of(fr, fb)
    orc.step(p, prob.A, fr, fb, h, 0, 1)
    uz_t1 = uz_of(fr, fb)
    lam = np.maximum(uz_t1, 0.0)
    exp_r = (hr0 + lam * fr[:, below]) / (1 + lam)
    exp_b = (hb0 + lam * fb[:, below]) / (1 + lam)
    assert np.abs(fr[:, top] - exp_r).max() < 1e-15
    assert np.abs(fb[:, top] - exp_b).max() < 1e-15
    # the history holds the new outlet plane (red then blue)
    Q = len(c)
    assert np.array_equal(h[:Q], fr[:, top]) and np.array_equal(h[Q:], fb[:, top])
    # lambda at time t would have given a different plane: the test discriminates
    lam_t = np.maximum(uz_t, 0.0)
    alt = (hr0 + lam_t * fr[:, below]) / (1 + lam_t)
    assert np.abs(alt - exp_r).max() > 1e-5
    assert (uz_t1 < 0).any() and (uz_t1 > 0).any()


# ---------------------------------------------------------------- symmetry
def test_noise_free_jet_keeps_square_symmetry(orc):
    """Centred inlet (x_c = (nx-1)/2) on a square cross-section, no noise: the
    fields keep the x and y reflections and the x <-> y swap."""
    n, nz = 12, 10
    prob = _jet(n, n, nz, inlet_D=6.0, inlet_u=0.06, g=(0.0, 0.0, 1e-5))
    p = make_params(prob)
    N = prob.n_nodes
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    orc.step(p, prob.A, fr, fb, h, 0, 25)
    rr, rb, u, ph = orc.macroscopic(p, fr, fb)
    sh = (nz, n, n)
    R, PH = (rr + rb).reshape(sh), ph.reshape(sh)
    UX, UY, UZ = (u[:, a].reshape(sh) for a in range(3))
    assert rr.sum() > 1.0 and np.abs(UZ).max() > 0.02
    tol = 1e-12
    for F in (R, PH, UZ):
        assert np.abs(F - F[:, :, ::-1]).max() < tol
        assert np.abs(F - F[:, ::-1, :]).max() < tol
        assert np.abs(F - F.transpose(0, 2, 1)).max() < tol
    assert np.abs(UX + UX[:, :, ::-1]).max() < tol and np.abs(UX - UX[:, ::-1, :]).max() < tol
    assert np.abs(UY + UY[:, ::-1, :]).max() < tol
    assert np.abs(UX - UY.transpose(0, 2, 1)).max() < tol
    # an off-centre inlet breaks the x reflection
    q = make_params(prob.replace(inlet_cx=n / 2))
    fr, fb, h = orc.init_fields(q, np.zeros(N), np.full(N, prob.rho_b0))
    orc.step(q, prob.A, fr, fb, h, 0, 5)
    rr2 = orc.macroscopic(q, fr, fb)[0].reshape(sh)
    assert np.abs(rr2 - rr2[:, :, ::-1]).max() > 1e-3
