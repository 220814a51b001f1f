"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  Values printed in the paper live in
tests/golden/ (Appendix A matrices, Table I).  None of these tests needs a GPU.
"""
import itertools
import math

import numpy as np
import pytest

from golden_io import int_matrix, poly_matrix
from oracle import make_params
from paper_1804_08923_amd.workloads import Problem

Q = 27


@pytest.fixture(scope="module")
def lat(orc):
    c, w = orc.lattice()
    return c.astype(np.float64), w


def _prob(**kw):
    base = dict(name="t", nx=4, ny=4, nz=4, bc="periodic", rho_r0=1.0, rho_b0=0.5,
                nu_r=0.02, nu_b=0.05, A=1e-3, g=(0.0, 0.0, 0.0))
    base.update(kw)
    return Problem(**base)


# ---------------------------------------------------------------- lattice
def test_lattice_is_d3q27_with_paper_weights(lat):
    """Eq. velVec / weights: 27 distinct velocities in {-1,0,1}^3, weights by |c|^2,
    and the isotropy of the even lattice tensors up to fourth order."""
    c, w = lat
    assert len({tuple(v) for v in c.astype(int)}) == 27
    assert np.allclose(w.sum(), 1.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-15)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-15)
    # odd moments vanish
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    # the paper's ordering pairs i (odd) with its opposite i+1
    for i in range(1, 27, 2):
        assert np.array_equal(c[i], -c[i + 1])


# ---------------------------------------------------------------- Appendix A
def test_M_equals_appendix(orc):
    """Eq. (M): the oracle's raw-moment matrix T(0) equals the printed M."""
    M = orc.moment_matrix([0.0, 0.0, 0.0])
    assert np.array_equal(M, int_matrix("appA_M.txt"))


def test_Minv_equals_appendix(orc):
    """Appendix A: inverse of M equals the printed (1/48) x integer matrix."""
    M = orc.moment_matrix([0.0, 0.0, 0.0])
    Mi = orc.invert(M)
    assert np.abs(Mi * 48 - int_matrix("appA_Minv.txt")).max() < 1e-12
    assert np.array_equal(M @ int_matrix("appA_Minv.txt"), 48 * np.eye(Q))


@pytest.mark.parametrize("seed", range(5))
def test_shift_matrix_equals_appendix(orc, seed):
    """Appendix A: N(u) = T(u) M^-1 equals the printed N, and its inverse the printed N^-1."""
    u = np.random.default_rng(seed).uniform(-0.3, 0.3, 3)
    N = orc.shift_matrix(u)
    assert np.abs(N - poly_matrix("appA_N.txt", u)).max() < 1e-14
    assert np.abs(orc.invert(N) - poly_matrix("appA_Ninv.txt", u)).max() < 1e-13
    # N is unit lower triangular (Sec. II: lower-triangular shift matrix)
    assert np.abs(np.triu(N, 1)).max() < 1e-15
    assert np.allclose(np.diag(N), 1.0, atol=1e-15)


@pytest.mark.parametrize("seed", range(8))
def test_moment_transform_invertible(orc, seed):
    """T(u) = N(u) M is invertible to round-off for |u| <= 0.2."""
    rng = np.random.default_rng(100 + seed)
    u = rng.normal(size=3)
    u *= rng.uniform(0, 0.2) / np.linalg.norm(u)
    T = orc.moment_matrix(u)
    Ti = orc.invert(T)
    assert np.abs(T @ Ti - np.eye(Q)).max() < 1e-13
    assert np.abs(Ti @ T - np.eye(Q)).max() < 1e-13
    # T(u) = N(u) M with the printed N and M
    assert np.abs(poly_matrix("appA_N.txt", u) @ int_matrix("appA_M.txt") - T).max() < 1e-14


# ---------------------------------------------------------------- equilibrium
def test_phi_coeffs_sound_speed(orc, lat):
    """Eq. varphi_ik with Eq. press: sum varphi_i = 1 and sum varphi_i c c = 9(1-a)/19 I;
    alpha_b = 8/27 gives the standard weights (c_s^2 = 1/3, Sec. II)."""
    c, w = lat
    for ab in (8 / 27, 0.5, 0.9993):
        ph = orc.phi_coeffs(ab)
        assert abs(ph.sum() - 1) < 1e-15
        assert np.allclose(np.einsum("i,ia,ib->ab", ph, c, c), 9 * (1 - ab) / 19 * np.eye(3), atol=1e-15)
    assert np.allclose(orc.phi_coeffs(8 / 27), w, atol=1e-16)


def _hermite3_equilibrium(rho, u, c, w):
    """Third-order Hermite expansion of the Maxwellian on D3Q27 (c_s^2 = 1/3),
    built from Hermite tensors (a textbook construction, independent of Eq. EES)."""
    cs2 = 1.0 / 3.0
    d = np.eye(3)
    out = np.zeros(Q)
    for i in range(Q):
        ci = c[i]
        H1 = ci
        H2 = np.outer(ci, ci) - cs2 * d
        H3 = np.einsum("a,b,c->abc", ci, ci, ci) - cs2 * (
            np.einsum("a,bc->abc", ci, d) + np.einsum("b,ac->abc", ci, d) + np.einsum("c,ab->abc", ci, d))
        out[i] = w[i] * rho * (1 + H1 @ u / cs2 + np.einsum("ab,a,b", H2, u, u) / (2 * cs2 ** 2)
                               + np.einsum("abc,a,b,c", H3, u, u, u) / (6 * cs2 ** 3))
    return out


def test_equilibrium_reduces_to_third_order_hermite(orc, lat):
    """Eq. EES with Phi_i = 0 and alpha = 8/27 is the third-order equilibrium."""
    c, w = lat
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho, u = rng.uniform(0.5, 1.5), rng.uniform(-0.1, 0.1, 3)
        feq = orc.equilibrium(rho, u, 8 / 27, 0.1, [0, 0, 0])
        assert np.abs(feq - _hermite3_equilibrium(rho, u, c, w)).max() < 1e-15


def test_equilibrium_moments(orc, lat):
    """Moments of Eq. EES with Eq. Phi: mass rho, momentum rho u, and second moment
    rho c_s^2 I + rho u u + nu [u (x) grad rho + grad rho (x) u + (u . grad rho) I]."""
    c, w = lat
    rng = np.random.default_rng(2)
    for _ in range(10):
        rho, u, ab = rng.uniform(0.3, 1.5), rng.uniform(-0.1, 0.1, 3), rng.uniform(0.2, 0.9)
        nub, gr = rng.uniform(1e-4, 0.2), rng.normal(size=3) * 0.1
        feq = orc.equilibrium(rho, u, ab, nub, gr)
        assert abs(feq.sum() - rho) < 1e-14
        assert np.abs(feq @ c - rho * u).max() < 1e-15
        P = np.einsum("i,ia,ib->ab", feq, c, c)
        ref = rho * 9 * (1 - ab) / 19 * np.eye(3) + rho * np.outer(u, u) + nub * (
            np.outer(u, gr) + np.outer(gr, u) + (u @ gr) * np.eye(3))
        assert np.abs(P - ref).max() < 1e-15


def test_forcing_moments(orc, lat):
    """Eq. ketFd (Guo): sum F' = 0, sum F' c = F, sum F' c c = u F + F u."""
    c, _ = lat
    rng = np.random.default_rng(3)
    for _ in range(10):
        u, F = rng.uniform(-0.1, 0.1, 3), rng.normal(size=3) * 1e-3
        Fp = orc.forcing_pop(u, F)
        assert abs(Fp.sum()) < 1e-18
        assert np.abs(Fp @ c - F).max() < 1e-18
        assert np.abs(np.einsum("i,ia,ib->ab", Fp, c, c) - np.outer(u, F) - np.outer(F, u)).max() < 1e-18


def test_gradient_exact_on_polynomials(orc, lat):
    """Isotropic gradient (end of Sec. II) is exact for a x + b y^2 + d x y z + const."""
    c, _ = lat
    rng = np.random.default_rng(4)
    for _ in range(5):
        a1, a2, a3, a0 = rng.normal(size=4)
        x0 = rng.normal(size=3)
        pts = x0 + c
        chi = a0 + a1 * pts[:, 0] + a2 * pts[:, 1] ** 2 + a3 * pts[:, 0] * pts[:, 1] * pts[:, 2]
        g = orc.gradient(chi)
        ref = [a1 + a3 * x0[1] * x0[2], 2 * a2 * x0[1] + a3 * x0[0] * x0[2], a3 * x0[0] * x0[1]]
        assert np.abs(g - ref).max() < 1e-13


# ---------------------------------------------------------------- collision
def _consistent_node(orc, c, rng, F=None):
    """A node with random populations, u from Eq. Momentum and f^(e), F' at that u."""
    rho = rng.uniform(0.6, 1.4)
    u0 = rng.uniform(-0.08, 0.08, 3)
    ab, nub = rng.uniform(0.25, 0.7), rng.uniform(1e-3, 0.1)
    gr = rng.normal(size=3) * 0.05
    f = orc.equilibrium(rho, u0, ab, nub, gr) + rng.normal(size=Q) * 1e-3
    F = rng.normal(size=3) * 1e-3 if F is None else np.asarray(F, float)
    rho = f.sum()
    u = (f @ c + F / 2) / rho
    feq = orc.equilibrium(rho, u, ab, nub, gr)
    Fp = orc.forcing_pop(u, F)
    return f, feq, Fp, u, F, rho


@pytest.mark.parametrize("shift", [0, 1])
def test_collision_single_relaxation_time_is_bgk_guo(orc, lat, shift):
    """Sec. II: equal rates give BGK, and the forcing reduces to Guo's scheme
    (P = (1 - s/2) F'), whether or not the moments are shifted."""
    c, _ = lat
    rng = np.random.default_rng(5 + shift)
    for s in (0.3, 1.0, 1.7):
        p = make_params(_prob(), shift=shift, rates=(s,) * 8)
        f, feq, Fp, u, F, rho = _consistent_node(orc, c, rng)
        out = orc.collide(p, f, feq, Fp, u, s)
        ref = f - s * (f - feq) + (1 - s / 2) * Fp
        assert np.abs(out - ref).max() < 1e-14


def test_collision_conserves_mass_and_adds_force(orc, lat):
    """Eqs. scoll/ketF with s0 = s1 = 0: mass conserved, momentum gains exactly F."""
    c, _ = lat
    rng = np.random.default_rng(7)
    p = make_params(_prob())
    for s2 in (0.4, 1.0, 1.95):
        f, feq, Fp, u, F, rho = _consistent_node(orc, c, rng)
        out = orc.collide(p, f, feq, Fp, u, s2)
        assert abs(out.sum() - f.sum()) < 1e-14
        assert np.abs(out @ c - (f @ c + F)).max() < 1e-15


def test_collision_unit_shear_rate_gives_equilibrium_plus_half_force(orc, lat):
    """With s2nu = 1 and the paper's rates (s2b = s3..s6 = 1) every non-conserved
    moment relaxes fully: fdag = f^(e) + F'/2."""
    c, _ = lat
    rng = np.random.default_rng(8)
    p = make_params(_prob())
    for _ in range(4):
        f, feq, Fp, u, F, rho = _consistent_node(orc, c, rng)
        out = orc.collide(p, f, feq, Fp, u, 1.0)
        assert np.abs(out - (feq + Fp / 2)).max() < 1e-15


def test_collision_relaxes_central_moments(orc, lat):
    """Eq. scoll in central-moment space, with T = N M from the printed matrices:
    rows 4..8 of T (fdag - f^(e) - F'/2) are (1 - s2nu) times rows 4..8 of
    T (f - f^(e) + F'/2), and every other row vanishes."""
    c, _ = lat
    rng = np.random.default_rng(9)
    p = make_params(_prob())
    M = int_matrix("appA_M.txt")
    for s2 in (0.3, 1.4, 1.99):
        f, feq, Fp, u, F, rho = _consistent_node(orc, c, rng)
        out = orc.collide(p, f, feq, Fp, u, s2)
        T = poly_matrix("appA_N.txt", u) @ M
        post = T @ (out - feq - Fp / 2)
        pre = T @ (f - feq + Fp / 2)
        assert np.abs(post[4:9] - (1 - s2) * pre[4:9]).max() < 1e-14
        mask = np.ones(Q, bool)
        mask[4:9] = False
        assert np.abs(post[mask]).max() < 1e-14


def test_collision_shift_matters(orc, lat):
    """The central-moment (shifted) and raw-moment (N = I, Sec. II MRT limit)
    collisions agree at u = 0 and differ at u != 0 when s2nu != 1."""
    c, _ = lat
    rng = np.random.default_rng(10)
    p1, p0 = make_params(_prob(), shift=1), make_params(_prob(), shift=0)
    f, feq, Fp, u, F, rho = _consistent_node(orc, c, rng, F=[0, 0, 0])
    assert np.abs(orc.collide(p1, f, feq, Fp, u, 1.5) - orc.collide(p0, f, feq, Fp, u, 1.5)).max() > 1e-8
    z = np.zeros(3)
    opp = [0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17, 20, 19, 22, 21, 24, 23, 26, 25]
    f0 = f + f[opp]  # symmetric under c -> -c: zero momentum
    feq0 = orc.equilibrium(f0.sum(), z, 0.4, 0.01, z)
    Fp0 = np.zeros(Q)
    a = orc.collide(p1, f0, feq0, Fp0, z, 1.5)
    b = orc.collide(p0, f0, feq0, Fp0, z, 1.5)
    assert np.abs(a - b).max() < 1e-15


def _cube_group(c):
    """All 48 signed permutations of the axes as (matrix, population permutation)."""
    out = []
    key = {tuple(v): i for i, v in enumerate(c.astype(int))}
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3))
            for a in range(3):
                R[a, perm[a]] = signs[a]
            P = np.array([key[tuple((R @ c[i]).astype(int))] for i in range(Q)])
            out.append((R, P))
    return out


def test_node_update_is_cube_symmetric(orc, lat):
    """The full node update (Eq. Momentum to Eq. op3b) commutes with every lattice
    symmetry: rotating the inputs rotates the outputs (catches sign/index errors)."""
    c, _ = lat
    rng = np.random.default_rng(11)
    p = make_params(_prob(g=(0.0, 0.0, 0.0)))
    fr = rng.uniform(0.0, 0.05, Q)
    fb = rng.uniform(0.0, 0.05, Q)
    phi27 = rng.uniform(-1, 1, Q)
    rho27 = rng.uniform(0.5, 1.0, Q)
    Cr, Cb = orc.collide_node(p, 2e-3, fr, fb, phi27, rho27)
    for R, P in _cube_group(c)[1:]:
        # rotated field: value at c_P[i] equals old value at c_i
        fr2, fb2, ph2, rh2 = (np.empty(Q) for _ in range(4))
        fr2[P], fb2[P], ph2[P], rh2[P] = fr, fb, phi27, rho27
        Cr2, Cb2 = orc.collide_node(p, 2e-3, fr2, fb2, ph2, rh2)
        assert np.abs(Cr2[P] - Cr).max() < 1e-15
        assert np.abs(Cb2[P] - Cb).max() < 1e-15


# ---------------------------------------------------------------- interface operators
def test_perturbation_moments(orc, lat):
    """Eq. perturb (squared projection, prefactor A on the colour-blind f):
    zero mass and momentum; second moment (2A/9)|grad phi| (n n - I), whose
    Chapman-Enskog stress gives sigma = (4/9) A tau (Eq. sigma)."""
    c, _ = lat
    rng = np.random.default_rng(12)
    p = make_params(_prob())
    for _ in range(10):
        gphi = rng.normal(size=3) * rng.uniform(0.01, 1)
        A = rng.uniform(1e-4, 1e-2)
        om = orc.perturb(p, A, gphi)
        gn = np.linalg.norm(gphi)
        n = gphi / gn
        assert abs(om.sum()) < 1e-17
        assert np.abs(om @ c).max() < 1e-17
        S = np.einsum("i,ia,ib->ab", om, c, c)
        assert np.abs(S - 2 * A / 9 * gn * (np.outer(n, n) - np.eye(3))).max() < 1e-17
    assert np.all(orc.perturb(p, 1e-3, [0.0, 0.0, 0.0]) == 0)


def test_recolouring_conserves_colours(orc, lat):
    """Eqs. op3r/op3b: the colours sum to fdag, each colour keeps its mass, and the
    red momentum moves by beta rho_r rho_b / rho sum varphi_i cos(theta_i) c_i along n."""
    c, _ = lat
    rng = np.random.default_rng(13)
    p = make_params(_prob())
    for _ in range(10):
        rho_r, rho_b = rng.uniform(0.01, 1.0, 2)
        ab = rng.uniform(0.2, 0.8)
        gphi = rng.normal(size=3)
        fdag = orc.equilibrium(rho_r + rho_b, rng.uniform(-0.05, 0.05, 3), ab, 0.01, [0, 0, 0])
        fr, fb = orc.recolour(p, fdag, rho_r, rho_b, ab, gphi)
        rho = rho_r + rho_b
        assert np.abs(fr + fb - fdag).max() < 1e-15
        assert abs(fr.sum() - rho_r / rho * fdag.sum()) < 1e-15
        n = gphi / np.linalg.norm(gphi)
        ph = orc.phi_coeffs(ab)
        k = 2 * ph[1] + 8 * ph[7] / math.sqrt(2) + 8 * ph[19] / math.sqrt(3)
        shift = fr @ c - rho_r / rho * (fdag @ c)
        assert np.abs(shift - p.beta * rho_r * rho_b / rho * k * n).max() < 1e-15
    # beta = 0: pure proportional split
    p0 = make_params(_prob(beta=0.0))
    fr, fb = orc.recolour(p0, fdag, 0.3, 0.7, 0.5, [1.0, 0, 0])
    assert np.abs(fr - 0.3 * fdag).max() < 1e-16


# ---------------------------------------------------------------- whole-lattice invariants
def test_rest_state_is_fixed_point(orc):
    """A single-phase fluid at rest stays at rest (periodic box)."""
    prob = _prob(nx=5, ny=4, nz=3)
    p = make_params(prob)
    N = prob.n_nodes
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0))
    fr0, fb0 = fr.copy(), fb.copy()
    orc.step(p, prob.A, fr, fb, h, 0, 3)
    assert np.abs(fb - fb0).max() < 1e-16 and np.abs(fr).max() == 0


def test_uniform_flow_is_fixed_point(orc):
    """A uniform single-phase flow is a fixed point of collision and streaming."""
    prob = _prob(nx=4, ny=5, nz=3, nu_b=0.01)
    p = make_params(prob)
    N = prob.n_nodes
    u = np.tile([0.03, -0.02, 0.01], (N, 1))
    fr, fb, h = orc.init_fields(p, np.zeros(N), np.full(N, prob.rho_b0), u)
    fb0 = fb.copy()
    orc.step(p, prob.A, fr, fb, h, 0, 3)
    assert np.abs(fb - fb0).max() < 1e-16


def _random_state(orc, prob, seed):
    from synth import population_noise, random_state_fields
    p = make_params(prob)
    rr, rb, u = random_state_fields(prob, seed)
    fr, fb, h = orc.init_fields(p, rr, rb, u)
    nz = population_noise(prob.n_nodes, seed, amp=2e-4)
    fr += np.where(fr > 1e-3, nz[0], 0.0)
    fb += np.where(fb > 1e-3, nz[1], 0.0)
    return p, fr, fb, h


def test_periodic_conservation(orc, lat):
    """Per-colour mass and total momentum are conserved to round-off with g = 0;
    with gravity the momentum grows by sum_x F(x) each step (Eq. bodyForceJet)."""
    c, _ = lat
    prob = _prob(nx=8, ny=6, nz=5)
    p, fr, fb, h = _random_state(orc, prob, 21)
    m0 = (fr.sum(), fb.sum(), ((fr + fb).sum(axis=1) @ c))
    orc.step(p, prob.A, fr, fb, h, 0, 5)
    m1 = (fr.sum(), fb.sum(), ((fr + fb).sum(axis=1) @ c))
    assert abs(m1[0] - m0[0]) < 1e-12 * abs(m0[0])
    assert abs(m1[1] - m0[1]) < 1e-12 * abs(m0[1])
    assert np.abs(m1[2] - m0[2]).max() < 1e-13
    g = (1e-4, -2e-4, 3e-4)
    prob2 = prob.replace(g=g)
    p2, fr, fb, h = _random_state(orc, prob2, 22)
    rho = (fr + fb).sum(axis=0)
    P0 = (fr + fb).sum(axis=1) @ c
    orc.step(p2, prob2.A, fr, fb, h, 0, 1)
    P1 = (fr + fb).sum(axis=1) @ c
    Ftot = (rho - prob2.rho_b0).sum() * np.array(g)
    assert np.abs(P1 - P0 - Ftot).max() < 1e-13


def test_droplet_keeps_cube_symmetry(orc):
    """A droplet centred at ((n-1)/2, ...) keeps all 48 lattice symmetries
    (Sec. III set-up); gamma != 1, tau != 1 to exercise every operator."""
    prob = _prob(nx=12, ny=12, nz=12, drop_R=3.0, drop_W=2.0, rho_b0=0.5, nu_r=0.02, nu_b=0.05)
    p = make_params(prob)
    fr, fb, h = orc.init_droplet(p, prob.center, 3.0, 2.0)
    orc.step(p, prob.A, fr, fb, h, 0, 4)
    rr, rb, u, ph = orc.macroscopic(p, fr, fb)
    f3 = ph.reshape(12, 12, 12)
    ux = u[:, 0].reshape(12, 12, 12)
    uy = u[:, 1].reshape(12, 12, 12)
    for tr in [(0, 1, 2), (1, 0, 2), (2, 1, 0), (0, 2, 1)]:
        assert np.abs(np.transpose(f3, tr) - f3).max() < 1e-14
    assert np.abs(f3[:, :, ::-1] - f3).max() < 1e-14
    tol = 1e-11 * np.abs(ux).max()
    assert np.abs(ux[:, :, ::-1] + ux).max() < tol
    # (z, y, x) -> (z, x, y) maps u_x to u_y
    assert np.abs(np.transpose(ux, (0, 2, 1)) - uy).max() < tol


def test_splitmix64_published_vectors(orc):
    """SplitMix64 as published (seed 1234567: first outputs of the reference generator)."""
    expected = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                4593380528125082431, 16408922859458223821]
    for n, e in enumerate(expected):
        x = orc.noise(1234567, 0, n, 0, 1 << 20, 1)
        assert x == (e >> 11) * 2.0 ** -53 * 2 - 1


def test_complex_step_is_tangent_linear(orc, orc_cs):
    """The complex-step build gives the directional derivative of the FP64 step
    (checked against a central difference of the FP64 oracle)."""
    prob = _prob(nx=6, ny=5, nz=4, g=(0, 0, 1e-4))
    p, fr, fb, h = _random_state(orc, prob, 31)
    rng = np.random.default_rng(5)
    v = rng.normal(size=fr.shape) * np.where(fr > 1e-3, 1.0, 0.0)
    hcs = 1e-30
    frc, fbc, hc = fr.astype(complex) + 1j * hcs * v, fb.astype(complex), h.astype(complex)
    orc_cs.step(p, prob.A + 1j * hcs * 0.3, frc, fbc, hc, 0, 2)
    tl = frc.imag / hcs
    eps = 1e-6
    out = []
    for s in (1, -1):
        a, b, hh = fr + s * eps * v, fb.copy(), h.copy()
        orc.step(p, prob.A * (1 + 0 * s) + s * eps * 0.3, a, b, hh, 0, 2)
        out.append(a)
    fd = (out[0] - out[1]) / (2 * eps)
    assert np.abs(tl - fd).max() < 1e-7 * max(1.0, np.abs(tl).max())
    # and the real part is the FP64 result
    a, b, hh = fr.copy(), fb.copy(), h.copy()
    orc.step(p, prob.A, a, b, hh, 0, 2)
    assert np.abs(frc.real - a).max() < 1e-15
