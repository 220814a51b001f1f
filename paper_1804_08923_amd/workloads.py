"""Problem descriptions and the synthetic workloads of the benchmarks.

A :class:`Problem` holds lattice-unit parameters.  :func:`jet_problem` maps the
dimensionless groups of the jet problem (density ratio gamma, viscosity ratio
eta, Re, We, Fr; Eqs. densityRatio to Froude of the paper) to lattice units
with c = delta_t = 1, the jet phase red with rho_r0 = 1 and the coolant blue
with rho_b0 = 1/gamma (Sec. IV B), and the perturbation strength A from the
surface tension through Eq. sigma, sigma = (4/9) A tau.  Where the two phases
have different viscosities tau is taken at the interface (phi = 0), where the
harmonic mean gives nu_bar = 2 nu_r nu_b / (nu_r + nu_b).

All inputs are synthetic: the static droplet of Sec. III and the jet set-up of
Sec. IV A (all-blue domain at rest, circular inlet, free-slip walls,
convective outlet, buoyancy on the dispersed phase).  No dataset is involved.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional, Tuple


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    bc: str = "periodic"          # "periodic" | "jet"
    rho_r0: float = 1.0
    rho_b0: float = 1.0
    alpha_b: float = 8.0 / 27.0
    nu_r: float = 1.0 / 6.0
    nu_b: float = 1.0 / 6.0
    A: float = 1e-3
    beta: float = 0.7
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    grad_eps: float = 1e-10
    inlet_cx: float = 0.0
    inlet_cy: float = 0.0
    inlet_D: float = 0.0
    inlet_u: float = 0.0
    noise_amp: float = 0.0
    noise_seed: int = 0
    init: str = "droplet"         # "droplet" | "jet" (all blue at rest) | "fields"
    drop_R: float = 8.0
    drop_W: float = 2.0
    drop_center: Optional[Tuple[float, float, float]] = None
    steps: int = 200
    storage: str = "fp32"         # "fp32" | "bf16" | "fp16" | "bf16eq" | "fp16eq"
    lattice: int = 27             # 27 (D3Q27) | 19 (D3Q19; its colours take alpha_b = 1/3)
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def gamma(self) -> float:
        return self.rho_r0 / self.rho_b0

    @property
    def alpha_r(self) -> float:
        return 1.0 - (1.0 - self.alpha_b) / self.gamma

    @property
    def center(self) -> Tuple[float, float, float]:
        if self.drop_center is not None:
            return self.drop_center
        return ((self.nx - 1) / 2.0, (self.ny - 1) / 2.0, (self.nz - 1) / 2.0)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def tau_interface(nu_r: float, nu_b: float) -> float:
    nu_bar = 2.0 * nu_r * nu_b / (nu_r + nu_b)
    return 3.0 * nu_bar + 0.5


def jet_problem(name, nx, ny, nz, D, u, gamma, eta, Re, We, Fr, steps, noise_amp=0.01,
                noise_seed=20180423) -> Problem:
    """Jet of Sec. IV in lattice units from its dimensionless groups."""
    nu_j = u * D / Re                     # Re = rho_j u D / mu_j
    nu_c = nu_j / eta                     # eta = nu_j / nu_c
    sigma = 1.0 * u * u * D / We          # We = rho_j u^2 D / sigma, rho_j = 1
    g = u * u / (Fr * D)                  # Fr = u^2 / (g D)
    tau = tau_interface(nu_j, nu_c)
    A = 9.0 * sigma / (4.0 * tau)         # Eq. sigma
    return Problem(name=name, nx=nx, ny=ny, nz=nz, bc="jet", rho_r0=1.0, rho_b0=1.0 / gamma,
                   nu_r=nu_j, nu_b=nu_c, A=A, g=(0.0, 0.0, g),
                   inlet_cx=(nx - 1) / 2.0, inlet_cy=(ny - 1) / 2.0, inlet_D=D, inlet_u=u,
                   noise_amp=noise_amp, noise_seed=noise_seed, init="jet", steps=steps,
                   meta=dict(gamma=gamma, eta=eta, Re=Re, We=We, Fr=Fr, sigma=sigma, tau=tau))


def droplet_small() -> Problem:
    """32^3 periodic static droplet: R = 8, interface width 2, gamma = 1, tau = 1,
    A = 1e-3, beta = 0.7, 200 steps."""
    return Problem(name="droplet-32", nx=32, ny=32, nz=32, bc="periodic", nu_r=1 / 6, nu_b=1 / 6,
                   A=1e-3, drop_R=8.0, drop_W=2.0, steps=200,
                   meta=dict(gamma=1.0, tau=1.0, sigma=4.0 / 9.0 * 1e-3))


def droplet_cm() -> Problem:
    """Same droplet with tau != 1, gamma = 2, unequal viscosities and gravity, so
    that the central-moment relaxation of the shear moments is exercised."""
    return Problem(name="droplet-32-cm", nx=32, ny=32, nz=32, bc="periodic", rho_r0=1.0, rho_b0=0.5,
                   nu_r=0.01, nu_b=0.03, A=1e-3, g=(0.0, 0.0, 1e-5), drop_R=8.0, drop_W=2.0, steps=200)


def jet_128() -> Problem:
    """128x128x512 liquid-liquid jet: D = 16, u = 0.04, gamma = 2, eta = 1,
    Re = 1e3, We = 50, Fr = 10, 1 % radial inlet noise, 5000 steps."""
    return jet_problem("jet-128x128x512", 128, 128, 512, 16, 0.04, 2.0, 1.0, 1e3, 50.0, 10.0, 5000)


def jet_256() -> Problem:
    """256x256x1024 high-Re jet: D = 24, u = 0.05, gamma = 2, eta = 0.01,
    Re = 1e6, We = 1e3, Fr = 10, 1 % inlet noise, 20000 steps."""
    return jet_problem("jet-256x256x1024", 256, 256, 1024, 24, 0.05, 2.0, 0.01, 1e6, 1e3, 10.0, 20000)


def jet_64() -> Problem:
    """64x64x256 jet for differentiation: D = 12, u = 0.03, gamma = 2, eta = 1,
    Re = 500, We = 30, Fr = 10, no inlet noise, 2000 steps."""
    return jet_problem("jet-64x64x256", 64, 64, 256, 12, 0.03, 2.0, 1.0, 500.0, 30.0, 10.0, 2000,
                       noise_amp=0.0)


# The UT melt-jet cases of Sec. IV B (Table II): an 8 D x 8 D x 40 D lattice
# with D = 30, u = 0.05, gamma = 8.3, eta = 0.54, and the case's Re, We, Fr.
UT_CASES = {1: (6.1e4, 2.3e2, 64.0), 2: (6.5e4, 1.8e2, 24.0), 3: (1.1e5, 3.3e2, 20.0), 4: (1.5e5, 4.5e2, 16.0)}


def jet_ut(case: int) -> Problem:
    """UT case `case` at the paper's resolution (240x240x1200, 69 M nodes),
    20 000 steps, 1 % inlet noise."""
    Re, We, Fr = UT_CASES[case]
    return jet_problem(f"jet-ut{case}-240x240x1200", 240, 240, 1200, 30, 0.05, 8.3, 0.54, Re, We, Fr, 20000)


def jet_ft(fine: bool) -> Problem:
    """FT T1 (Sec. IV D, Table IV): an 8 D x 8 D x 20 D lattice, D = 30 (coarse,
    240x240x600, 34.6 M nodes) or D = 60 (fine, 480x480x1200, 276 M nodes);
    u = 0.05, gamma = 10.1, eta = 1.4, Re = 1.1e6, We = 9.3e4, Fr = 200."""
    D = 60 if fine else 30
    return jet_problem(f"jet-ft-{'fine' if fine else 'coarse'}-{8 * D}x{8 * D}x{20 * D}", 8 * D, 8 * D, 20 * D, D,
                       0.05, 10.1, 1.4, 1.1e6, 9.3e4, 200.0, 20000)


WORKLOADS = {
    "droplet-32": droplet_small,
    "droplet-32-cm": droplet_cm,
    "jet-128x128x512": jet_128,
    "jet-256x256x1024": jet_256,
    "jet-64x64x256": jet_64,
    "jet-ut1-240x240x1200": lambda: jet_ut(1),
    "jet-ut2-240x240x1200": lambda: jet_ut(2),
    "jet-ut3-240x240x1200": lambda: jet_ut(3),
    "jet-ut4-240x240x1200": lambda: jet_ut(4),
    "jet-ft-coarse-240x240x600": lambda: jet_ft(False),
    "jet-ft-fine-480x480x1200": lambda: jet_ft(True),
}
