"""ctypes wrapper around the C oracle (``cglbm_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Three builds of the
same C source are exposed:

* ``"f64"`` -- the FP64 oracle;
* ``"cs"``  -- complex-step build (double complex); ``Im(step(x + i h v))/h``
  is the tangent-linear (directional derivative) of the FP64 scheme to
  round-off (Squire and Trapp 1998, complex-step differentiation);
* ``"f32"`` -- the same plain scheme in single precision, used to measure the
  FP32 round-off floor of the unmodified populations;
* ``"q19"`` -- the FP64 scheme on the D3Q19 subset of the velocity set (the
  reduced lattice of Sec. II, with the derived coefficients noted in the C
  source); its arrays have 19 directions (``Oracle.Q``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cglbm_oracle.c")
_LIBS = {
    "f64": ("liboracle.so", []),
    "cs": ("liboracle_cs.so", ["-DOR_COMPLEX"]),
    "f32": ("liboracle_f32.so", ["-DOR_FLOAT"]),
    "q19": ("liboracle_q19.so", ["-DOR_Q19"]),
}
_DTYPES = {"f64": np.float64, "cs": np.complex128, "f32": np.float32, "q19": np.float64}
_NQ = {"f64": 27, "cs": 27, "f32": 27, "q19": 19}
_lock = threading.Lock()
_cache: dict = {}

Q = 27
BC_PERIODIC, BC_JET = 0, 1


def build_oracle(force: bool = True) -> None:
    """Compile the three oracle builds with gcc (-O2, OpenMP, no fast-math)."""
    for kind, (name, defs) in _LIBS.items():
        out = os.path.join(_HERE, name)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               *defs, "-o", out + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


class OrParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc", C.c_int32),
        ("shift", C.c_int32), ("pad0", C.c_int32),
        ("rho_r0", C.c_double), ("rho_b0", C.c_double), ("alpha_b", C.c_double),
        ("nu_r", C.c_double), ("nu_b", C.c_double), ("beta", C.c_double),
        ("g", C.c_double * 3), ("rates", C.c_double * 8), ("grad_eps", C.c_double),
        ("inlet_cx", C.c_double), ("inlet_cy", C.c_double), ("inlet_D", C.c_double),
        ("inlet_u", C.c_double), ("noise_amp", C.c_double), ("noise_seed", C.c_uint64),
    ]


def make_params(prob, shift: int = 1, rates=None) -> OrParams:
    """Oracle parameter block from a problem description (``workloads.Problem``)."""
    p = OrParams()
    p.nx, p.ny, p.nz = prob.nx, prob.ny, prob.nz
    p.bc = BC_JET if prob.bc == "jet" else BC_PERIODIC
    p.shift = shift
    p.rho_r0, p.rho_b0, p.alpha_b = prob.rho_r0, prob.rho_b0, prob.alpha_b
    p.nu_r, p.nu_b, p.beta = prob.nu_r, prob.nu_b, prob.beta
    for a in range(3):
        p.g[a] = prob.g[a]
    r = rates if rates is not None else (0.0, 0.0, -1.0, 1.0, 1.0, 1.0, 1.0, 1.0)
    for k in range(8):
        p.rates[k] = r[k]
    p.grad_eps = prob.grad_eps
    p.inlet_cx, p.inlet_cy = prob.inlet_cx, prob.inlet_cy
    p.inlet_D, p.inlet_u = prob.inlet_D, prob.inlet_u
    p.noise_amp, p.noise_seed = prob.noise_amp, prob.noise_seed
    return p


def load_oracle(kind: str = "f64"):
    with _lock:
        if kind in _cache:
            return _cache[kind]
        name = _LIBS[kind][0]
        path = os.path.join(_HERE, name)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build_oracle(force=False)
        lib = C.CDLL(path)
        _cache[kind] = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Oracle:
    """Numpy-facing API of one oracle build."""

    def __init__(self, kind: str = "f64"):
        self.kind = kind
        self.dtype = _DTYPES[kind]
        self.Q = _NQ[kind]
        self.lib = load_oracle(kind)
        L = self.lib
        vp = C.c_void_p
        L.or_lattice.argtypes = [vp, vp]
        L.or_moment_matrix.argtypes = [vp, vp]
        L.or_invert.argtypes = [C.c_int, vp, vp]
        L.or_invert.restype = C.c_int
        L.or_shift_matrix.argtypes = [vp, vp]
        L.or_phi_coeffs.argtypes = [self._scalar_t(), vp]
        L.or_gradient.argtypes = [vp, vp]
        L.or_equilibrium.argtypes = [self._scalar_t(), vp, self._scalar_t(), self._scalar_t(), vp, vp]
        L.or_forcing_pop.argtypes = [vp, vp, vp]
        L.or_collide.argtypes = [C.POINTER(OrParams), vp, vp, vp, vp, self._scalar_t(), vp]
        L.or_perturb.argtypes = [C.POINTER(OrParams), self._scalar_t(), vp, vp]
        L.or_recolour.argtypes = [C.POINTER(OrParams), vp, self._scalar_t(), self._scalar_t(),
                                  self._scalar_t(), vp, vp, vp]
        L.or_collide_node.argtypes = [C.POINTER(OrParams), self._scalar_t(), vp, vp, vp, vp, vp, vp]
        L.or_init_fields.argtypes = [C.POINTER(OrParams), vp, vp, vp, vp, vp, vp]
        L.or_init_droplet.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, vp, vp, vp]
        L.or_step.argtypes = [C.POINTER(OrParams), vp, vp, vp, vp, vp, C.c_int64, C.c_int32]
        L.or_step.restype = C.c_int
        L.or_macroscopic.argtypes = [C.POINTER(OrParams), vp, vp, vp, vp, vp, vp]
        L.or_noise.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.or_noise.restype = C.c_double
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]

    # scalar argument type of this variant (complex is passed as a 2-double struct)
    def _scalar_t(self):
        if self.kind == "cs":
            class _Cplx(C.Structure):
                _fields_ = [("re", C.c_double), ("im", C.c_double)]
            self._Cplx = _Cplx
            return _Cplx
        return C.c_float if self.kind == "f32" else C.c_double

    def _s(self, v):
        if self.kind == "cs":
            v = complex(v)
            return self._Cplx(v.real, v.imag)
        return float(v)

    def arr(self, a) -> np.ndarray:
        return np.ascontiguousarray(np.asarray(a), dtype=self.dtype)

    # ---- tables and per-node operators ---------------------------------
    def lattice(self):
        c = np.zeros((self.Q, 3), np.int32)
        w = np.zeros(self.Q, np.float64)
        self.lib.or_lattice(_ptr(c), _ptr(w))
        return c, w

    def moment_matrix(self, u):
        u = self.arr(u)
        T = np.zeros((self.Q, self.Q), self.dtype)
        self.lib.or_moment_matrix(_ptr(u), _ptr(T))
        return T

    def invert(self, A):
        A = self.arr(A)
        n = A.shape[0]
        out = np.zeros_like(A)
        rc = self.lib.or_invert(n, _ptr(A), _ptr(out))
        if rc != 0:
            raise np.linalg.LinAlgError("singular")
        return out

    def shift_matrix(self, u):
        u = self.arr(u)
        N = np.zeros((self.Q, self.Q), self.dtype)
        self.lib.or_shift_matrix(_ptr(u), _ptr(N))
        return N

    def phi_coeffs(self, ab):
        out = np.zeros(self.Q, self.dtype)
        self.lib.or_phi_coeffs(self._s(ab), _ptr(out))
        return out

    def gradient(self, chi27):
        chi = self.arr(chi27)
        g = np.zeros(3, self.dtype)
        self.lib.or_gradient(_ptr(chi), _ptr(g))
        return g

    def equilibrium(self, rho, u, ab, nub, grho):
        u, grho = self.arr(u), self.arr(grho)
        out = np.zeros(self.Q, self.dtype)
        self.lib.or_equilibrium(self._s(rho), _ptr(u), self._s(ab), self._s(nub), _ptr(grho), _ptr(out))
        return out

    def forcing_pop(self, u, F):
        u, F = self.arr(u), self.arr(F)
        out = np.zeros(self.Q, self.dtype)
        self.lib.or_forcing_pop(_ptr(u), _ptr(F), _ptr(out))
        return out

    def collide(self, p: OrParams, f, feq, Fp, u, s2nu):
        f, feq, Fp, u = self.arr(f), self.arr(feq), self.arr(Fp), self.arr(u)
        out = np.zeros(self.Q, self.dtype)
        self.lib.or_collide(C.byref(p), _ptr(f), _ptr(feq), _ptr(Fp), _ptr(u), self._s(s2nu), _ptr(out))
        return out

    def perturb(self, p: OrParams, A, gphi):
        g = self.arr(gphi)
        out = np.zeros(self.Q, self.dtype)
        self.lib.or_perturb(C.byref(p), self._s(A), _ptr(g), _ptr(out))
        return out

    def recolour(self, p: OrParams, fdag, rho_r, rho_b, ab, gphi):
        fd, g = self.arr(fdag), self.arr(gphi)
        fr = np.zeros(self.Q, self.dtype)
        fb = np.zeros(self.Q, self.dtype)
        self.lib.or_recolour(C.byref(p), _ptr(fd), self._s(rho_r), self._s(rho_b), self._s(ab),
                             _ptr(g), _ptr(fr), _ptr(fb))
        return fr, fb

    def collide_node(self, p: OrParams, A, fr27, fb27, phi27, rho27):
        a, b, c, d = (self.arr(v) for v in (fr27, fb27, phi27, rho27))
        Cr = np.zeros(self.Q, self.dtype)
        Cb = np.zeros(self.Q, self.dtype)
        self.lib.or_collide_node(C.byref(p), self._s(A), _ptr(a), _ptr(b), _ptr(c), _ptr(d),
                                 _ptr(Cr), _ptr(Cb))
        return Cr, Cb

    # ---- whole lattice ---------------------------------------------------
    def new_state(self, p: OrParams):
        N = p.nx * p.ny * p.nz
        fr = np.zeros((self.Q, N), self.dtype)
        fb = np.zeros((self.Q, N), self.dtype)
        hist = np.zeros((2 * self.Q, p.nx * p.ny), self.dtype)
        return fr, fb, hist

    def init_fields(self, p: OrParams, rho_r, rho_b, u=None):
        fr, fb, hist = self.new_state(p)
        a, b = self.arr(rho_r).ravel(), self.arr(rho_b).ravel()
        uu = self.arr(u).reshape(-1, 3) if u is not None else None
        self.lib.or_init_fields(C.byref(p), _ptr(a), _ptr(b), _ptr(uu), _ptr(fr), _ptr(fb), _ptr(hist))
        return fr, fb, hist

    def init_droplet(self, p: OrParams, center, R, W):
        fr, fb, hist = self.new_state(p)
        self.lib.or_init_droplet(C.byref(p), float(center[0]), float(center[1]), float(center[2]),
                                 float(R), float(W), _ptr(fr), _ptr(fb), _ptr(hist))
        return fr, fb, hist

    def step(self, p: OrParams, A, fr, fb, hist, t0: int, nsteps: int, inlet_uz=None):
        """Advance (fr, fb, hist) in place by ``nsteps`` steps starting at time ``t0``."""
        for a in (fr, fb, hist):
            assert a.dtype == self.dtype and a.flags.c_contiguous
        Aa = self.arr([A])
        iu = self.arr(inlet_uz).ravel() if inlet_uz is not None else None
        rc = self.lib.or_step(C.byref(p), _ptr(Aa), _ptr(iu), _ptr(fr), _ptr(fb), _ptr(hist),
                              int(t0), int(nsteps))
        if rc != 0:
            raise MemoryError("oracle step failed to allocate")

    def macroscopic(self, p: OrParams, fr, fb):
        N = p.nx * p.ny * p.nz
        rr = np.zeros(N, self.dtype)
        rb = np.zeros(N, self.dtype)
        u = np.zeros((N, 3), self.dtype)
        ph = np.zeros(N, self.dtype)
        self.lib.or_macroscopic(C.byref(p), _ptr(fr), _ptr(fb), _ptr(rr), _ptr(rb), _ptr(u), _ptr(ph))
        return rr, rb, u, ph

    def noise(self, seed, t, x, y, nx, ny) -> float:
        return self.lib.or_noise(seed, t, x, y, nx, ny)

    def num_threads(self) -> int:
        return self.lib.or_num_threads()

    def set_num_threads(self, n: int) -> None:
        self.lib.or_set_num_threads(int(n))
