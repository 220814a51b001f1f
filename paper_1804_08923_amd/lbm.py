"""Thin ctypes binding of liblbm.so (include/cglbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides device memory and the stream.  There is no
CPU fallback: without the built library or a GPU every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

from .workloads import Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK = 0
BC = {"periodic": 0, "jet": 1}
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16eq": 3, "fp16eq": 4}
INIT = {"fields": 0, "droplet": 1, "jet": 2}
Q = 27


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class lbm_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32), ("storage", C.c_int32), ("init", C.c_int32),
        ("rho_r0", C.c_double), ("rho_b0", C.c_double), ("alpha_b", C.c_double),
        ("nu_r", C.c_double), ("nu_b", C.c_double), ("A", C.c_double), ("beta", C.c_double),
        ("g", C.c_double * 3),
        ("s_b", C.c_double), ("s3", C.c_double), ("s4", C.c_double), ("s5", C.c_double), ("s6", C.c_double),
        ("grad_eps", C.c_double),
        ("inlet_cx", C.c_double), ("inlet_cy", C.c_double), ("inlet_D", C.c_double), ("inlet_u", C.c_double),
        ("noise_amp", C.c_double), ("noise_seed", C.c_uint64),
        ("drop_cx", C.c_double), ("drop_cy", C.c_double), ("drop_cz", C.c_double),
        ("drop_R", C.c_double), ("drop_W", C.c_double),
        ("lattice", C.c_int32), ("lattice_pad", C.c_int32),
    ]


class lbm_sizes(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("n_nodes", "pop_bytes", "field_bytes", "hist_bytes", "audit_bytes",
                                          "inlet_bytes", "adjoint_bytes", "state_bytes", "snap_bytes")]


class lbm_jet_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("jet_nodes", "front_z", "column_volume", "n_fragments")]


class lbm_buffers(C.Structure):
    _fields_ = [("pop_a", C.c_void_p), ("pop_b", C.c_void_p), ("fields", C.c_void_p), ("hist", C.c_void_p),
                ("audit", C.c_void_p), ("inlet_uz", C.c_void_p), ("adjoint", C.c_void_p)]


EXPORTS = ("lbm_query_sizes", "lbm_init", "lbm_step", "lbm_macroscopic", "lbm_get_state", "lbm_set_state",
           "lbm_time", "lbm_step_into", "lbm_snapshot_save", "lbm_snapshot_load", "lbm_adjoint_step",
           "lbm_adjoint_step_snapshot", "lbm_diag_bytes", "lbm_jet_diagnostics", "lbm_jet_diagnostics_static",
           "lbm_profile", "lbm_profile_read", "lbm_destroy", "lbm_status_string", "lbm_last_error")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_1804_08923_amd/build.py")
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.lbm_query_sizes.argtypes = [C.POINTER(lbm_params), C.POINTER(lbm_sizes)]
    lib.lbm_init.argtypes = [C.POINTER(vp), C.POINTER(lbm_params), C.POINTER(lbm_buffers), vp, vp, vp, vp]
    lib.lbm_step.argtypes = [vp, i32]
    lib.lbm_macroscopic.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_double)]
    lib.lbm_get_state.argtypes = [vp, vp]
    lib.lbm_set_state.argtypes = [vp, vp, i64]
    lib.lbm_time.argtypes = [vp]
    lib.lbm_time.restype = i64
    lib.lbm_adjoint_step.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp]
    lib.lbm_adjoint_step_snapshot.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp]
    lib.lbm_step_into.argtypes = [vp, vp]
    lib.lbm_snapshot_save.argtypes = [vp, vp]
    lib.lbm_snapshot_load.argtypes = [vp, vp, i64]
    lib.lbm_diag_bytes.argtypes = [C.POINTER(lbm_params), C.POINTER(C.c_uint64)]
    lib.lbm_jet_diagnostics.argtypes = [vp, vp, C.POINTER(lbm_jet_stats), C.POINTER(C.c_int64), C.c_int64]
    lib.lbm_jet_diagnostics_static.argtypes = [vp, C.POINTER(lbm_jet_stats), C.POINTER(C.c_int64), C.c_int64]
    lib.lbm_profile.argtypes = [vp, C.c_int]
    lib.lbm_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_status_string.argtypes = [C.c_int]
    lib.lbm_status_string.restype = C.c_char_p
    lib.lbm_last_error.restype = C.c_char_p
    for name in ("lbm_query_sizes", "lbm_init", "lbm_step", "lbm_macroscopic", "lbm_get_state",
                 "lbm_set_state", "lbm_step_into", "lbm_snapshot_save", "lbm_snapshot_load", "lbm_adjoint_step",
                 "lbm_adjoint_step_snapshot", "lbm_diag_bytes", "lbm_jet_diagnostics",
                 "lbm_jet_diagnostics_static", "lbm_profile", "lbm_profile_read", "lbm_destroy"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(lib, rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, f"{lib.lbm_status_string(rc).decode()}: {lib.lbm_last_error().decode()}")


def make_params(prob: Problem) -> lbm_params:
    p = lbm_params()
    p.nx, p.ny, p.nz = prob.nx, prob.ny, prob.nz
    p.bc, p.storage, p.init = BC[prob.bc], STORAGE[prob.storage], INIT[prob.init]
    p.rho_r0, p.rho_b0, p.alpha_b = prob.rho_r0, prob.rho_b0, prob.alpha_b
    p.nu_r, p.nu_b, p.A, p.beta = prob.nu_r, prob.nu_b, prob.A, prob.beta
    for a in range(3):
        p.g[a] = prob.g[a]
    p.s_b = p.s3 = p.s4 = p.s5 = p.s6 = 1.0
    p.grad_eps = prob.grad_eps
    p.inlet_cx, p.inlet_cy, p.inlet_D, p.inlet_u = prob.inlet_cx, prob.inlet_cy, prob.inlet_D, prob.inlet_u
    p.noise_amp, p.noise_seed = prob.noise_amp, prob.noise_seed
    c = prob.center
    p.drop_cx, p.drop_cy, p.drop_cz, p.drop_R, p.drop_W = c[0], c[1], c[2], prob.drop_R, prob.drop_W
    p.lattice = prob.lattice
    return p


def lbm_query_sizes(params: lbm_params) -> lbm_sizes:
    lib = load_library()
    s = lbm_sizes()
    _check(lib, lib.lbm_query_sizes(C.byref(params), C.byref(s)))
    return s


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class LBM:
    """One simulation on one GPU: owns the torch buffers and the library handle."""

    def __init__(self, prob: Problem, device: str = "cuda:0", rho_r=None, rho_b=None, u=None,
                 inlet_uz=None, adjoint: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a ROCm GPU; no device is visible")
        self.torch = torch
        self.lib = load_library()
        self.prob = prob
        self.Q = prob.lattice      # directions per colour: 27, or 19 on D3Q19
        self.device = torch.device(device)
        self.params = make_params(prob)
        self.sizes = lbm_query_sizes(self.params)
        s = self.sizes
        dev = self.device

        def buf(nbytes, dtype=torch.uint8):
            el = torch.empty((), dtype=dtype).element_size()
            return torch.empty(max(1, int(nbytes) // el), dtype=dtype, device=dev)

        self.pop_a = buf(s.pop_bytes)
        self.pop_b = buf(s.pop_bytes)
        self.fields = buf(s.field_bytes, torch.float32)
        self.hist = buf(s.hist_bytes, torch.float32) if s.hist_bytes else None
        self.audit = buf(s.audit_bytes, torch.float64)
        self.adjoint = buf(s.adjoint_bytes) if (adjoint and s.adjoint_bytes) else None
        self.inlet = None
        if inlet_uz is not None:
            self.inlet = torch.as_tensor(inlet_uz, dtype=torch.float32, device=dev).contiguous().reshape(-1)
            assert self.inlet.numel() == prob.nx * prob.ny
        b = lbm_buffers()
        b.pop_a, b.pop_b = _ptr(self.pop_a), _ptr(self.pop_b)
        b.fields, b.hist, b.audit = _ptr(self.fields), _ptr(self.hist), _ptr(self.audit)
        b.inlet_uz, b.adjoint = _ptr(self.inlet), _ptr(self.adjoint)
        self._bufs = b
        fr = fb = fu = None
        if prob.init == "fields":
            fr = torch.as_tensor(rho_r, dtype=torch.float32, device=dev).contiguous()
            fb = torch.as_tensor(rho_b, dtype=torch.float32, device=dev).contiguous()
            fu = None if u is None else torch.as_tensor(u, dtype=torch.float32, device=dev).contiguous()
            self._init_fields = (fr, fb, fu)
        self.stream = torch.cuda.current_stream(dev)
        h = C.c_void_p()
        _check(self.lib, self.lib.lbm_init(C.byref(h), C.byref(self.params), C.byref(b), _ptr(fr), _ptr(fb),
                                           _ptr(fu), self.stream.cuda_stream))
        self.h = h

    # -- entry points ------------------------------------------------------
    def step(self, n: int = 1):
        _check(self.lib, self.lib.lbm_step(self.h, int(n)))

    def macroscopic(self, audit: bool = False):
        torch = self.torch
        N = self.sizes.n_nodes
        out = {k: torch.empty(N, dtype=torch.float32, device=self.device) for k in ("rho_r", "rho_b", "phi")}
        out["u"] = torch.empty((N, 3), dtype=torch.float32, device=self.device)
        a = (C.c_double * 5)() if audit else None
        _check(self.lib, self.lib.lbm_macroscopic(self.h, out["rho_r"].data_ptr(), out["rho_b"].data_ptr(),
                                                  out["u"].data_ptr(), out["phi"].data_ptr(), a))
        if audit:
            out["audit"] = list(a)
        return out

    def get_state(self):
        st = self.torch.empty((2 * self.Q, self.sizes.n_nodes), dtype=self.torch.float32, device=self.device)
        _check(self.lib, self.lib.lbm_get_state(self.h, st.data_ptr()))
        return st

    def set_state(self, state, t: int = 0):
        st = self.torch.as_tensor(state, dtype=self.torch.float32, device=self.device).contiguous()
        assert st.numel() == 2 * self.Q * self.sizes.n_nodes
        self._set_state_keep = st
        _check(self.lib, self.lib.lbm_set_state(self.h, st.data_ptr(), int(t)))

    @property
    def time(self) -> int:
        return int(self.lib.lbm_time(self.h))

    # -- snapshots (lbm_step_into, lbm_snapshot_save / _load) ----------------
    def new_snapshot(self):
        """An uninitialised device buffer of snap_bytes (256-byte aligned)."""
        return self.torch.empty(int(self.sizes.snap_bytes), dtype=self.torch.uint8, device=self.device)

    def _snap(self, snap):
        assert snap.dtype == self.torch.uint8 and snap.numel() >= self.sizes.snap_bytes and snap.is_contiguous()
        return snap.data_ptr()

    def step_to_snapshot(self, snap):
        """One step written into ``snap``, which becomes the current state (it
        must not be modified until the next step or load)."""
        _check(self.lib, self.lib.lbm_step_into(self.h, self._snap(snap)))
        self._current_snapshot = snap

    def save_snapshot(self, snap):
        _check(self.lib, self.lib.lbm_snapshot_save(self.h, self._snap(snap)))

    def load_snapshot(self, snap, t: int):
        _check(self.lib, self.lib.lbm_snapshot_load(self.h, self._snap(snap), int(t)))

    def adjoint_step(self, state_t, t: int, lam_in, lam_out, dJ_dA, dJ_du_in=None):
        """One reverse step (see lbm_adjoint_step): lam_out = (d x_{t+1}/d x_t)^T lam_in;
        dJ_dA (float64, 1 element) and dJ_du_in (float32, nx*ny) are incremented."""
        for a in (state_t, lam_in, lam_out):
            assert a.dtype == self.torch.float32 and a.is_contiguous() and a.numel() == 2 * self.Q * self.sizes.n_nodes
        assert dJ_dA.dtype == self.torch.float64 and dJ_dA.numel() >= 1
        if dJ_du_in is not None:
            assert dJ_du_in.dtype == self.torch.float32 and dJ_du_in.numel() == self.prob.nx * self.prob.ny
        _check(self.lib, self.lib.lbm_adjoint_step(self.h, state_t.data_ptr(), int(t), lam_in.data_ptr(),
                                                   lam_out.data_ptr(), dJ_dA.data_ptr(), _ptr(dJ_du_in)))

    def adjoint_step_snapshot(self, snap_t, t: int, lam_in, lam_out, dJ_dA, dJ_du_in=None):
        """adjoint_step with the forward state at time t given as a snapshot."""
        for a in (lam_in, lam_out):
            assert a.dtype == self.torch.float32 and a.is_contiguous() and a.numel() == 2 * self.Q * self.sizes.n_nodes
        assert dJ_dA.dtype == self.torch.float64 and dJ_dA.numel() >= 1
        if dJ_du_in is not None:
            assert dJ_du_in.dtype == self.torch.float32 and dJ_du_in.numel() == self.prob.nx * self.prob.ny
        _check(self.lib, self.lib.lbm_adjoint_step_snapshot(self.h, self._snap(snap_t), int(t), lam_in.data_ptr(),
                                                            lam_out.data_ptr(), dJ_dA.data_ptr(), _ptr(dJ_du_in)))

    def jet_diagnostics(self, cap: Optional[int] = None):
        """Leading edge and fragments of the jet phase (lbm_jet_diagnostics):
        a dict of the four statistics and the fragment volumes (numpy int64,
        sorted in descending order; at most ``cap`` of them, all by default)."""
        import numpy as np
        torch = self.torch
        if getattr(self, "_diag_work", None) is None:
            nb = C.c_uint64()
            _check(self.lib, self.lib.lbm_diag_bytes(C.byref(self.params), C.byref(nb)))
            self._diag_work = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        st = lbm_jet_stats()
        want = cap is None
        cap = min(self.sizes.n_nodes, 1 << 16) if want else int(cap)
        vol = (C.c_int64 * max(cap, 1))()
        _check(self.lib, self.lib.lbm_jet_diagnostics(self.h, self._diag_work.data_ptr(), C.byref(st), vol, cap))
        if want and st.n_fragments > cap:  # all of them were asked for: again with room for every one
            cap = st.n_fragments
            vol = (C.c_int64 * cap)()
            _check(self.lib, self.lib.lbm_jet_diagnostics(self.h, self._diag_work.data_ptr(), C.byref(st), vol,
                                                          cap))
        n = min(cap, st.n_fragments)
        v = np.sort(np.frombuffer(vol, dtype=np.int64, count=n))[::-1].copy()
        return {k: int(getattr(st, k)) for k, _ in lbm_jet_stats._fields_}, v

    def jet_diagnostics_static(self, cap: int):
        """jet_diagnostics through lbm_jet_diagnostics_static (the library's
        static work memory; no device buffer is allocated): the four
        statistics and the first min(cap, n_fragments) fragment volumes,
        sorted in descending order."""
        import numpy as np
        st = lbm_jet_stats()
        vol = (C.c_int64 * max(int(cap), 1))()
        _check(self.lib, self.lib.lbm_jet_diagnostics_static(self.h, C.byref(st), vol, int(cap)))
        n = min(int(cap), st.n_fragments)
        v = np.sort(np.frombuffer(vol, dtype=np.int64, count=n))[::-1].copy()
        return {k: int(getattr(st, k)) for k, _ in lbm_jet_stats._fields_}, v

    def profile(self, enable: bool = True):
        _check(self.lib, self.lib.lbm_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """(ms, launches): index 0 density pass, 1 fused kernel, 2 boundary kernels."""
        ms = (C.c_double * 3)()
        n = (C.c_int64 * 3)()
        _check(self.lib, self.lib.lbm_profile_read(self.h, ms, n))
        return list(ms), list(n)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
