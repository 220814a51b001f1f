"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/cglbm.h declares, sizes buffers and validates."""
import ctypes as C
import os
import re

import pytest

from paper_1804_08923_amd import lbm
from paper_1804_08923_amd.workloads import WORKLOADS, droplet_small, jet_128

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cglbm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(lbm_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1804_08923_amd.build import build
        build()
    return lbm.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lbm.EXPORTS)
    assert len(names) == 20


def test_query_sizes(lib):
    for name, mk in WORKLOADS.items():
        prob = mk()
        s = lbm.lbm_query_sizes(lbm.make_params(prob))
        N = prob.n_nodes
        NP = (prob.nx + 2) * (prob.ny + 2) * (prob.nz + 2)
        assert s.n_nodes == N
        assert s.pop_bytes == 54 * NP * 4
        assert s.state_bytes == 54 * N * 4
        assert s.field_bytes == 44 * NP
        assert s.hist_bytes == (2 * 54 * prob.nx * prob.ny * 4 if prob.bc == "jet" else 0)
        # snapshot: 27 FP32 planes, one 16-byte record per padded node, the jet's outlet plane
        a = lambda b: (b + 255) // 256 * 256
        assert s.snap_bytes == a(27 * NP * 4) + a(16 * NP) + (a(2 * 27 * prob.nx * prob.ny * 4) if prob.bc == "jet"
                                                              else 0)
        for st, b, fb in (("bf16", 2, 44), ("fp16", 2, 44), ("bf16eq", 2, 76), ("fp16eq", 2, 76)):
            s2 = lbm.lbm_query_sizes(lbm.make_params(prob.replace(storage=st)))
            assert s2.pop_bytes == 54 * NP * b
            assert s2.field_bytes == fb * NP


@pytest.mark.parametrize("field,value,code", [
    ("nu_r", 0.0, -1), ("nu_b", -1.0, -1), ("rho_b0", 0.0, -1), ("alpha_b", 1.0, -1),
    ("beta", 1.5, -1), ("s4", 0.9, -2), ("nx", 0, -1), ("bc", 7, -1), ("storage", 9, -1),
])
def test_validation(lib, field, value, code):
    p = lbm.make_params(droplet_small())
    setattr(p, field, value)
    s = lbm.lbm_sizes()
    assert lib.lbm_query_sizes(C.byref(p), C.byref(s)) == code
    assert lib.lbm_last_error().decode() != ""


def test_alpha_r_range(lib):
    # gamma < 1 - alpha_b makes alpha_r negative
    p = lbm.make_params(droplet_small().replace(rho_r0=0.5, rho_b0=1.0))
    s = lbm.lbm_sizes()
    assert lib.lbm_query_sizes(C.byref(p), C.byref(s)) == -1


def test_jet_minimum_size(lib):
    p = lbm.make_params(jet_128().replace(nz=2))
    s = lbm.lbm_sizes()
    assert lib.lbm_query_sizes(C.byref(p), C.byref(s)) == -1


def test_inlet_touching_a_side_wall_is_rejected(lib):
    s = lbm.lbm_sizes()
    ok = jet_128()
    assert lib.lbm_query_sizes(C.byref(lbm.make_params(ok)), C.byref(s)) == 0
    for bad in (ok.replace(inlet_D=130.0), ok.replace(inlet_cx=1.0), ok.replace(inlet_cy=126.5, inlet_D=4.0)):
        assert lib.lbm_query_sizes(C.byref(lbm.make_params(bad)), C.byref(s)) == -1
        assert "inlet" in lib.lbm_last_error().decode()


def test_snapshot_entry_points_reject_null_handles(lib):
    assert lib.lbm_step_into(None, None) == -5
    assert lib.lbm_snapshot_save(None, None) == -5
    assert lib.lbm_snapshot_load(None, None, 0) == -5
    assert lib.lbm_adjoint_step_snapshot(None, None, 0, None, None, None, None) == -5
    assert lib.lbm_jet_diagnostics_static(None, None, None, 0) == -5


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.lbm_status_string(code).decode().startswith("LBM_")


def test_null_handle_is_rejected(lib):
    assert lib.lbm_step(None, 1) == -5
    assert lib.lbm_destroy(None) == 0
    assert lib.lbm_time(None) == -1


def test_q19_sizes_and_validation(lib):
    """lattice = 19 (D3Q19): buffer sizes of its two state forms and of the
    jet's outlet history; 16-bit storage is LBM_ERR_UNSUPPORTED; a lattice
    other than 19 or 27, or a bad inlet, is invalid."""
    prob = droplet_small().replace(lattice=19, alpha_b=1 / 3, nx=13, ny=7, nz=5)
    s = lbm.lbm_query_sizes(lbm.make_params(prob))
    N = 13 * 7 * 5
    a = lambda b: (b + 255) // 256 * 256
    assert s.n_nodes == N
    assert s.pop_bytes == max(39 * N * 4, a(76 * N) + 16 * N)
    assert s.state_bytes == 38 * N * 4 and s.field_bytes == 16 * N
    assert s.snap_bytes == 0 and s.adjoint_bytes == 0 and s.hist_bytes == 0
    big = prob.replace(nx=256, ny=256, nz=1024)
    assert lbm.lbm_query_sizes(lbm.make_params(big)).pop_bytes == 39 * 256 * 256 * 1024 * 4
    jet = jet_128().replace(lattice=19, alpha_b=1 / 3)
    sj = lbm.lbm_query_sizes(lbm.make_params(jet))
    assert sj.hist_bytes == 2 * 2 * 19 * 128 * 128 * 4 and sj.snap_bytes == 0
    r = lbm.lbm_sizes()
    for bad, code in ((prob.replace(storage="bf16"), -2), (jet.replace(storage="fp16"), -2),
                      (prob.replace(lattice=23), -1), (jet.replace(inlet_D=130.0), -1)):
        assert lib.lbm_query_sizes(C.byref(lbm.make_params(bad)), C.byref(r)) == code
        assert lib.lbm_last_error().decode() != ""
    # 0 (a zeroed parameter block) still means D3Q27
    p = lbm.make_params(droplet_small())
    p.lattice = 0
    assert lib.lbm_query_sizes(C.byref(p), C.byref(r)) == 0 and r.pop_bytes == 54 * 34 ** 3 * 4
