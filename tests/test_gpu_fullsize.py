"""Parity at full size: the 128x128x512 jet (the benchmark workload, in the
launch configuration bench.py times) and the 256x256x1024 high-Re jet
(67 M nodes), FP32 storage.

One step from a random physical state of the whole lattice, taken over with
lbm_set_state.  The oracle cannot step 8.4 M nodes in test time, so the
comparison runs on sampled nodes: for each, the oracle's node update
(collision, perturbation, recolouring) of every one of its 27 source nodes,
with the density stencils from the oracle's macroscopic fields, gives the
streamed populations, compared population by population.  Samples are
interior nodes spread over the whole lattice (first and last blocks, plane
ends, ragged positions); the boundary rules themselves are covered at small
size by the other parity tests, which run the same kernels.
"""
import numpy as np
import pytest

from harness import Q, say
from oracle import make_params as or_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible ROCm device"
    return t


@pytest.mark.parametrize("workload", ["jet-128x128x512", "jet-256x256x1024"])
def test_full_size_jet_sampled_step(torch, orc, workload):
    from synth import population_noise_planes, random_state_fields

    from paper_1804_08923_amd.lbm import LBM
    from paper_1804_08923_amd.workloads import WORKLOADS
    prob = WORKLOADS[workload]()
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    N = prob.n_nodes
    say(f"full size {nx}x{ny}x{nz}: building a random state")
    p = or_params(prob)
    rr, rb, u = random_state_fields(prob, seed=101)
    fr, fb, _ = orc.init_fields(p, rr, rb, u)
    del rr, rb, u
    # the same noise as population_noise(N, 101, 2e-4), drawn plane by plane
    st = np.empty((2 * Q, N), np.float32)
    for j, (f, noise) in enumerate(zip([fr[i] for i in range(Q)] + [fb[i] for i in range(Q)],
                                       population_noise_planes(N, seed=101, amp=2e-4))):
        st[j] = f + np.where(f > 1e-3, noise, 0.0)
    del fr, fb
    fr64 = st[:Q].astype(np.float64)
    fb64 = st[Q:].astype(np.float64)
    t0 = 7
    say(f"full size {nx}x{ny}x{nz}: one GPU step")
    sim = LBM(prob)
    sim.set_state(torch.from_numpy(st).cuda(), t=t0)
    sim.step(1)
    out = sim.get_state().cpu().numpy()
    sim.close()
    del st
    torch.cuda.empty_cache()

    say(f"full size {nx}x{ny}x{nz}: oracle fields and sampled node updates")
    _, _, _, phi = orc.macroscopic(p, fr64, fb64)
    rho = fr64.sum(axis=0) + fb64.sum(axis=0)
    c, _ = orc.lattice()
    c = np.asarray(c).reshape(Q, 3)

    def nid(x, y, z):
        return (z * ny + y) * nx + x

    cache = {}

    def post(s):
        if s not in cache:
            x, y, z = s
            idx = [nid(x + c[j, 0], y + c[j, 1], z + c[j, 2]) for j in range(Q)]
            n = nid(x, y, z)
            cache[s] = orc.collide_node(p, prob.A, fr64[:, n], fb64[:, n], phi[idx], rho[idx])
        return cache[s]

    rng = np.random.default_rng(5)
    samples = [(2, 2, 2), (nx - 3, ny - 3, nz - 3), (nx - 3, ny // 2, nz // 2), (nx // 2, 2, nz // 2 + 44),
               (2, ny - 3, 5), (nx // 2 - 1, 3, 2), (nx // 2, 3, nz - 4), (nx // 2 + 1, ny // 2, nz - 3)]
    samples += [tuple(int(v) for v in (rng.integers(2, nx - 2), rng.integers(2, ny - 2), rng.integers(2, nz - 3)))
                for _ in range(60)]
    fmax = np.abs(out).max()
    worst = 0.0
    for (x, y, z) in samples:
        n = nid(x, y, z)
        for i in range(Q):
            Cr, Cb = post((x - c[i, 0], y - c[i, 1], z - c[i, 2]))
            er = abs(out[i, n] - Cr[i])
            eb = abs(out[Q + i, n] - Cb[i])
            worst = max(worst, er, eb)
    say(f"  {len(samples)} nodes x 54 populations: max |gpu - oracle| = {worst:.3e} (max |f| = {fmax:.3f})")
    assert worst <= 2e-6 * fmax
