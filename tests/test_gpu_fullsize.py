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


def _ulp16(v, storage):
    """Spacing of the 16-bit storage format at |v| (BF16: 8 significant bits,
    FP16: 11, with FP16's subnormal spacing 2^-24 as the floor)."""
    a = np.maximum(np.abs(v), 1e-30)
    e = np.floor(np.log2(a))
    if storage.startswith("bf16"):
        return 2.0 ** (e - 7)
    return np.maximum(2.0 ** (e - 10), 2.0 ** -24)


def _stored_general_state(torch, storage, fr, fb, rr_field, rb_field, w, rho_b0):
    """The populations the library decodes from the general state it writes
    from fields (k_init): d = f - w rho_b0 formed in FP64, rounded to FP32 and
    then to the storage format; the node's minority colour (rho_r > rho_b in
    the given fields picks blue) stored the same way; the other colour formed
    as (d + w rho_b0) - f^k in FP64 and rounded to FP32."""
    def enc(x):
        x32 = torch.from_numpy(np.ascontiguousarray(x, np.float64).astype(np.float32))
        if storage == "fp32":
            return x32.numpy().astype(np.float64)
        tdt = torch.bfloat16 if storage.startswith("bf16") else torch.float16
        return x32.to(tdt).float().numpy().astype(np.float64)
    d = enc((fr + fb) - w[:, None] * rho_b0)
    blue = (rr_field > rb_field)[None, :]
    fk = enc(np.where(blue, fb, fr))
    fo = ((d + w[:, None] * rho_b0) - fk).astype(np.float32).astype(np.float64)
    return np.where(blue, fo, fk), np.where(blue, fk, fo)


@pytest.mark.parametrize("workload,storage", [
    ("jet-ft-fine-480x480x1200", "fp32"), ("jet-ft-fine-480x480x1200", "bf16"),
    ("jet-256x256x1024", "bf16"), ("jet-128x128x512", "fp16")])
def test_fields_init_sampled_step(torch, orc, workload, storage):
    """One step from a state the library builds from fields (LBM_INIT_FIELDS),
    at full size in the launch configuration bench.py times, with 16-bit
    storage and on the 480x480x1200 lattice of the paper's fine FT jet (279 M
    padded nodes, above 2^28: the 64-bit offsets of the 16-byte records).
    Sampled interior nodes: every streamed population of both colours against
    the oracle's node update of its source node, the oracle starting from the
    populations the storage format holds (the codec is pinned bit for bit in
    test_gpu_storage).  Bar: FP32 arithmetic, 2e-6 of max |f|; with 16-bit
    storage plus one spacing of the format at the stored deviation."""
    from synth import separable_state_fields

    from paper_1804_08923_amd.lbm import LBM
    from paper_1804_08923_amd.workloads import WORKLOADS, Problem
    prob = WORKLOADS[workload]().replace(storage=storage, init="fields")
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    say(f"fields-init step {workload} {storage}: building fields")
    rr, rb, u = separable_state_fields(prob, seed=77)
    rng = np.random.default_rng(9)
    # corners of the sampled region, tile edges (128-node rows), random nodes
    samples = [(2, 2, 2), (nx - 3, ny - 3, nz - 3), (nx // 2, ny // 2, nz // 2), (nx - 3, 2, nz // 3),
               (min(129, nx - 3), min(130, ny - 3), 131), (min(127, nx - 3), ny - 3, 7)]
    samples += [tuple(int(v) for v in (rng.integers(2, nx - 2), rng.integers(2, ny - 2), rng.integers(2, nz - 2)))
                for _ in range(18)]

    def nid(x, y, z):
        return (z * ny + y) * nx + x

    blocks = []
    for (x, y, z) in samples:
        zz, yy, xx = np.meshgrid(np.arange(z - 2, z + 3), np.arange(y - 2, y + 3), np.arange(x - 2, x + 3),
                                 indexing="ij")
        blocks.append(nid(xx, yy, zz).ravel())
    blk_fields = [(rr[b].astype(np.float64), rb[b].astype(np.float64), u[b].astype(np.float64)) for b in blocks]
    say(f"fields-init step {workload} {storage}: one GPU step")
    sim = LBM(prob, rho_r=rr, rho_b=rb, u=u)
    del rr, rb, u
    sim.step(1)
    st = sim.get_state()
    cols = torch.from_numpy(np.array([nid(*s) for s in samples], np.int64)).to(st.device)
    out = st[:, cols].cpu().numpy().astype(np.float64)
    del st
    sim.close()
    torch.cuda.empty_cache()

    say(f"fields-init step {workload} {storage}: oracle node updates")
    p = or_params(prob)
    small = Problem(name="blk", nx=5, ny=5, nz=5, bc="periodic", rho_r0=prob.rho_r0, rho_b0=prob.rho_b0,
                    alpha_b=prob.alpha_b, nu_r=prob.nu_r, nu_b=prob.nu_b, A=prob.A, g=prob.g)
    p5 = or_params(small)
    c, w = orc.lattice()
    c = np.asarray(c).reshape(Q, 3)
    w = np.asarray(w, np.float64)

    def bid(x, y, z):
        return (z * 5 + y) * 5 + x

    worst = 0.0
    fmax = np.abs(out).max()
    for k, (brr, brb, bu) in enumerate(blk_fields):
        fr5, fb5, _ = orc.init_fields(p5, brr, brb, bu)
        fr5, fb5 = _stored_general_state(torch, storage, fr5, fb5, brr, brb, w, prob.rho_b0)
        r5, b5, _, ph5 = orc.macroscopic(p5, fr5, fb5)
        rho5 = r5 + b5
        for i in range(Q):
            sx, sy, sz = 2 - c[i, 0], 2 - c[i, 1], 2 - c[i, 2]
            sten = [bid(sx + c[j, 0], sy + c[j, 1], sz + c[j, 2]) for j in range(Q)]
            m = bid(sx, sy, sz)
            Cr, Cb = orc.collide_node(p, prob.A, fr5[:, m], fb5[:, m], ph5[sten], rho5[sten])
            tol = 2e-6 * fmax
            if storage != "fp32":
                tol = tol + _ulp16(Cr[i] + Cb[i] - w[i] * prob.rho_b0, storage)
            er, eb = abs(out[i, k] - Cr[i]), abs(out[Q + i, k] - Cb[i])
            worst = max(worst, max(er, eb) / tol)
            assert er <= tol and eb <= tol, (samples[k], i, out[i, k], Cr[i], out[Q + i, k], Cb[i], tol)
    say(f"  {len(samples)} nodes x 54 populations: max error / bar = {worst:.3f}")
