"""Pins of the diagnostics oracle (Sec. IV C fragment procedure) on fields
whose components are known by construction."""
import numpy as np

from oracle.diagnostics import equivalent_diameter, jet_diagnostics, mass_median_diameter


def _field(nx, ny, nz):
    return -np.ones((nz, ny, nx))


def test_boxes_and_column():
    nx, ny, nz = 12, 10, 20
    f = _field(nx, ny, nz)
    f[0:6, 4:6, 4:6] = 1.0          # column from the inlet plane: 6 x 2 x 2 = 24
    f[8:11, 1:3, 1:4] = 0.5          # box of 3 x 2 x 3 = 18
    f[15, 7, 9] = 0.1                # single cell
    f[14:16, 2:4, 8:9] = 1.0         # 2 x 2 x 1 = 4, touches nothing else
    stats, vol = jet_diagnostics(f.ravel(), nx, ny, nz)
    assert stats == dict(jet_nodes=24 + 18 + 1 + 4, front_z=15, column_volume=24, n_fragments=3)
    assert vol.tolist() == [18, 4, 1]


def test_face_connectivity_only():
    # cells touching along an edge or a corner are separate components
    nx = ny = nz = 6
    f = _field(nx, ny, nz)
    f[2, 2, 2] = f[3, 3, 2] = f[4, 4, 4] = 1.0     # edge- and corner-adjacent pairs
    f[2, 2, 3] = 1.0                               # face neighbour of the first
    stats, vol = jet_diagnostics(f.ravel(), nx, ny, nz)
    assert stats["n_fragments"] == 3 and vol.tolist() == [2, 1, 1]


def test_no_wrap_around_and_zero_phi_is_not_jet():
    nx, ny, nz = 8, 5, 7
    f = _field(nx, ny, nz)
    f[3, 2, 0] = f[3, 2, nx - 1] = 1.0   # opposite x faces: two components
    f[5, 1, 3] = 0.0                      # phi = 0 is not the jet phase
    stats, vol = jet_diagnostics(f.ravel(), nx, ny, nz)
    assert stats["jet_nodes"] == 2 and stats["n_fragments"] == 2 and stats["front_z"] == 3
    empty, v0 = jet_diagnostics(_field(nx, ny, nz).ravel(), nx, ny, nz)
    assert empty == dict(jet_nodes=0, front_z=-1, column_volume=0, n_fragments=0) and v0.size == 0


def test_brute_force_components_on_random_fields():
    # a plain flood fill on small random fields gives the same volumes
    rng = np.random.default_rng(7)
    for _ in range(5):
        nx, ny, nz = 7, 6, 5
        f = np.where(rng.random((nz, ny, nx)) < 0.35, 1.0, -1.0)
        seen = np.zeros(f.shape, bool)
        frag, col = [], 0
        for z, y, x in zip(*np.nonzero(f > 0)):
            if seen[z, y, x]:
                continue
            stack, size, touches = [(z, y, x)], 0, False
            seen[z, y, x] = True
            while stack:
                c = stack.pop()
                size += 1
                touches |= c[0] == 0
                for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    n = (c[0] + dz, c[1] + dy, c[2] + dx)
                    if all(0 <= n[a] < f.shape[a] for a in range(3)) and f[n] > 0 and not seen[n]:
                        seen[n] = True
                        stack.append(n)
            if touches:
                col += size
            else:
                frag.append(size)
        stats, vol = jet_diagnostics(f.ravel(), nx, ny, nz)
        assert stats["column_volume"] == col and sorted(frag, reverse=True) == vol.tolist()


def test_equivalent_diameter_of_a_sphere_and_mass_median():
    # V = pi d^3 / 6 inverts exactly
    d = np.array([1.0, 2.5, 7.0])
    assert np.allclose(equivalent_diameter(np.pi * d ** 3 / 6), d, rtol=1e-14)
    # volumes 1, 1, 8: total 10, half = 5 lies in the largest fragment
    assert np.isclose(mass_median_diameter([1, 8, 1]), equivalent_diameter(8))
    # volumes 4, 4, 1, 1: cumulative (1, 2, 6, 10) reaches 5 at the first 4
    assert np.isclose(mass_median_diameter([4, 1, 4, 1]), equivalent_diameter(4))


def test_run_jet_mass_median_matches_the_oracle():
    from paper_1804_08923_amd.run_jet import mass_median
    rng = np.random.default_rng(3)
    for n in (1, 2, 5, 40):
        v = rng.integers(1, 500, size=n)
        assert np.isclose(mass_median(v), mass_median_diameter(v), rtol=1e-12)
    assert np.isnan(mass_median([]))
