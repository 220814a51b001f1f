"""Plain CPU reference of the jet diagnostics of Sec. IV C (leading edge,
fragments).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The fragment procedure of Sec. IV C, step by step:
  1. binarise the order parameter: 1 for the jet phase, 0 elsewhere;
  2. connected components of the 1-cells are the fragments;
  3. the volume V of each;
  4. the equivalent spherical diameter d = (6 V / pi)^(1/3);
the continuous column from the nozzle is left out of the fragment list.  The
paper uses the mass-median diameter of the fragments as its size metric.

Readings (the same as the library's): the jet phase is phi > 0; components
are face-connected (6-neighbourhood) on the lattice without wrap-around, which
is the default structuring element of ``scipy.ndimage.label`` in three
dimensions; V counts lattice cells; the column is every component with a cell
on the inlet plane z = 0; the leading edge is the largest z of a jet cell.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def jet_diagnostics(phi: np.ndarray, nx: int, ny: int, nz: int):
    """``phi`` in node order (x fastest).  Returns (stats, fragment volumes
    sorted in descending order); stats as ``lbm_jet_diagnostics`` reports them."""
    jet = (np.asarray(phi).reshape(nz, ny, nx) > 0)                      # step 1
    labels, n = ndimage.label(jet)                                      # step 2 (6-connectivity)
    vol = np.bincount(labels.ravel(), minlength=n + 1)[1:]              # step 3
    column = np.zeros(n + 1, bool)
    column[np.unique(labels[0])] = True                                 # components on z = 0
    column = column[1:]
    zs = np.nonzero(jet.any(axis=(1, 2)))[0]
    stats = dict(jet_nodes=int(jet.sum()), front_z=int(zs.max()) if zs.size else -1,
                 column_volume=int(vol[column].sum()), n_fragments=int((~column).sum()))
    return stats, np.sort(vol[~column])[::-1].astype(np.int64)


def equivalent_diameter(volume):
    """d = (6 V / pi)^(1/3) (step 4)."""
    return np.cbrt(6.0 * np.asarray(volume, np.float64) / np.pi)


def mass_median_diameter(volumes) -> float:
    """The diameter below which half of the fragment mass (volume) lies: the
    smallest d_k (fragments sorted by size) whose cumulative volume reaches
    half of the total."""
    v = np.sort(np.asarray(volumes, np.float64))
    if v.size == 0:
        return float("nan")
    c = np.cumsum(v)
    k = int(np.searchsorted(c, 0.5 * c[-1]))
    return float(equivalent_diameter(v[k]))
