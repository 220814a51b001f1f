"""Readers for the text fixtures in tests/golden/ (values printed in the paper)."""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for ln in fh:
            if ln.startswith("#") or not ln.strip():
                continue
            out.append([e.strip() for e in ln.rstrip("\n").split(" ; ")])
    return out


def int_matrix(name):
    return np.array([[int(e) for e in r] for r in _rows(name)], dtype=np.float64)


def poly_matrix(name, u):
    """Evaluate a fixture of polynomial entries in ux, uy, uz at velocity u."""
    env = {"ux": float(u[0]), "uy": float(u[1]), "uz": float(u[2]), "__builtins__": {}}
    rows = _rows(name)
    return np.array([[eval(compile(e, name, "eval"), env) for e in r] for r in rows])


def laplace_table():
    """Table I: (gamma, sigma_th, sigma_Lap, E%, |u|max) rows."""
    out = []
    with open(os.path.join(GOLDEN, "table1_laplace.txt")) as fh:
        for ln in fh:
            if ln.startswith("#") or not ln.strip():
                continue
            out.append([float(v) for v in ln.split()])
    return np.array(out)


assert math  # keep import for eval environments that may need it
