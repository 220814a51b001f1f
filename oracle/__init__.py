"""Plain CPU reference of the colour-gradient D3Q27 central-moment LBM step.

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; the product package never imports it.
"""
from .oracle import Oracle, OrParams, build_oracle, load_oracle, make_params  # noqa: F401
