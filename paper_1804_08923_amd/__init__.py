"""MI355X-native colour-gradient D3Q27 central-moment lattice Boltzmann step
(Saito et al., arXiv:1804.08923): HIP kernels behind the C ABI of
include/cglbm.h, with a thin ctypes binding (:mod:`.lbm`)."""
from .workloads import Problem, WORKLOADS  # noqa: F401
