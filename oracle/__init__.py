"""Oracle: a plain, slow, FP64 CPU implementation of the Shan-Chen D3Q19 lattice Boltzmann step
(arXiv:2105.08772, Sec. 2), its observables (Sec. 3, Sec. 4) and the equation of state (Eq. bulkp).

TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg
may import it. It shares no code with the HIP library in paper_2105_08772_amd/ and imports
nothing from it.

Modules:
  core      ctypes binding of lbm_oracle.c (the 3D step, force, pressure tensor, init)
  eos       bulk pressure, critical coupling, spinodals, leading-order coexistence rule
  reduced   independent D1Q3 / D2Q9 numpy lattices (reductions of D3Q19) and flat coexistence
  observe   mass, momentum, centre of mass, probes, profiles, sigma[R], R_s, R_e, sigma_0, du
"""
from . import core, eos, observe, reduced  # noqa: F401
from .core import build  # noqa: F401
