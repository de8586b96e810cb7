"""Plain FP64 CPU oracle for the zero-centred MRT lattice Boltzmann sweep.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: it exists so that tests/, the smoke check in
__graft_entry__.smoke() and the cpu_baseline leg of bench.py can compare the HIP
kernels against the definitions of Hennig, Holzer and Ruede, "Advanced
Automatic Code Generation for Multiple Relaxation-Time Lattice Boltzmann
Methods" (arXiv 2211.02435).

The oracle evaluates the *dense* definitions of the paper, step by step, in
float64 numpy: the moment matrix M.f (section 2.3.1), the central-moment matrix
K(u).f (section 2.3.2), cumulants as derivatives of log M written out through
set partitions (section 2.3.3), the equilibria of section 2.4, the three
collision equations of section 2.2 (absolute, deviation-only, zero-centred with
absolute equilibrium) and explicit periodic streaming (eq. LbUpdateScheme).
It shares no code with the GPU path.

Parity status per function is listed in the header of lbm_oracle.py.
"""
from .lbm_oracle import *  # noqa: F401,F403
