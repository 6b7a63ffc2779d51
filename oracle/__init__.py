"""CPU oracle for Multipole-Accelerated Hamiltonian Interpolation (MAHI).

TEST INFRASTRUCTURE.  This package computes, slowly and in float64, the exact
Hamiltonian-interpolation (HI) energy, atom forces, per-form derivatives
dE/dlambda-tilde and per-form charge derivatives, straight from the paper's
general formulation (Theory, "Hamiltonian Interpolation Formulation", eq
iter_ham_lambda) and, for tiny inputs, from the enumeration of all
sub-Hamiltonians (eq rek_ham_lambda and its appendix).  It shares no code with
the GPU library and must only be imported by the tests, by the smoke check and
by the benchmark's CPU-baseline leg.

Modules:
  kernels  pair kernels: open-boundary Coulomb and periodic Ewald (dense, small N)
  ewald    ctypes wrapper of ewald.c (potential and field at targets; pair kernel)
  hi       HI energy, forces, dE/dlambda-tilde and dE/dq from the general formulation
  brute    enumeration of all site-form combinations (tiny inputs only)
  lmap     lambda -> lambda-tilde transform and the back-map of derivatives (Appendix)
"""
from .hi import evaluate, hi_dense, hi_periodic  # noqa: F401
