"""MI355X-native steady-state solver for optomechanical Lindblad systems.

The method (Nation, Johansson, Blencowe, Rimberg): the Liouvillian of the
driven optomechanical system in the Fock basis, the trace-constrained linear
system for vec(rho_ss), reverse Cuthill-McKee reordering, a dual-threshold
incomplete-LU preconditioner and restarted GMRES.  All numerical work runs in
libomss.so (HIP kernels for gfx950 plus host C++); this package only
marshals arguments.
"""
from ._lib import LibraryMissing, OmError, lib  # noqa: F401
from .api import (Csr, GmresOpts, Ilu, csr_permute, csr_spmv, gmres_solve, host_ilut, host_rcm,  # noqa: F401
                  ilu_apply, ilu_factor, liouvillian_apply, liouvillian_build, objective_vectors, observables,
                  param_gradient,
                  rcm_permute, steady_state)
from .autograd import SolveConfig, SteadyStateObs  # noqa: F401,E402
