"""Reference (oracle) implementation of the MRT lattice Boltzmann kinetic model
for combustion (Xu, Lin, Zhang, Li, arXiv:1411.6697).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, obviously correct
CPU implementation in float64 (NumPy for set-up, PyTorch CPU tensors for the
field arithmetic) written from the paper's equations.  Only the test-suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  The
GPU library never calls into it, and it never calls into the GPU library:
the two share no code.

Modules
-------
dvm      : the D2V24 discrete-velocity model, the moment matrix M and an
           exactly-computed, correctly-rounded inverse (Sec. II).
model    : equilibrium moments, modification terms, chemistry, NND streaming,
           one forward-Euler time step, initialisation and the TNE readouts
           (Sec. II, Sec. VI).
physics  : independent physics references used to pin the model: the exact
           Riemann solution of the Euler equations, the Chapman-Jouguet and
           von Neumann states, and Gauss-Hermite moments of the continuous
           Maxwellian.

Parity status of each function is stated in its docstring.
"""

from .dvm import DVM, velocity_set, moment_matrix, inverse_moment_matrix
from .model import Params, Tables, make_tables, equilibrium_moments, macroscopic, \
    modification_terms, cochran_increment, chemical_term, nnd_derivative, \
    collision, step, run, init_f, moments, tne, reductions

__all__ = [
    "DVM", "velocity_set", "moment_matrix", "inverse_moment_matrix",
    "Params", "Tables", "make_tables", "equilibrium_moments", "macroscopic",
    "modification_terms", "cochran_increment", "chemical_term", "nnd_derivative",
    "collision", "step", "run", "init_f", "moments", "tne", "reductions",
]
