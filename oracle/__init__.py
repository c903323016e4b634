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
           Riemann solution of the Euler equations, oblique-shock relations, the
           Chapman-Jouguet and von Neumann states, and Gauss-Hermite moments of
           the continuous Maxwellian.

What pins each function (tests/test_oracle_pins.py, checked against the paper or
the mathematics, never against the oracle itself):

  velocity_set          geometry of the three 8-velocity groups
  moment_matrix,        exact rational inverse; M^-1 M = I; equilibrium recovery
  inverse_moment_matrix
  equilibrium_moments   Gauss-Hermite moments of the continuous Maxwellian (all 24
                        rows); the printed rows 14/16 without T fail that check
  macroscopic           equilibrium recovery; a uniform state is a fixed point
  collision             mass, momentum and energy conservation; closed-form decay
                        (1 - R_k dt)^n of every non-conserved moment (pins forward
                        Euler and the R-to-moment mapping)
  collision_srt         one SRT step with tau equals one MRT step with every R_k =
                        1/tau (A_hat then vanishes; an identity of Eqs. SRT and MRT);
                        closed-form decay (1 - dt/tau)^n of every component of f - f^eq
  wall_layers, padded   reflecting walls pass no mass, energy or tangential momentum
                        (exact flux cancellation at the wall face); Dirichlet and
                        co-moving extrapolation walls keep a uniform state; the first
                        step under a moving extrapolation wall transfers exactly the
                        half-range flux of the equilibria; the shock-reflection states
                        (physics.oblique_shock reproduces the paper's incident shock)
  modification_terms    its sign: only the chosen sign makes the viscous heating
                        independent of R_8 (Chapman-Enskog, Sec. III), in a 1D wave and,
                        with the 1/R_8 part extrapolated away, in a 2D shear flow where
                        the shear term of A_hat_8 and every term of A_hat_9 are non-zero;
                        the exchange of the x and y axes maps solutions to solutions
                        (A_hat_9 is A_hat_8 mirrored, term by term); planted mistakes (a
                        dropped shear term, an exchanged derivative, a wrong velocity
                        factor) fail these
  cochran_increment     exact solution of the rate equation (against a fine RK4);
                        homogeneous heating 2 Q dlambda / (D + I)
  chemical_term         moments k = 1..9 equal the printed C_hat (Sec. II); for each
                        of the 24 velocities C_i / f^eq_i equals (2 Q F / (D+I)) times
                        the temperature derivative of log Eq. feq_continuous at
                        (v_i, eta_i) (Eqs. M_chemical_2, M_chemical_feq), which fixes the
                        bracket for every moment; the energy budget on a periodic grid
  nnd_derivative,       exact on linear data, zero on constants, upwind, second
  streaming             order on smooth monotone data, mirror symmetry
  step, run, init_f     Sod (I = 3), Lax (I = 1) and Sjogren (I = 4) against the exact
                        Riemann solutions; the CJ plateau of a
                        detonation; shear-wave decay at the Chapman-Enskog
                        viscosity; the relaxed heat-flux moment Delta_8 of a
                        temperature wave equals -2 kappa dT/dx with the conductivity
                        of Sec. III (pins R_8/R_9, c_p and f_hat^eq rows 8 and 14);
                        the relaxed normal stresses Delta_5, Delta_7 of a longitudinal
                        wave equal the Chapman-Enskog stresses for I = 1, 3, 4;
                        conservation on periodic grids
  tne, reductions       readout identities (Sec. VI)
  ignition_margin       equals min |T - T_ig| of the temperature field a state was
                        initialised from (over the cells with lambda < 1), +inf
                        when every cell has burnt
  (reverse-mode AD)     the gradient of a run agrees with central differences of
                        the oracle's forward run
  physics.*             the paper's CJ numbers (tests/golden/cj_state.txt); Rankine-
                        Hugoniot jump conditions of the exact Riemann solution

Inputs that no pin can fix: the Cochran rate constants omega_1, omega_2 (never
printed; a project choice of the workloads).
"""

from .dvm import DVM, velocity_set, moment_matrix, inverse_moment_matrix
from .model import Params, Tables, make_tables, equilibrium_moments, macroscopic, \
    modification_terms, cochran_increment, chemical_term, nnd_derivative, \
    collision, collision_srt, step, run, init_f, moments, tne, reductions, ignition_margin, wall_layers, \
    padded

__all__ = [
    "DVM", "velocity_set", "moment_matrix", "inverse_moment_matrix",
    "Params", "Tables", "make_tables", "equilibrium_moments", "macroscopic",
    "modification_terms", "cochran_increment", "chemical_term", "nnd_derivative",
    "collision", "step", "run", "init_f", "moments", "tne", "reductions", "ignition_margin",
]
