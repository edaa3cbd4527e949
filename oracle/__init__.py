"""CPU oracle for the multiscale two-component D3Q19 lattice-Boltzmann step.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never imports,
links or calls it, and it shares no code with the GPU library: it is a plain
fp64 numpy transcription of the method (paper, Sec. II, Eqs. (1)-(7)), written
for a reader to check by eye, with no blocking, fusion or reordering.

Pins (see tests/test_oracle_*.py): lattice identities; moments of the
equilibrium, force term and Hermite projection; exact mass conservation with
residual events; momentum conservation of the pseudo-potential force;
uniform-Darcy steady state (scalar and tensorial); Poiseuille flow with
halfway bounce-back; Brinkman channel convergence; Laplace's law; the
flat-interface capillary jump; J-scaling and residual-saturation closed forms;
tensor reductions; brute-force nested-loop equality on tiny grids; open x
faces (a reservoir at the rest state is neutral, steady pressure-driven flow
conserves mass through every plane and is Poiseuille-shaped); the single-phase
permeability run (uniform acceleration of an open box, the exact discrete
permeability of a BGK slit).

Parity unpinned: the coupled transient of the two-component dynamics with CSF,
capillary and residual terms acting together has no closed form; it is bounded
only by the invariants above.
"""
from .lattice import C, W, OPP, Q, CS2
from .model import Oracle
from .constitutive import lerp_table, crossing, gray_parameters
from .tensor import inverse_permeability, smooth_periodic, gradient_hessian, principal_axes

__all__ = ["C", "W", "OPP", "Q", "CS2", "Oracle", "lerp_table", "crossing", "gray_parameters",
           "inverse_permeability", "smooth_periodic", "gradient_hessian", "principal_axes"]
