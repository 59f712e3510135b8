"""Plain FP64 CPU oracle of the third-order relativistic lattice Boltzmann
scheme (RLBD) of Mendoza, Karlin, Succi and Herrmann, and of the
second-order model of its Appendix A.

This package is TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library never does, and
it shares no code with the HIP path (the only common inputs are the seeded
field generators and the quadrature table, which is data).

Everything here is written for a reader holding the paper: each function
cites the section or equation it follows, and computes it in the paper's
order with numpy in float64, with no blocking, fusion or reordering beyond
the equations themselves.

Modules
  lattice      the discrete 4-momenta p_i and weights w_i (Sec. II C)
  basis        Table I, the orthonormal polynomials J_0..J_29
  equilibrium  Maxwell-Juttner moments and the projected equilibrium (Eqs. coeff, disc1)
  landau       the Landau-Lifshitz eigenproblem (Eq. eigenproblem)
  rlb          moments, collision, exact streaming, the time step (Eq. rlb:disc)
"""
from .lattice import Lattice, load_lattice, model_lattice, default_table_path  # noqa: F401
from . import basis, equilibrium, landau, rlb  # noqa: F401
