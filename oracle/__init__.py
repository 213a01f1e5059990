"""FP64 CPU oracle for the Dirac matrix times a block of N_v vectors.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything here; only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do.  The oracle shares no code, table or constant with the GPU
library: the only common dependency is the seeded input generator module
``synthetic``, which holds none of the operators' arithmetic.

Everything is plain numpy in complex128, written from the definitions of
S. Duerr, "Three Dirac operators on two architectures with one piece of code and
no hassle" (LATTICE 2018):

* ``lattice``  -- coordinates, periodic shifts, staggered phases (Sec. 3)
* ``gamma``    -- Euclidean chiral gamma basis (the paper fixes none)
* ``staggered``-- D_S (Sec. 3, the D_S equation)
* ``wilson``   -- D_W at c_SW=0 (Sec. 4, eq. def_wils with its 2-point
                  derivative and 9-point Laplacian)
* ``brillouin``-- off-axis links W (Tab. 1) and D_B at c_SW=0 (Sec. 5,
                  eqs. def_bril, def_der, def_lap)
* ``dense``    -- brute-force dense matrices built entry by entry from the
                  delta-function forms, independently of the shift-based code
* ``grad``     -- link gradient of L = Re sum chi^dag D psi, and finite
                  differences (the paper is silent on gradients)
* ``solver``   -- CG on the normal equations and defect correction in FP64
                  (the paper is silent on solvers)
* ``local``    -- the same operators evaluated at a sample of sites only, by
                  explicit neighbour gathers, for lattices too large to apply
                  in full on the host

Pins (tests marked ``not gpu``) tie every function to closed forms, invariants
or brute force; see the test modules ``tests/test_oracle_*.py``.
"""
from . import lattice, gamma, staggered, wilson, brillouin, dense, grad, solver, local  # noqa: F401
