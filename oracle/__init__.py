"""Plain CPU FP64 oracle of the DGSEM right-hand side, its time stepping, the
finite-rate chemistry source and the discrete adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under this package: only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, tables or constant generators); the only code both
sides consume is the seeded input generators in ``dginputs``, which hold none of
the method's arithmetic.

Every routine is written for a reader holding the paper: plain torch-CPU float64,
vectorised over elements, explicit Python loops over directions, faces and
reactions, and a citation of the passage it follows.  Where the paper is silent,
the reading taken is stated in the docstring.

Parity status of each part (what pins it, outside itself) is listed in the
module docstrings; the one part without an external pin is the absolute value of
a general RHS node, which is fixed only by the readings of the discretisation.
"""

from .refelem import gll, mortar_matrices, lagrange_eval  # noqa: F401
from .mesh import Mesh, cartesian_mesh  # noqa: F401
