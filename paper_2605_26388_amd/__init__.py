"""MI355X-native DGSEM right-hand-side library (paper arXiv 2605.26388, MARUT).

The computation lives in libdg.so (HIP kernels for gfx950 behind the C ABI of
include/dg.h); this package is its thin binding.  Build it with
`python -m paper_2605_26388_amd.build`.
"""

from ._abi import DGError, load  # noqa: F401
from .solver import Solver, mechanism_struct  # noqa: F401
from .rollout import DGRollout  # noqa: F401
