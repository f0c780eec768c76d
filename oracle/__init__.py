"""Plain FP64 / complex128 CPU oracle of block GCRO-DR (block recycled GMRES).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library.
"""
from .bgcrodr import (  # noqa: F401
    qr_pos, block_arnoldi_cycle, harmonic_ritz_first, harmonic_ritz_augmented, ritz_augmented,
    select_ritz, refresh_first, refresh_augmented, recycle_import, solve, solve_sequence,
    splitmix64, enlarging_vectors, apply_projected,
)
from .ilu import ilu0, apply_inverse, right_preconditioned  # noqa: F401
