"""FP64 CPU oracle for ODF generation.  TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU path
computes, written from the paper (Witzke et al. 2021, MPS-ATLAS):
populations (Sec. 2.1, App. A, App. E stage one), the line absorption
coefficient (Sec. 2.1, eq. l_nu_line), line pre-selection (Sec. 4.3, App. E),
the R = 500 000 grid (App. E, grid formula), and the ODF reduction
(Sec. 2.3: sort each bin ascending, split into sub-bins, geometric or
arithmetic mean; App. E stage three).

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library; the
only common input is the seeded workload generator, which holds no physics.
"""
from .constants import *  # noqa: F401,F403
from .physics import (point_state, stage_fractions, populations, line_quantities,  # noqa: F401
                      ionisation_equilibrium, electron_density, saha_ratios)
from .voigt import voigt_h  # noqa: F401
from .odf import (grid_size, grid_lambda_nm, fine_opacity, odf_reduce_bin, odf_point, odf,  # noqa: F401
                  fine_table_point, slab_fine_intensity, slab_odf_intensity)
