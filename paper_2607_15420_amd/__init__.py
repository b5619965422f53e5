"""MI355X (gfx950) interior-point solver for the scenario-based equilibrium
CO2-absorber diameter-minimisation NLP (paper eq. 10).

The compute path is the HIP library ``libabsorber.so`` (C ABI declared in
``include/absorber.h``); this package only marshals arguments to it.  Importing
the package does not load the library; the first call does, and fails loudly if
it has not been built (``python -m paper_2607_15420_amd.build``).
"""

from .binding import (  # noqa: F401
    ABS_OK,
    ERRORS,
    Absorber,
    AbsorberError,
    IpmOptions,
    IpmResult,
    Mlp,
    MlpTrainOptions,
    absorber_create,
    lib,
    params_struct,
)
