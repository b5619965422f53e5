"""Seeded synthetic inputs for the scenario-based absorber design NLP.

This package holds problem data only: the physical constants (``params.json``),
the per-scenario feed tables, the workload definitions and the problem-size
accounting.  It contains none of the solver's arithmetic and is the one module
that both the GPU path and the CPU oracle read.

Feed table layout (one row per scenario, ``NF = 18`` doubles, row-major):

====  ==========================================================
0     V_0     gas feed flow entering stage 1 from below [mol/s]
1-4   y_0     gas feed mole fractions (CO2, H2O, N2, O2)
5     T_gas   gas feed temperature [K]
6     L_in    lean-solvent flow entering stage N from above [mol/s]
7-15  x_in    lean-solvent mole fractions of the 9 liquid species
16    T_liq   lean-solvent temperature [K]
17    P       absorber pressure P_omega^abs [Pa]
====  ==========================================================
"""

from .scenarios import (  # noqa: F401
    NF,
    CONFIGS,
    N_BASE_CASES,
    base_cases,
    batch_problems,
    convex_combinations,
    dims,
    feed_table,
    load_params,
    perturbations,
)
