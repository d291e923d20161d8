"""MI355X-native Path Integral Monte Carlo transition amplitudes (SPEEDUP method, Balaz et al.).

The computation runs in the HIP library ``libpimc.so`` (C ABI in ``include/pimc.h``); this package
only marshals arguments to it. Importing the package does not load the library; the first call
does, and raises ``PimcLibraryMissing`` if it has not been built (``python -m
paper_1105_0542_amd.build``). There is no CPU fallback.
"""
from .binding import (  # noqa: F401
    FLAG_FP32_POLY, FLAG_HIERARCHY, FLOW_NPARAM, Batch, Context, Flow, LevelResult, PimcError, PimcLibraryMissing,
    check_problem, level_table, level_table_mpt, level_table_poly, level_table_radial, lib_path, load_library,
    make_tasks, poly_potential, potential_from_coefs, quartic, radial_potential,
)
