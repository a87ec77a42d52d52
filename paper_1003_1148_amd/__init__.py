"""MI355X-native overdamped Langevin dynamics of the SOP protein model.

The compute path is the HIP library libsop.so (C ABI in include/sop.h);
this package holds its kernels (csrc/), its build script and a thin ctypes
binding.
"""
from ._sop import (  # noqa: F401
    Context,
    FORCES_PAIR,
    FORCES_PARTICLE,
    SopError,
    NTERMS,
    SCHEDULE_BATCHED,
    SCHEDULE_PLAIN,
    TERM_NAMES,
    LIB_PATH,
    declared_functions,
    from_system,
    lib,
    peak_force,
    ramp_params,
    ramp_run,
    ramp_run_static,
    RampParams,
    running_average,
    status_string,
    virial_temperature,
)
