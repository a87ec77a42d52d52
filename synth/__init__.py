"""Seeded synthetic SOP workloads shared by the oracle tests and the GPU path.

This package only builds inputs: C-alpha traces, chain topologies (backbone
bonds and native contacts with their reference distances), protocol settings
and run parameters.  It contains none of the force-field, pair-list, random
number or integrator arithmetic of the method; both the FP64 oracle and the
HIP library receive what it produces as plain arrays.
"""
from .structures import (  # noqa: F401
    System,
    RunParams,
    KB_KCAL,
    default_params,
    saw_batch,
    saw_confined,
    topology_from_chains,
    make_config,
    CONFIG_NAMES,
)
