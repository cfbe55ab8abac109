"""MI355X (gfx950) library for delayed approximate matrix assembly in
multigrid with dynamic precisions (Murray & Weinzierl, arXiv:2005.03606).

Thin Python binding over the C ABI in ``include/mgdelay.h``: argument
marshalling only, every step runs in the HIP kernels of ``libmgdelay.so``.
PyTorch supplies device memory and streams.  Importing this package does not
load the library; the first call does, and raises if it is missing.
"""
from .binding import (  # noqa: F401
    OK, EINVAL, ENOMEM, EHIP, ENOCONV, EDIVERGED, ESTARVED,
    FP64, MIXED, GEOMETRIC, BOXMG, STATIONARY, PCG, UPFRONT, LAZY,
    PUBLISH_ASYNC, PUBLISH_DETERMINISTIC, PUBLISH_EVERY, STORE_AUTO, STORE_DECODE, STORE_COPY,
    START_CARRY, START_BEST, CYCLE_V, CYCLE_ADAFAC_PI, CYCLE_ADAFAC_JAC,
    MgdError, Context, Eps, Hierarchy,
    assemble_cells, ladder_step_keep, p3_encode, centre_samples, gather_stencils, solve, solve_opts,
    solve_footprint, Server,
    n_half, n_pairs, lib, library_path,
)
