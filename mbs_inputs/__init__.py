"""Seeded synthetic inputs for the modified Born series (MBS) Helmholtz solver.

This package only *generates* inputs (refractive-index media, sources, request
streams, workload descriptions).  It holds none of the method's arithmetic: no
wavenumber, no absorbing ramp, no scaling factor, no FFT of the method.  Both
the FP64 oracle and the HIP path receive the arrays it returns.
"""

from .generators import (  # noqa: F401
    WORKLOADS,
    Workload,
    gaussian_beam_source,
    plane_source,
    point_source,
    poisson_requests,
    smoothed_random_medium,
    source_tensor,
    sphere_medium,
    workload,
    workload_inputs,
)
