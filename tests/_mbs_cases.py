"""Shared helpers of the GPU tests: run the HIP path and the oracle on the same inputs."""

import math

import numpy as np

from mbs_inputs import workload, workload_inputs
from oracle import mbs_oracle as O


def rel_l2(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def random_case(shape, seed=0, n_min=1.0, n_max=1.5, sigma=2.0, src="point"):
    """Smoothed random medium and a point (or plane) source for a small grid."""
    from mbs_inputs import smoothed_random_medium, point_source, plane_source
    n = smoothed_random_medium(shape, seed, n_min, n_max, sigma)
    if src == "point":
        S = point_source(shape, (shape[0] // 3, shape[1] // 2, shape[2] // 2))
    else:
        S = plane_source(shape, min(shape[2] - 1, 5))
    return n, S


def gpu_solve(shape, split, periodic, t, n, S, k_vac, ramp_width, ramp_max, tol, max_iter,
              alpha=0.75, flags=0, check_every=0, x0=None):
    import torch
    from paper_2410_02395_amd import mbs
    dev = torch.device("cuda:0")
    nt = torch.from_numpy(np.ascontiguousarray(n, dtype=np.complex64)).to(dev)
    St = torch.from_numpy(np.ascontiguousarray(S, dtype=np.complex64)).to(dev)
    with mbs.Plan(shape, split, periodic, t, 1, alpha, flags, check_every) as plan:
        plan.set_medium(0, nt, k_vac, ramp_width, ramp_max)
        x0t = None if x0 is None else torch.from_numpy(np.ascontiguousarray(x0, np.complex64)).to(dev)
        out, res = plan.solve(0, St, tol, max_iter, x0=x0t)
        hist = plan.history(0)
        torch.cuda.synchronize()
        return out.cpu().numpy(), res, hist


def oracle_problem(shape, split, periodic, t, n, k_vac, ramp_width, ramp_max, alpha=0.75):
    return O.MBSProblem(shape, split, periodic, t, np.asarray(n, np.complex64), k_vac, ramp_width,
                        ramp_max, alpha=alpha)


__all__ = ["rel_l2", "random_case", "gpu_solve", "oracle_problem", "workload", "workload_inputs",
           "O", "math"]
