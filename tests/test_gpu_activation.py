"""Subdomain activation (Sec. 3.1, end) on the GPU.

Subdomains without source start idle and join once the field their iterated
neighbours transfer into them exceeds a threshold.  The iteration converges to
the same fixed point from any start, so activation is checked at convergence:
the field agrees with the solve that iterates every subdomain throughout, its
full residual (every subdomain, evaluated by the library's unfused residual
path) meets the tolerance, and fewer subdomain-iterations were spent.  When the
source touches every subdomain nothing is skipped and the result is bitwise the
plain one.
"""

import math

import numpy as np
import pytest

from _mbs_cases import random_case, rel_l2

pytestmark = pytest.mark.gpu


def _solve(shape, split, periodic, t, n, S, k, tol, activation, flags=0, x0=None, check_every=8):
    import torch
    from paper_2410_02395_amd import mbs
    dev = torch.device("cuda:0")
    nt = torch.from_numpy(np.ascontiguousarray(n, np.complex64)).to(dev)
    St = torch.from_numpy(np.ascontiguousarray(S, np.complex64)).to(dev)
    with mbs.Plan(shape, split, periodic, t, 1, 0.75, flags, check_every, activation=activation) as plan:
        plan.set_medium(0, nt, k, (4, 4, 4), 0.2)
        x0t = None if x0 is None else torch.from_numpy(np.ascontiguousarray(x0, np.complex64)).to(dev)
        out, res = plan.solve(0, St, tol, 20000, x0=x0t)
        full = plan.residual(0, out)
        torch.cuda.synchronize()
        return out.cpu().numpy(), res, full


def test_activation_converges_to_the_same_field_with_fewer_subdomain_iterations():
    shape, split, periodic, t = (64, 32, 128), (2, 1, 2), (0, 0, 0), 8
    n, _ = random_case(shape, seed=21)
    S = np.zeros(shape, np.complex64)
    S[10, 16, 20] = 1                      # inside subdomain (0, 0, 0) only
    k = 2 * math.pi / 4
    tol = 1e-4
    xa, ra, fa = _solve(shape, split, periodic, t, n, S, k, tol, 0.0)
    xb, rb, fb = _solve(shape, split, periodic, t, n, S, k, tol, 1e-5)
    d = rel_l2(xb, xa)
    print(f"plain: {ra['iterations']} it, {ra['subdomain_iterations']} subdomain-it, full residual {fa:.2e}; "
          f"activation: {rb['iterations']} it, {rb['subdomain_iterations']} subdomain-it, full residual "
          f"{fb:.2e}; fields differ by {d:.2e}", flush=True)
    assert ra["converged"] == 1 and rb["converged"] == 1
    assert ra["subdomain_iterations"] == 4 * ra["iterations"]
    assert rb["subdomain_iterations"] < 4 * rb["iterations"]
    assert rb["iterations"] <= 1.2 * ra["iterations"]
    assert fb < 1.5 * tol
    assert d < 20 * tol


def test_activation_with_source_in_every_subdomain_changes_nothing():
    shape, split, periodic, t = (32, 32, 64), (2, 2, 2), (0, 0, 0), 4
    n, _ = random_case(shape, seed=22)
    S = np.zeros(shape, np.complex64)
    S[:, :, 31:33] = 1                     # a slab across the z interface: every subdomain holds source
    k = 2 * math.pi / 4
    xa, ra, _ = _solve(shape, split, periodic, t, n, S, k, 1e-4, 0.0)
    xb, rb, _ = _solve(shape, split, periodic, t, n, S, k, 1e-4, 1e-3)
    assert ra["iterations"] == rb["iterations"]
    assert rb["subdomain_iterations"] == 8 * rb["iterations"]
    assert np.array_equal(xa, xb)


def test_activation_with_a_start_field_iterates_every_subdomain():
    from paper_2410_02395_amd import mbs
    shape, split, periodic, t = (64, 32, 128), (2, 1, 2), (0, 0, 0), 8
    n, _ = random_case(shape, seed=23)
    S = np.zeros(shape, np.complex64)
    S[10, 16, 20] = 1
    k = 2 * math.pi / 4
    x0 = np.zeros(shape, np.complex64)
    xa, ra, _ = _solve(shape, split, periodic, t, n, S, k, 1e-4, 0.0, flags=mbs.MBS_X0_GIVEN, x0=x0)
    xb, rb, _ = _solve(shape, split, periodic, t, n, S, k, 1e-4, 1e-5, flags=mbs.MBS_X0_GIVEN, x0=x0)
    assert rb["subdomain_iterations"] == 4 * rb["iterations"]
    assert np.array_equal(xa, xb)
