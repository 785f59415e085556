"""Convergence studies of Sec. 4.2 on the GPU, with seeded synthetic media.

``truncation``: one periodic domain against the same domain split in two along x
(cyclic neighbours), for several truncations t of the correction blocks
(Sec. 4.2.1, Fig. 7): relative error of the decomposed field, iterations, time.

``subdomains``: the same medium split into P = 1, 2, 3, 4 subdomains along x
(Sec. 4.2.2, Fig. 8): iterations and time to the tolerance.  P = 1 is the
periodic single domain (a_x = 0); every P >= 2 has a_x = 2 and so the same c
(Eq. 9).

``decomposition``: the 512^3 workload (random medium, Gaussian beam, absorbing
layers) solved as 2x2x2 subdomains and as one domain with the same boundaries
(wrap-around removed on every axis, Sec. 4.1), both to the tolerance: the
fields differ by the truncation error of the interfaces.

The medium stands in for the paper's random sphere packings (not available):
smoothed seeded noise with n in [1, 1.33] and Im n = 0.01, the paper's indices,
at 4 points per wavelength; a point source.  Run as
``python -m paper_2410_02395_amd.studies truncation`` (or ``subdomains``); one
JSON line per study.
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import torch

from . import mbs


def _medium(shape, seed, device):
    from mbs_inputs import smoothed_random_medium
    n = smoothed_random_medium(shape, seed, 1.0, 1.33, sigma=2.0, device=device)
    return n + 0.01j


def _source(shape, device):
    S = torch.zeros(shape, dtype=torch.complex64, device=device)
    S[shape[0] // 4, shape[1] // 2, shape[2] // 2] = 1
    return S


def _run(plan, S, tol, max_iter, tag):
    """Solve on slot 0, reporting the iteration count of a long solve every 20 s."""
    out = torch.empty(plan.shape, dtype=torch.complex64, device=S.device)
    torch.cuda.synchronize()
    t0 = last = time.perf_counter()
    plan.solve_async(0, S, tol, max_iter, out)
    while True:
        res = plan.poll(0)
        if res is not None:
            break
        now = time.perf_counter()
        if now - last > 20.0:
            it, eps = plan.progress.get(0, (0, 0.0))
            print(f"[study] {tag}: iteration {it}, residual {eps:.3e}", file=sys.stderr, flush=True)
            last = now
        time.sleep(0.002)
    torch.cuda.synchronize()
    return out, res, time.perf_counter() - t0


def _solve(shape, split, t, n, S, k, tol, max_iter):
    with mbs.Plan(shape, split, (1, 1, 1), t, 1, 0.75, 0, 50) as plan:
        plan.set_medium(0, n, k)
        return _run(plan, S, tol, max_iter, f"split {split} t={t}")


def truncation(shape=(256, 192, 192), ts=(1, 2, 4, 8, 12, 16), tol=1e-5, seed=7, max_iter=60000):
    dev = torch.device("cuda:0")
    k = 2 * math.pi / 4
    n = _medium(shape, seed, dev)
    S = _source(shape, dev)
    ref, rref, tref = _solve(shape, (1, 1, 1), 8, n, S, k, tol, max_iter)
    rows = [{"split": [1, 1, 1], "t": None, "iterations": rref["iterations"], "seconds": round(tref, 3),
             "rel_residual": rref["rel_residual"]}]
    print(f"[study] single domain: {rows[-1]}", file=sys.stderr, flush=True)
    nr = torch.linalg.vector_norm(ref)
    for t in ts:
        x, r, dt = _solve(shape, (2, 1, 1), t, n, S, k, tol, max_iter)
        err = float(torch.linalg.vector_norm(x - ref) / nr)
        rows.append({"split": [2, 1, 1], "t": t, "iterations": r["iterations"], "seconds": round(dt, 3),
                     "rel_residual": r["rel_residual"], "rel_error": err, "squared_rel_error": err * err})
        print(f"[study] t={t}: {rows[-1]}", file=sys.stderr, flush=True)
        del x
    return {"study": "truncation (Sec. 4.2.1, Fig. 7)", "shape": list(shape), "tol": tol, "ppw": 4,
            "medium": "smoothed noise n in [1, 1.33] + 0.01i, seed %d" % seed, "rows": rows}


def subdomains(shape=(384, 128, 128), parts=(1, 2, 3, 4), t=8, tol=1e-5, seed=7, max_iter=60000):
    dev = torch.device("cuda:0")
    k = 2 * math.pi / 4
    n = _medium(shape, seed, dev)
    S = _source(shape, dev)
    rows = []
    ref = None
    for P in parts:
        x, r, dt = _solve(shape, (P, 1, 1), t, n, S, k, tol, max_iter)
        row = {"split": [P, 1, 1], "iterations": r["iterations"], "seconds": round(dt, 3),
               "ms_per_iteration": round(1e3 * dt / max(1, r["iterations"]), 4), "c_imag": r["c_imag"],
               "rel_residual": r["rel_residual"]}
        if ref is None:
            ref = x
        else:
            row["rel_difference_from_P1"] = float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref))
            del x
        rows.append(row)
        print(f"[study] P={P}: {row}", file=sys.stderr, flush=True)
    return {"study": "number of subdomains (Sec. 4.2.2, Fig. 8)", "shape": list(shape), "t": t, "tol": tol,
            "ppw": 4, "medium": "smoothed noise n in [1, 1.33] + 0.01i, seed %d" % seed, "rows": rows}


def decomposition(name="dd512", tol=1e-4, ts=(4, 8, 16), max_iter=40000):
    from mbs_inputs import smoothed_random_medium, source_tensor, workload
    w = workload(name)
    dev = torch.device("cuda:0")
    n = smoothed_random_medium(w.shape, w.medium["seed"], w.medium["n_min"], w.medium["n_max"],
                               sigma=w.ppw / 2.0, device=dev)
    S = source_tensor(w, dev)
    # interior: the grid without its absorbing layers
    r = [slice(w.ramp_width[d], w.shape[d] - w.ramp_width[d]) for d in range(3)]
    rows = []
    for t in ts:
        fields = []
        for split in (w.split, (1, 1, 1)):
            with mbs.Plan(w.shape, split, w.periodic, t, 1, w.alpha, 0, 50) as plan:
                plan.set_medium(0, n, w.k_vac, w.ramp_width, w.ramp_max)
                out, res, dt = _run(plan, S, tol, max_iter, f"split {split} t={t}")
                full = plan.residual(0, out)
            rows.append({"split": list(split), "t": t, "iterations": res["iterations"], "seconds": round(dt, 3),
                         "rel_residual": res["rel_residual"], "full_residual": full, "c_imag": res["c_imag"]})
            fields.append(out)
            print(f"[study] {rows[-1]}", file=sys.stderr, flush=True)
        a_, b_ = fields
        d = float(torch.linalg.vector_norm(a_ - b_) / torch.linalg.vector_norm(b_))
        di = float(torch.linalg.vector_norm((a_ - b_)[r[0], r[1], r[2]]) /
                   torch.linalg.vector_norm(b_[r[0], r[1], r[2]]))
        rows[-2]["rel_l2_difference"] = d
        rows[-2]["rel_l2_difference_interior"] = di
        print(f"[study] t={t}: decomposed vs one domain: rel L2 {d:.3e}, interior {di:.3e}", file=sys.stderr,
              flush=True)
        del fields, a_, b_
    return {"study": "decomposed against undecomposed (Sec. 4.1)", "workload": name, "shape": list(w.shape),
            "periodic": list(w.periodic), "ramp": list(w.ramp_width), "tol": tol, "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("study", choices=("truncation", "subdomains", "decomposition"))
    ap.add_argument("--tol", type=float, default=None)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.study == "truncation":
        out = truncation(tol=args.tol or 1e-5)
    elif args.study == "subdomains":
        out = subdomains(tol=args.tol or 1e-5)
    else:
        out = decomposition(tol=args.tol or 1e-4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
