"""Throughput benchmark of the MBS iteration on one MI355X.

A step is one iteration of the modified Born series (Eq. 6 of the paper) over
every subdomain of the workload: edge corrections, the five FFT passes with the
fused pointwise work, the face update and the FP64 residual reduction.  The
default workload is the 1024^3 grid decomposed 2x2x2 into 512^3 subdomains
(planar source, 32-voxel absorbing ramps, t = 8), run for a fixed number of
iterations with all inputs already resident in HBM.

Prints one JSON line with whole-job voxel-updates/s, the roofline of the
dominant kernel (HIP events around every launch of the timed region) and a
bounded timing of the FP64 CPU oracle.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE on the dd1024 workload with the fused
# z pass, scaled by the same counters on a plain 2 GiB copy (FETCH factor 0.5, WRITE factor 1.0).
# Valid only for the kernel code they were taken on (sha256 of the source without its comments,
# kernel_code_digest); any other code reports traffic = null.
PMC_TRAFFIC = {
    "workload": "dd1024",
    "fused": True,
    "kernel_code_sha256": "f173a94caa19822e85f38b98cb1ee687098b189243fa8eb2e618e3c11f21e5b6",
    "bytes": {"z_fwd": 1.869e9, "yxy_slabs": 51.576e9, "z_inv": 39.272e9, "edge_corr": 2.685e9,
              "face": 3.100e9},
}
METRIC = "MBS voxel-updates/s + HBM GB/s at 1024³; served solves/s and p99 latency"


def kernel_code_digest():
    """sha256 of the kernel source with its // comments and blank lines left out: edits to the
    comments keep a counter record valid, any change to the code voids it."""
    import re
    src = os.path.join(ROOT, "paper_2410_02395_amd", "csrc", "mbs_kernels.hip")
    with open(src) as fh:
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in fh]
    code = "\n".join(ln for ln in lines if ln.strip())
    return hashlib.sha256(code.encode()).hexdigest()


def slab_elems(n, S, t, a, d):
    plane = n[1] * n[2] if d == 0 else (n[0] * n[2] if d == 1 else n[0] * n[1])
    return S * 2 * t * plane if a[d] else 0


def face_voxels(n, t, a):
    """Voxels per subdomain in the union of the t-deep edge slabs of corrected axes."""
    inner = 1
    for d in range(3):
        inner *= (n[d] - 2 * t) if a[d] else n[d]
    return n[0] * n[1] * n[2] - inner


def algorithmic_bytes(shape, split, periodic, t, src_box, fused=True, b_bytes=8):
    """Compulsory HBM bytes per iteration of each kernel kind for one slot.  ``b_bytes``: bytes of
    B per voxel, 8, or 4 for a lossless medium (Im n = 0: the library stores Im B only and rebuilds
    Re B from the absorbing ramp)."""
    b = b_bytes
    n = [shape[d] // split[d] for d in range(3)]
    S = split[0] * split[1] * split[2]
    a = [2 if split[d] >= 2 else (0 if periodic[d] else 1) for d in range(3)]
    V = S * n[0] * n[1] * n[2]
    slabs = sum(slab_elems(n, S, t, a, d) for d in range(3))
    fv = S * face_voxels(n, t, a)
    L = 2048 // n[2] if n[2] < 2048 else 1
    n_main = (S * n[0] * n[1] + L - 1) // L
    n_face = (fv + 255) // 256
    if fused:
        # x/y edge-slab lines (whole lines), per subdomain column
        in0 = n[0] - 2 * t if a[0] else n[0]
        in1 = n[1] - 2 * t if a[1] else n[1]
        SLV = S * (n[0] * n[1] - in0 * in1) * n[2]
        slabs01 = sum(slab_elems(n, S, t, a, d) for d in range(2))
        return {
            # w pass on the x/y edge-slab lines: read x, B, Ex_0/Ex_1; write W
            "z_fwd": (16 + b) * SLV + 8 * slabs01,
            "y_fwd": 16 * V,
            "x_green": 16 * V,
            "y_inv": 16 * V,
            # the same three passes run slab by slab (the slab stays in the memory-side cache
            # between them, so the algorithmic bytes are those of the three passes)
            "yxy_slabs": 48 * V,
            # fused z pass: read W, x, B (+ source box); write x, W (d on edge-slab lines),
            # the u values of the x/y edge slabs, partial sums
            "z_inv": (32 + b) * V + 8 * src_box + 8 * slabs01 + 8 * n_main,
            # twice per iteration (u, then x), axes 0 and 1: read the slab values, write the
            # corrections
            "edge_corr": 2 * 16 * slabs01,
            # edge-slab lines: read d, x, Eu_0/Eu_1; write x and the iterate's X_0/X_1 slabs
            "face": 24 * SLV + 16 * slabs01 + 8 * ((SLV + 255) // 256),
            "reduce": 8 * (n_main + (SLV + 255) // 256),
        }
    return {
        # read x, B (+ edge corrections, source box), write W
        "z_fwd": (16 + b) * V + 8 * slabs + 8 * src_box,
        "y_fwd": 16 * V,
        "x_green": 16 * V,
        "y_inv": 16 * V,
        # read W, x, B, write x (+ edge slabs of u, partial sums)
        "z_inv": (24 + b) * V + 8 * slabs + 8 * n_main,
        # twice per iteration (x, then u), every corrected axis: read the slab values, write the
        # corrections
        "edge_corr": 2 * 16 * slabs,
        # read corrections, u, B, x; write x and the iterate's edge slabs
        "face": 8 * (2 * slabs + 3 * fv) + b * fv + 8 * n_face,
        "reduce": 8 * (n_main + n_face),
    }


def cpu_baseline(n_dev, S_dev, w, iters=16, edge=256):
    """Time the FP64 oracle on a bounded sample: the first edge^3 block of the
    workload's medium and source, decomposed like the workload."""
    import numpy as np
    from oracle import mbs_oracle as O
    n = n_dev[:edge, :edge, :edge].cpu().numpy()
    S = S_dev[:edge, :edge, :edge].cpu().numpy()
    shape = (edge,) * 3
    pr = O.MBSProblem(shape, w.split, w.periodic, w.t, n, w.k_vac, w.ramp_width, w.ramp_max, alpha=w.alpha)
    y = pr.source_term(S)
    x = np.zeros(shape, np.complex128)
    t0 = time.perf_counter()
    for _ in range(iters):
        x, _ = pr.step(x, y)
    dt = time.perf_counter() - t0
    return {
        "value": edge ** 3 * iters / dt,
        "unit": "voxel-updates/s",
        "cores": O.WORKERS,
        "kind": "oracle",
        "sample": (f"{iters} iterations of the FP64 oracle on the first {edge}^3 block of the workload's "
                   f"medium and source, split {w.split[0]}x{w.split[1]}x{w.split[2]} like the workload "
                   f"(t={w.t}, ramp {w.ramp_width[0]}), {dt:.1f} s"),
    }


def make_requests(count, device):
    """The seeded Poisson stream of mixed-size solves with inputs generated on the device."""
    import torch
    from mbs_inputs import poisson_requests, smoothed_random_medium, source_tensor
    from paper_2410_02395_amd.serve import Request
    out = []
    for spec in poisson_requests(count):
        w = spec["workload"]
        n = smoothed_random_medium(w.shape, w.medium["seed"], w.medium["n_min"], w.medium["n_max"],
                                   sigma=w.ppw / 2.0, device=device)
        S = source_tensor(w, device)
        out.append(Request(spec["id"], spec["arrival"], w.shape, w.k_vac, n, S, w.ramp_width, w.ramp_max,
                           w.tol, w.max_iter))
    torch.cuda.synchronize()
    return out


def serving_bench(args):
    """Mixed-size stream: continuous batching vs one-at-a-time solves of the same requests."""
    import copy
    import torch
    from paper_2410_02395_amd.serve import Server, run_serial, summarize
    reqs = make_requests(args.requests, "cuda:0")
    print(f"[bench] {len(reqs)} requests generated", file=sys.stderr, flush=True)
    # warm up kernels and graphs of every shape once
    warm = [copy.copy(r) for r in {r.shape: r for r in reqs}.values()]
    for r in warm:
        r.out = None
    srv = Server(200e9)
    srv.run(warm, realtime=False)
    srv.close()
    report = {}
    for mode, realtime in (("poisson_20hz", True), ("saturating", False)):
        mix = [copy.copy(r) for r in reqs]
        ser = [copy.copy(r) for r in reqs]
        for r in mix + ser:
            r.out = None
        srv = Server(200e9)
        done_mix = srv.run(mix, realtime=realtime)
        srv.close()
        print(f"[bench] {mode}: batched done", file=sys.stderr, flush=True)
        done_ser = run_serial(ser, realtime=realtime)
        print(f"[bench] {mode}: serial done", file=sys.stderr, flush=True)
        same = sum(1 for a, b in zip(sorted(done_mix, key=lambda r: r.id), sorted(done_ser, key=lambda r: r.id))
                   if torch.equal(a.out, b.out))
        report[mode] = {"batched": summarize(done_mix), "serial": summarize(done_ser),
                        "bitwise_equal_results": same}
    mix = report["saturating"]["batched"]
    line = {
        "metric": METRIC,
        "value": mix["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 1,
        "ms_per_step": 1e3 / mix["solves_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"serving: {len(reqs)} seeded Poisson requests (20 req/s), cubic edges "
                                "{64,96,128,192,256}, 3-6 ppw, smoothed random media n in [1.0,1.4], point or "
                                "Gaussian-beam sources, tol 1e-4, 200 GB HBM budget; value = saturating replay")},
        "serving": report,
    }
    print(json.dumps(line), flush=True)


def stream_ceilings():
    """HBM rates of plain streams: the hand-written HIP streams of ``csrc/stream_ceilings.hip``
    (a child process, run before this process touches the GPU), then plain torch kernels over
    8 GiB complex64 arrays (best of 5)."""
    import subprocess
    from paper_2410_02395_amd.build import STREAM_CEILINGS, build_stream_ceilings
    if not os.path.exists(STREAM_CEILINGS):
        build_stream_ceilings()
    hip = []
    proc = subprocess.run([STREAM_CEILINGS], capture_output=True, text=True, timeout=300)
    if proc.returncode != 0:
        raise RuntimeError(f"stream_ceilings failed ({proc.returncode}): {proc.stderr.strip()}")
    for line in proc.stdout.splitlines():
        hip.append(json.loads(line))
        print(f"[bench] {hip[-1]}", file=sys.stderr, flush=True)
    import torch
    dev = torch.device("cuda:0")
    n = 1 << 30
    a = torch.ones(n, dtype=torch.complex64, device=dev)
    b = torch.ones(n, dtype=torch.complex64, device=dev)
    c = torch.ones(n, dtype=torch.complex64, device=dev)
    d = torch.empty(n, dtype=torch.complex64, device=dev)
    ar, br, cr, dr = (torch.view_as_real(t) for t in (a, b, c, d))
    cases = {
        "read": (lambda: torch.sum(ar), 8 * n),
        "write": (lambda: d.fill_(1.0), 8 * n),
        "copy (read 1, write 1)": (lambda: d.copy_(a), 16 * n),
        "addcmul (read 3, write 1)": (lambda: torch.addcmul(ar, br, cr, out=dr), 32 * n),
    }
    out = {}
    for name, (fn, nbytes) in cases.items():
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None or ms < best else best
        out[name] = {"ms": round(best, 4), "gbps": round(nbytes / (best * 1e-3) / 1e9, 1)}
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "HBM streaming ceilings", "unit": "GB/s", "hip_streams_2GiB": hip,
                      "torch_8GiB_complex64": out}), flush=True)


def tolerance_study(args, w, n, S, mbs):
    """Solve to a tolerance with every subdomain iterated and with subdomain activation
    (Sec. 3.1) at each threshold: iterations, subdomain-iterations, wall time, the full
    residual of each field (every subdomain) and its difference from the field of the run
    that iterates every subdomain."""
    import torch
    dev = n.device
    runs = {}
    ref = None
    taus = [0.0] + [float(x) for x in str(args.activation).split(",") if x]
    for act in taus:
        name = "all_subdomains" if act == 0.0 else f"activation_{act:g}"
        plan = mbs.Plan(w.shape, w.split, w.periodic, w.t, 1, w.alpha, 0, 50, activation=act)
        plan.set_medium(0, n, w.k_vac, w.ramp_width, w.ramp_max)
        out = torch.empty(w.shape, dtype=torch.complex64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve_async(0, S, args.tol, args.max_iter, out)
        last = t0
        while True:
            res = plan.poll(0)
            if res is not None:
                break
            now = time.perf_counter()
            if now - last > 20.0:  # a long solve reports how far it has come
                it, eps = plan.progress.get(0, (0, 0.0))
                print(f"[bench] {name}: iteration {it}, residual {eps:.3e}, {now - t0:.0f} s",
                      file=sys.stderr, flush=True)
                last = now
            time.sleep(0.002)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        full = plan.residual(0, out)
        plan.close()
        runs[name] = {"iterations": res["iterations"], "subdomain_iterations": res["subdomain_iterations"],
                      "seconds": round(dt, 3), "rel_residual": res["rel_residual"], "full_residual": full,
                      "converged": res["converged"]}
        if ref is None:
            ref = out
        else:
            runs[name]["field_rel_difference"] = float(torch.linalg.vector_norm(out - ref)
                                                       / torch.linalg.vector_norm(ref))
            del out
        print(f"[bench] {name}: {runs[name]}", file=sys.stderr, flush=True)
    best = min((r["seconds"] for k, r in runs.items() if k != "all_subdomains"), default=None)
    line = {
        "metric": "MBS solve to tolerance: wall time with and without subdomain activation",
        "value": runs["all_subdomains"]["seconds"] / best if best else None,
        "unit": "speed-up",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "shape": list(w.shape), "split": list(w.split), "tol": args.tol,
                   "activation": taus[1:]},
        "runs": runs,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="dd1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 2 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--stream-ceilings", action="store_true",
                    help="only measure plain streaming kernels over 8 GiB arrays (read, write, copy, "
                         "3 reads + 1 write): the HBM rates the iteration's byte mixes can reach")
    ap.add_argument("--serving", action="store_true",
                    help="run the mixed-size request-stream benchmark instead of the 1024^3 iteration")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--no-fusion", action="store_true",
                    help="separate last inverse and next forward z passes (for comparison)")
    ap.add_argument("--zblock", type=int, default=0,
                    help="z slab of the strided passes (0 automatic, -1 whole passes)")
    ap.add_argument("--tol", type=float, default=0.0,
                    help="solve the workload to this relative residual, with and without subdomain "
                         "activation, and report iterations and wall time instead of the fixed-count run")
    ap.add_argument("--max-iter", type=int, default=100000, help="iteration cap of the --tol study")
    ap.add_argument("--activation", default="1e-3",
                    help="comma-separated activation thresholds (relative to ||Gamma^-1 y||) of the "
                         "--tol study")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: every subdomain of the workload is resident on a single "
              f"MI355X; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from mbs_inputs import source_tensor, workload, workload_inputs
    from paper_2410_02395_amd import mbs

    if args.serving:
        serving_bench(args)
        return
    if args.stream_ceilings:
        stream_ceilings()
        return

    w = workload(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] workload {w.name} shape {w.shape} split {w.split}", file=sys.stderr, flush=True)
    n, _ = (None, None)
    if w.medium["kind"] == "random":
        from mbs_inputs import smoothed_random_medium
        n = smoothed_random_medium(w.shape, w.medium["seed"], w.medium["n_min"], w.medium["n_max"],
                                   sigma=w.ppw / 2.0, device="cuda:0")
    else:
        n = torch.from_numpy(workload_inputs(w)[0]).to(dev)
    S = source_tensor(w, "cuda:0")
    nz = torch.nonzero(S.abs() > 0)
    box = 1
    for d in range(3):
        box *= int(nz[:, d].max() - nz[:, d].min() + 1)
    torch.cuda.synchronize()
    if args.tol > 0:
        tolerance_study(args, w, n, S, mbs)
        return
    flags = mbs.MBS_TIMING | (mbs.MBS_NO_FUSION if args.no_fusion else 0)
    plan = mbs.Plan(w.shape, w.split, w.periodic, w.t, 1, w.alpha, flags=flags,
                    check_every=min(50, max(1, args.steps)), zblock=args.zblock)
    plan.set_medium(0, n, w.k_vac, w.ramp_width, w.ramp_max)
    out = torch.empty(w.shape, dtype=torch.complex64, device=dev)
    print("[bench] medium set; warmup", file=sys.stderr, flush=True)
    if args.warmup > 0:
        plan.solve(0, S, 0.0, args.warmup, out=out)
    plan.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, res = plan.solve(0, S, 0.0, args.steps, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = plan.timing()
    assert res["iterations"] == args.steps, res
    print(f"[bench] timed {args.steps} iterations in {dt:.3f} s", file=sys.stderr, flush=True)

    vox = w.voxels
    value = vox * args.steps / dt
    lossless = bool(torch.all(n.imag == 0))  # the library's own test for storing Im B only
    ab = algorithmic_bytes(w.shape, w.split, w.periodic, w.t, box, fused=not args.no_fusion,
                           b_bytes=4 if lossless else 8)
    kernels = {}
    total_bytes_iter = 0
    for k, (ms, cnt) in tim.items():
        if cnt == 0:
            continue
        # a kind may be launched in several parts per iteration (slabs of the strided passes,
        # one launch per axis of the corrections): bytes and time are taken per iteration
        per_iter_ms = ms / args.steps
        kernels[k] = {"ms_per_iteration": per_iter_ms, "avg_launch_ms": ms / cnt,
                      "launches_per_iteration": cnt / args.steps, "bytes": ab[k],
                      "gbps": ab[k] / (per_iter_ms * 1e-3) / 1e9}
        total_bytes_iter += ab[k]
    # the dominant single kernel (the slab sequence of the strided passes is many launches)
    dom = max((k for k in kernels if k != "yxy_slabs"), key=lambda k: kernels[k]["ms_per_iteration"])
    dk = kernels[dom]
    achieved = dk["gbps"]
    traffic = None
    digest = kernel_code_digest()
    if (w.name == PMC_TRAFFIC["workload"] and digest == PMC_TRAFFIC["kernel_code_sha256"]
            and PMC_TRAFFIC["fused"] == (not args.no_fusion)):
        traffic = PMC_TRAFFIC["bytes"].get(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "avg_launch_ms": round(dk["avg_launch_ms"], 4),
                "bytes_per_launch": int(round(dk["bytes"] / dk["launches_per_iteration"]))}
    hbm_gbps = total_bytes_iter * args.steps / dt / 1e9

    copy = None
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.complex64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        copy = {"bytes_read": src.numel() * 8, "bytes_written": src.numel() * 8, "avg_ms": round(ms, 4),
                "gbps": round(2 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1)}
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(n, S, w)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: {w.shape[0]}x{w.shape[1]}x{w.shape[2]} complex64 as "
                         f"{w.split[0]}x{w.split[1]}x{w.split[2]} subdomains, t={w.t}, {w.ppw:g} ppw, "
                         f"seeded smoothed random medium n in [{w.medium.get('n_min', 1)},"
                         f"{w.medium.get('n_max', 1)}], {w.source['kind']} source, "
                         f"{w.ramp_width[0]}-voxel absorbing ramps, fixed {args.steps} iterations"),
            "voxels": vox,
            "residual_reductions": "f64",
        },
        "hbm_gbps": round(hbm_gbps, 1),
        "bytes_per_voxel_update": round(total_bytes_iter / vox, 2),
        "rel_residual_after": res["rel_residual"],
        "kernels": {k: {"ms_per_iteration": round(v["ms_per_iteration"], 4), "gbps": round(v["gbps"], 1),
                        "launches_per_iteration": v["launches_per_iteration"]} for k, v in kernels.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "copy_reference": copy,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
