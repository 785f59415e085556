"""GPU path vs the FP64 oracle, element by element, through the C ABI.

The bar (relative L2 <= 2e-5 at a fixed iteration count) compares complex64
FFT/pointwise arithmetic with FP64 residual reductions against an all-FP64
reference on identical inputs.
"""

import math

import numpy as np
import pytest

from _mbs_cases import gpu_solve, oracle_problem, random_case, rel_l2, workload, workload_inputs

pytestmark = pytest.mark.gpu

TOL = 2e-5


def _compare(shape, split, periodic, t, n, S, k_vac, rw, rm, iters, tol_bar=TOL, flags=0):
    x_gpu, res, hist = gpu_solve(shape, split, periodic, t, n, S, k_vac, rw, rm, 0.0, iters, flags=flags)
    pr = oracle_problem(shape, split, periodic, t, n, k_vac, rw, rm)
    ref = pr.solve(S, tol=0.0, max_iter=iters)
    print(f"shape={shape} split={split} periodic={periodic} t={t} iters={iters}", flush=True)
    assert res["iterations"] == iters
    # FP64 scalars agree with the oracle's own
    assert abs(res["kb2"] - pr.kb2) <= 1e-12 * abs(pr.kb2)
    assert abs(res["K"] - pr.K) <= 1e-12 * pr.K
    assert abs(res["c_imag"] - pr.c.imag) <= 1e-12 * abs(pr.c.imag)
    assert abs(res["normC"] - pr.normC) <= 1e-12 * pr.normC
    err = rel_l2(x_gpu, ref.x)
    print(f"  rel L2 vs oracle = {err:.3e}", flush=True)
    assert err <= tol_bar, err
    # per-iteration relative residuals agree too
    h = np.asarray(hist)
    e = np.asarray(ref.eps)
    assert np.max(np.abs(h - e) / e) < 1e-3
    return x_gpu


def test_plain_sphere_64_fixed_iterations():
    w = workload("plain64")
    n, S = workload_inputs(w)
    _compare(w.shape, w.split, w.periodic, w.t, n, S, w.k_vac, w.ramp_width, w.ramp_max, 100)


def test_plain_sphere_64_to_tolerance():
    """Run the oracle to 1e-6 and the GPU to its FP32 residual floor: the GPU
    field agrees with the converged FP64 field, and the GPU stops at 1e-5."""
    w = workload("plain64")
    n, S = workload_inputs(w)
    x_gpu, res, hist = gpu_solve(w.shape, w.split, w.periodic, w.t, n, S, w.k_vac, w.ramp_width,
                                 w.ramp_max, 1e-5, 5000)
    pr = oracle_problem(w.shape, w.split, w.periodic, w.t, n, w.k_vac, w.ramp_width, w.ramp_max)
    ref = pr.solve(S, tol=1e-6, max_iter=5000)
    err = rel_l2(x_gpu, ref.x)
    h = np.asarray(hist)
    print(f"plain64: gpu {res['iterations']} it to {res['rel_residual']:.2e}, oracle {ref.iterations} it "
          f"to 1e-6, rel L2 {err:.3e}; ||x||/rho_ref = {np.linalg.norm(x_gpu) / res['rho_ref']:.1f}; "
          f"gpu eps tail {h[-5:]}", flush=True)
    assert res["converged"] == 1 and ref.converged
    assert err <= 5e-5
    # oracle's own relative residual of the GPU field
    ro = pr.relative_residual(x_gpu.astype(np.complex128), S)
    print(f"  oracle residual of the GPU field: {ro:.3e}", flush=True)
    assert ro < 2e-5
    # the library's residual evaluation of a given field agrees with the oracle's
    import torch
    from paper_2410_02395_amd import mbs
    dev = torch.device("cuda:0")
    with mbs.Plan(w.shape, w.split, w.periodic, w.t) as plan:
        plan.set_medium(0, torch.from_numpy(n).to(dev), w.k_vac, w.ramp_width, w.ramp_max)
        _, r2 = plan.solve(0, torch.from_numpy(S).to(dev), 1e-3, 5000)
        rr_last = plan.residual(0)
        rr = plan.residual(0, torch.from_numpy(x_gpu).to(dev))
        print(f"  library residual of the GPU field {rr:.3e}, of its own 1e-3 iterate {rr_last:.3e} "
              f"(solve reported {r2['rel_residual']:.3e})", flush=True)
        assert abs(rr - ro) <= 0.2 * ro + 2e-6
        assert rr_last < 1.2e-3


@pytest.mark.parametrize("shape,split,periodic,t", [
    ((64, 64, 64), (2, 2, 2), (0, 0, 0), 8),     # 8 subdomains of 32^3, wrap removal everywhere
    ((48, 24, 96), (2, 1, 2), (1, 0, 0), 4),     # ragged tiles, cyclic split axis, radix 3
    ((32, 64, 16), (1, 2, 1), (0, 1, 1), 4),     # periodic split axis, mixed a_d
    ((24, 16, 12), (3, 2, 1), (0, 0, 0), 2),     # three subdomains along x, tiny edges
])
def test_decomposed_fixed_iterations(shape, split, periodic, t):
    n, S = random_case(shape, seed=7)
    k = 2 * math.pi / 4
    _compare(shape, split, periodic, t, n, S, k, (4, 4, 4), 0.2, 60)


@pytest.mark.parametrize("shape,split,periodic,t", [
    ((64, 64, 64), (2, 2, 2), (0, 0, 0), 8),
    ((48, 24, 96), (2, 1, 2), (1, 0, 0), 4),
])
def test_lossy_medium_fixed_iterations(shape, split, periodic, t):
    """A medium with Im n > 0 keeps the whole of B in memory; a lossless one (every other case
    here) stores Im B only and rebuilds Re B = 1 + c_im k0^2 ramp from the absorbing layers."""
    n, S = random_case(shape, seed=19)
    n = (n + 0.01j).astype(np.complex64)
    k = 2 * math.pi / 4
    _compare(shape, split, periodic, t, n, S, k, (4, 4, 4), 0.2, 60)


@pytest.mark.parametrize("shape,split,periodic,t", [
    ((64, 64, 64), (2, 2, 2), (0, 0, 0), 8),
    ((48, 24, 96), (2, 1, 2), (1, 0, 0), 4),
    ((16, 24, 144), (1, 1, 3), (1, 1, 1), 4),    # three segments on a cyclic z axis
    ((16, 16, 2048), (1, 1, 2), (0, 0, 0), 8),   # two 1024-point segments per workgroup
])
def test_separate_and_fused_z_passes_agree(shape, split, periodic, t):
    """The two launch sequences (the inverse z pass of one iteration fused with the
    forward z pass of the next, or kept apart) both meet the bar and differ only by
    rounding order."""
    from paper_2410_02395_amd import mbs
    n, S = random_case(shape, seed=9)
    k = 2 * math.pi / 4
    fused = _compare(shape, split, periodic, t, n, S, k, (4, 4, 4), 0.2, 50)
    apart = _compare(shape, split, periodic, t, n, S, k, (4, 4, 4), 0.2, 50, flags=mbs.MBS_NO_FUSION)
    d = rel_l2(fused, apart)
    print(f"  fused vs separate: rel L2 {d:.3e}", flush=True)
    assert d <= 1e-5


@pytest.mark.parametrize("rw_z", [64, 80])
def test_z_ramp_at_and_beyond_the_butterfly_stride(rw_z):
    """Two 512-point z segments (first radix 8, so a thread's elements are 64 apart) of a
    lossless medium, whose Re B the fused z pass rebuilds from the ramp: a 64-voxel z ramp
    reaches only the first and last element of each butterfly, an 80-voxel one reaches
    further in and takes the per-element path; both against the oracle."""
    shape = (16, 16, 1024)
    n, S = random_case(shape, seed=23)
    _compare(shape, (1, 1, 2), (0, 0, 0), 8, n, S, 2 * math.pi / 4, (4, 4, rw_z), 0.2, 40)


@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 12, 24), (96, 32, 64), (12, 192, 8), (256, 8, 32), (384, 16, 32),
                                   (512, 8, 16), (768, 8, 16), (1024, 8, 16), (8, 768, 16), (8, 1024, 16),
                                   (16, 8, 768), (16, 8, 1024)])
def test_plain_sizes_and_radices(shape):
    n, S = random_case(shape, seed=3, src="plane")
    _compare(shape, (1, 1, 1), (1, 1, 1), 8, n, S, 2 * math.pi / 5, (2, 2, 2), 0.3, 40)


def test_zero_source_gives_zero_field():
    shape = (32, 32, 32)
    n, _ = random_case(shape)
    x, res, _ = gpu_solve(shape, (1, 1, 1), (1, 1, 1), 8, n, np.zeros(shape, np.complex64),
                          1.0, (4, 4, 4), 0.2, 1e-6, 100)
    assert res["iterations"] == 1 and res["converged"] == 1
    assert np.all(x == 0)


def test_resume_from_checkpoint_is_bitwise():
    """Richardson is memoryless: k iterations, then k more from x_k, equals 2k iterations."""
    from paper_2410_02395_amd import mbs
    shape, split, periodic = (32, 32, 32), (2, 1, 1), (0, 1, 1)
    n, S = random_case(shape, seed=11)
    k = 2 * math.pi / 4
    full, _, _ = gpu_solve(shape, split, periodic, 4, n, S, k, (4, 4, 4), 0.2, 0.0, 40)
    half, _, _ = gpu_solve(shape, split, periodic, 4, n, S, k, (4, 4, 4), 0.2, 0.0, 20)
    rest, res, _ = gpu_solve(shape, split, periodic, 4, n, S, k, (4, 4, 4), 0.2, 0.0, 20,
                             flags=mbs.MBS_X0_GIVEN, x0=half)
    assert np.array_equal(rest, full)


def test_async_solve_reports_progress_and_matches_the_blocking_solve():
    """mbs_solve_async + mbs_poll: while the slot runs, poll returns MBS_EBUSY with the iterations
    and residual of its last completed launch (non-decreasing iterations, at most the final count);
    the finished field is bitwise the blocking solve's."""
    import time
    import torch
    from paper_2410_02395_amd import mbs
    shape, split, periodic = (64, 64, 128), (2, 2, 2), (0, 0, 0)
    n, S = random_case(shape, seed=9)
    k = 2 * math.pi / 4
    dev = torch.device("cuda:0")
    nt = torch.from_numpy(np.ascontiguousarray(n, np.complex64)).to(dev)
    St = torch.from_numpy(np.ascontiguousarray(S, np.complex64)).to(dev)
    iters = 400
    with mbs.Plan(shape, split, periodic, 8, 1, 0.75, 0, 10) as plan:
        plan.set_medium(0, nt, k, (4, 4, 4), 0.2)
        ref, rref = plan.solve(0, St, 0.0, iters)
        ref = ref.cpu().numpy()
        out = torch.empty(shape, dtype=torch.complex64, device=dev)
        plan.solve_async(0, St, 0.0, iters, out)
        seen = []
        t0 = time.perf_counter()
        while True:
            res = plan.poll(0)
            if res is not None:
                break
            seen.append(plan.progress[0])
            assert time.perf_counter() - t0 < 60.0
            time.sleep(0.0005)
        torch.cuda.synchronize()
    its = [it for it, _ in seen]
    print(f"{len(seen)} busy polls, iterations seen {its[:3]} ... {its[-3:]}", flush=True)
    assert res["iterations"] == rref["iterations"] == iters
    assert all(a <= b for a, b in zip(its, its[1:]))
    assert all(0 <= it <= iters for it in its)
    assert all(e >= 0.0 for it, e in seen if it > 0)
    assert np.array_equal(out.cpu().numpy(), ref)


def test_slots_with_lossless_and_lossy_media_batch_bitwise():
    """Two slots of one plan iterate in the same launches, one with a lossless medium (Im B stored
    alone) and one with a lossy medium (the whole of B): each field is bitwise the field of the same
    slot solved alone."""
    import torch
    from paper_2410_02395_amd import mbs
    shape, split, periodic = (64, 32, 64), (2, 1, 2), (0, 0, 0)
    n0, S = random_case(shape, seed=31)
    n1 = (n0 + 0.02j).astype(np.complex64)
    k = 2 * math.pi / 4
    dev = torch.device("cuda:0")
    media = [torch.from_numpy(np.ascontiguousarray(m, np.complex64)).to(dev) for m in (n0, n1)]
    St = torch.from_numpy(np.ascontiguousarray(S, np.complex64)).to(dev)
    iters = 37
    alone = []
    with mbs.Plan(shape, split, periodic, 8, 2, 0.75, 0, 8) as plan:
        for slot in range(2):
            plan.set_medium(slot, media[slot], k, (4, 4, 4), 0.2)
        for slot in range(2):
            out, res = plan.solve(slot, St, 0.0, iters)
            assert res["iterations"] == iters
            alone.append(out.cpu().numpy())
        outs = [torch.empty(shape, dtype=torch.complex64, device=dev) for _ in range(2)]
        for slot in range(2):
            plan.solve_async(slot, St, 0.0, iters, outs[slot])
        done = [None, None]
        while any(d is None for d in done):
            for slot in range(2):
                if done[slot] is None:
                    done[slot] = plan.poll(slot)
        torch.cuda.synchronize()
    assert all(d["iterations"] == iters for d in done)
    assert not np.array_equal(alone[0], alone[1])
    for slot in range(2):
        assert np.array_equal(outs[slot].cpu().numpy(), alone[slot]), slot


def test_graph_and_eager_launches_agree_bitwise():
    from paper_2410_02395_amd import mbs
    shape, split, periodic = (32, 32, 32), (2, 2, 1), (0, 0, 1)
    n, S = random_case(shape, seed=5)
    k = 2 * math.pi / 4
    a, ra, _ = gpu_solve(shape, split, periodic, 4, n, S, k, (4, 4, 4), 0.2, 0.0, 37, check_every=8)
    b, rb, _ = gpu_solve(shape, split, periodic, 4, n, S, k, (4, 4, 4), 0.2, 0.0, 37,
                         flags=mbs.MBS_NO_GRAPH)
    c, rc, _ = gpu_solve(shape, split, periodic, 4, n, S, k, (4, 4, 4), 0.2, 0.0, 37,
                         flags=mbs.MBS_TIMING, check_every=5)
    assert ra["iterations"] == rb["iterations"] == rc["iterations"] == 37
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_residual_history_is_monotone():
    w = workload("plain64")
    n, S = workload_inputs(w)
    _, res, hist = gpu_solve(w.shape, w.split, w.periodic, w.t, n, S, w.k_vac, w.ramp_width,
                             w.ramp_max, 1e-5, 3000)
    h = np.asarray(hist)
    assert len(h) == res["iterations"]
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-4))


def test_error_paths():
    import torch
    from paper_2410_02395_amd import mbs
    dev = torch.device("cuda:0")
    shape = (16, 16, 16)
    ones = torch.ones(shape, dtype=torch.complex64, device=dev)
    S = torch.zeros(shape, dtype=torch.complex64, device=dev)
    S[3, 3, 3] = 1
    with pytest.raises(mbs.MBSError) as e:
        mbs.Plan((100, 16, 16))
    assert e.value.status == mbs.MBS_EUNSUPPORTED
    with pytest.raises(mbs.MBSError) as e:
        mbs.Plan(shape, (2, 1, 1), (0, 0, 0), t=5)   # t > n/2
    assert e.value.status == mbs.MBS_EINVAL
    with mbs.Plan(shape) as plan:
        with pytest.raises(mbs.MBSError) as e:
            plan.solve(0, S, 1e-6, 10)
        assert e.value.status == mbs.MBS_ESTATE
        with pytest.raises(mbs.MBSError) as e:
            plan.set_medium(0, ones, 1.0)           # lossless homogeneous periodic: K = 0
        assert e.value.status == mbs.MBS_EDEGENERATE
        gain = ones.clone()
        gain[1, 2, 3] = 1.0 - 0.2j
        with pytest.raises(mbs.MBSError) as e:
            plan.set_medium(0, gain, 1.0, (2, 2, 2), 0.1)
        assert e.value.status == mbs.MBS_EGAIN
        bad = ones.clone()
        bad[0, 0, 0] = float("nan")
        with pytest.raises(mbs.MBSError) as e:
            plan.set_medium(0, bad, 1.0, (2, 2, 2), 0.1)
        assert e.value.status == mbs.MBS_ENONFINITE
        plan.set_medium(0, ones, 1.0, (2, 2, 2), 0.1)
        badS = S.clone()
        badS[1, 1, 1] = float("inf")
        with pytest.raises(mbs.MBSError) as e:
            plan.solve(0, badS, 1e-6, 10)
        assert e.value.status == mbs.MBS_ENONFINITE
        _, r = plan.solve(0, S, 1e-12, 3)          # not converging is not an error
        assert r["iterations"] == 3 and r["converged"] == 0


def test_slab_schedule_of_the_strided_passes_is_bitwise_neutral():
    """The y, x and inverse-y passes run pass by pass over every subdomain, or subdomain by
    subdomain on z slabs (zblock): each tile computes the same values either way."""
    from paper_2410_02395_amd import mbs
    import torch
    shape, split, periodic, t = (256, 256, 128), (2, 2, 2), (0, 0, 0), 8
    n, S = random_case(shape, seed=13)
    k = 2 * math.pi / 4
    dev = torch.device("cuda:0")
    nt = torch.from_numpy(n).to(dev)
    St = torch.from_numpy(S).to(dev)
    outs = {}
    for zb in (-1, 32, 64):
        for act in (0.0, 1e-2):
            with mbs.Plan(shape, split, periodic, t, 1, 0.75, 0, 8, activation=act, zblock=zb) as plan:
                plan.set_medium(0, nt, k, (4, 4, 4), 0.2)
                out, res = plan.solve(0, St, 0.0, 24)
                outs[(zb, act)] = out.cpu().numpy()
    for act in (0.0, 1e-2):
        assert np.array_equal(outs[(-1, act)], outs[(32, act)])
        assert np.array_equal(outs[(-1, act)], outs[(64, act)])


def test_slab_schedules_chosen_automatically_are_bitwise_neutral():
    """Where the work arrays exceed the memory-side cache the plan picks the slab schedule
    itself: whole subdomains alternating over two streams when two fit in the cache
    (512x512x256 as 2x2x2: 64 MiB subdomains), or slabs of 128 z values stored slab by slab
    with the inverse y pass writing z-lines to a second array (512x512x1024 as 1x1x2: 1 GiB
    subdomains, 512^2 cross-sections).  Either way every tile computes what the whole passes
    compute."""
    from paper_2410_02395_amd import mbs
    from mbs_inputs import smoothed_random_medium
    import torch
    dev = torch.device("cuda:0")
    k = 2 * math.pi / 4
    for shape, split in (((512, 512, 256), (2, 2, 2)), ((512, 512, 1024), (1, 1, 2))):
        print(f"shape {shape} split {split}", flush=True)
        n = smoothed_random_medium(shape, 17, 1.0, 1.5, 2.0, device=dev)
        S = torch.zeros(shape, dtype=torch.complex64, device=dev)
        S[shape[0] // 3, shape[1] // 2, shape[2] // 2 + 5] = 1
        outs = {}
        for zb in (-1, 0):
            for act in (0.0, 1e-2):
                with mbs.Plan(shape, split, (0, 0, 0), 8, 1, 0.75, 0, 6, activation=act, zblock=zb) as plan:
                    plan.set_medium(0, n, k, (8, 8, 8), 0.2)
                    out, res = plan.solve(0, S, 0.0, 12)
                    torch.cuda.synchronize()
                    outs[(zb, act)] = out
        for act in (0.0, 1e-2):
            assert torch.equal(outs[(-1, act)], outs[(0, act)]), (shape, act)
        del outs, n, S
        torch.cuda.empty_cache()
