"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test compares the oracle with something other than itself: closed forms,
brute-force sums, a dense direct solve built entry by entry, a textbook
spectral solution, analytic physics (Green's function, Fabry-Perot slab) and
the convergence guarantees of the method.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import mbs_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
RNG = np.random.default_rng(12345)


def _cplx(shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _medium(shape, rng=RNG):
    return (1.0 + 0.4 * rng.random(shape)).astype(np.complex128)


# ---------------------------------------------------------------------------
# Laplacian kernels (Eq. 5, Fig. 2d, Fig. 4)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m", [0, 1, 2, 3, 7, 16])
def test_infinite_kernel_matches_quadrature(m):
    """l(m) = (1/2pi) int_{-pi}^{pi} -p^2 cos(p m) dp, by numerical quadrature."""
    val, _ = integrate.quad(lambda p: -p * p * math.cos(p * m), -math.pi, math.pi, limit=400)
    assert abs(O.laplacian_kernel_infinite([m])[0] - val / (2 * math.pi)) < 1e-10


@pytest.mark.parametrize("n", [1, 2, 8, 9, 15, 16, 64, 96, 256])
def test_periodic_kernel_is_what_the_fft_applies(n):
    """ifft(-p^2) over the n-point frequency grid (Nyquist bin at -pi) equals
    the closed-form spectral second-derivative kernel."""
    p = 2 * math.pi * np.fft.fftfreq(n)
    ln = np.fft.ifft(-p * p)
    assert np.abs(ln.imag).max() < 1e-12
    assert np.abs(ln.real - O.laplacian_kernel_periodic_closed_form(n)).max() < 1e-12 * max(1, n)


@pytest.mark.parametrize("n", [8, 9, 32])
def test_periodic_kernel_is_sum_of_images(n):
    """Poisson summation: l_n(m) = sum_j l(m + j n) (tail beyond |j| > J bounded by 4/(J n^2))."""
    J = 20000
    j = np.arange(-J, J + 1)
    for m in range(n):
        s = O.laplacian_kernel_infinite(m + j * n).sum()
        assert abs(s - O.laplacian_kernel_periodic_closed_form(n)[m]) < 4.0 / (J * n * n) + 1e-12


@pytest.mark.parametrize("t", [2, 4, 8])
def test_correction_block_is_infinite_minus_periodic_response(t):
    """Fig. 4 construction: apply the Laplacian to a point source once on a
    very large grid (standing in for the infinite domain) and once as a
    periodic convolution over one subdomain; the response in the first t
    voxels of the next subdomain is column b of A12 (= C[:, b]), and inside
    the subdomain the difference at its first t voxels is -C[:, b] (up to the
    farther images, bounded by 2 sum_j 2/(j n - 2t)^2)."""
    n = 32
    M = 1 << 15
    pM = 2 * math.pi * np.fft.fftfreq(M)
    pn = 2 * math.pi * np.fft.fftfreq(n)
    C = O.correction_block(t)
    for b in range(t):
        src = n - t + b                       # among the last t voxels of subdomain 1
        big = np.zeros(M)
        big[src] = 1.0
        r_inf = np.fft.ifft(-pM * pM * np.fft.fft(big)).real
        sub = np.zeros(n)
        sub[src] = 1.0
        r_per = np.fft.ifft(-pn * pn * np.fft.fft(sub)).real
        # next subdomain: voxels n .. n+t-1; the periodic convolution puts nothing there
        assert np.abs(r_inf[n:n + t] - C[:, b]).max() < 1e-7
        # own wrap-around at the first t voxels of the subdomain
        diff = r_inf[:t] - r_per[:t]
        far = 2 * sum(2.0 / (j * n - 2 * t) ** 2 for j in range(1, 10000))
        assert np.abs(diff + C[:, b]).max() < far


def test_spectral_norm_invariants():
    C = O.correction_block(8)
    s = O.spectral_norm(C)
    u, sv, vt = np.linalg.svd(C)
    assert abs(np.linalg.norm(C @ vt[0]) - s) < 1e-12
    for _ in range(50):
        x = RNG.standard_normal(8)
        assert np.linalg.norm(C @ x) <= s * np.linalg.norm(x) * (1 + 1e-12)
    # grows with t towards a limit; bounded by the l1 row-sum bound
    vals = [O.spectral_norm(O.correction_block(t)) for t in (2, 4, 8, 16, 40)]
    assert all(b >= a for a, b in zip(vals, vals[1:]))
    assert vals[-1] < np.abs(O.laplacian_kernel_infinite(np.arange(1, 200))).sum()


# ---------------------------------------------------------------------------
# scalars (Eq. 4, Eq. 9)
# ---------------------------------------------------------------------------
def test_axis_flags_table():
    g = json.load(open(GOLDEN))["a_d_values"]
    assert O.axis_flags([1, 1, 1], [1, 1, 1]) == (g["periodic_single"],) * 3
    assert O.axis_flags([0, 0, 0], [1, 1, 1]) == (g["wrap_removal_only"],) * 3
    assert O.axis_flags([0, 1, 0], [2, 3, 1]) == (g["split_axis"], g["split_axis"], g["wrap_removal_only"])


def test_scaling_reduces_to_eq4_and_hand_values():
    """Sphere workload (64^3, n in {1, 1.5}, 4 ppw, 8-voxel ramp to 0.2):
    Re k^2 spans [k_vac^2, 2.25 k_vac^2] so k_b^2 = 1.625 k_vac^2, and the
    largest |k^2 - k_b^2| is in the vacuum ramp corner:
    |-0.625 k_vac^2 + 0.2 i k_vac^2|.  Periodic axes: Eq. 9 is Eq. 4."""
    g = json.load(open(GOLDEN))
    from mbs_inputs import workload, workload_inputs
    w = workload("plain64")
    n, S = workload_inputs(w)
    pr = O.MBSProblem(w.shape, w.split, w.periodic, w.t, n, w.k_vac, w.ramp_width, w.ramp_max)
    kv2 = w.k_vac ** 2
    assert abs(pr.kb2 - 1.625 * kv2) < 1e-12
    K = kv2 * math.hypot(0.625, 0.2)
    assert abs(pr.K - K) < 1e-12
    assert abs(pr.c - (-1j * g["c_numerator"]["value"] / K)) < 1e-14
    assert pr.alpha == g["alpha"]["value"]
    # Eq. 9 with wrap removal on all axes
    pr2 = O.MBSProblem(w.shape, (2, 1, 1), (0, 0, 0), 8, n, w.k_vac, w.ramp_width, w.ramp_max)
    assert pr2.a == (2, 1, 1)
    assert abs(pr2.c - (-0.95j / (K + 4 * O.spectral_norm(O.correction_block(8))))) < 1e-14


def test_gain_medium_rejected():
    n = np.ones((8, 8, 8), np.complex128)
    n[2, 2, 2] = 1.0 - 0.1j  # n^2 has negative imaginary part
    with pytest.raises(ValueError):
        O.MBSProblem((8, 8, 8), (1, 1, 1), (1, 1, 1), 4, n, 1.0)


def test_degenerate_lossless_homogeneous_periodic_rejected():
    n = np.ones((8, 8, 8), np.complex128)
    with pytest.raises(ValueError):
        O.MBSProblem((8, 8, 8), (1, 1, 1), (1, 1, 1), 4, n, 1.0)


# ---------------------------------------------------------------------------
# operators (Eq. 5, Eq. 8, Sec. 3.1)
# ---------------------------------------------------------------------------
CASES = [
    ((8, 8, 8), (1, 1, 1), (1, 1, 1)),
    ((8, 8, 8), (1, 1, 1), (0, 0, 0)),
    ((16, 8, 8), (2, 1, 1), (0, 1, 1)),
    ((16, 8, 8), (2, 1, 1), (1, 1, 1)),
    ((16, 16, 8), (2, 2, 1), (1, 0, 0)),
    ((24, 8, 8), (3, 1, 1), (0, 0, 1)),
]


@pytest.mark.parametrize("shape,split,periodic", CASES)
def test_matrix_free_operator_equals_dense(shape, split, periodic):
    """A x from the FFT convolution plus edge corrections equals the dense
    decomposed operator c (Lap + diag k^2) built entry by entry with the
    closed-form periodic kernel (L + V = A, Sec. 3)."""
    pr = O.MBSProblem(shape, split, periodic, 4, _medium(shape), 2 * math.pi / 4, (2, 2, 2), 0.2)
    x = _cplx(shape)
    Lap = O.dense_laplacian(shape, split, periodic, 4)
    dense = pr.c * (Lap @ x.ravel() + pr.k2.ravel() * x.ravel())
    got = pr.apply_A(x).ravel()
    assert np.abs(dense - got).max() <= 1e-12 * np.abs(dense).max()
    # (L + I)^-1 inverts L + I
    w = _cplx(shape)
    back = pr.conv_L(w)
    assert np.abs(pr.apply_L(back) + back - w).max() < 1e-12 * np.abs(w).max()


def test_conv_L_on_a_plane_wave_of_each_subdomain():
    """A Fourier mode of the subdomain grid is an eigenfunction of the
    per-subdomain convolution with eigenvalue G(p) = 1/(1 + c(k_b^2 - |p|^2))."""
    shape, split = (16, 24, 8), (2, 3, 1)
    pr = O.MBSProblem(shape, split, (1, 1, 1), 2, _medium(shape), 1.1, (0, 0, 0), 0.0, kb_rule="vacuum")
    n = pr.sub
    for q in [(0, 0, 0), (1, 2, 3), (4, 4, 4), (7, 0, 5), (3, 7, 1)]:
        p = [2 * math.pi * q[d] / n[d] for d in range(3)]
        i0, i1, i2 = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
        mode = np.exp(1j * (p[0] * i0 + p[1] * i1 + p[2] * i2))   # periodic on each subdomain
        pw = [((q[d] + n[d] // 2) % n[d] - n[d] // 2) * 2 * math.pi / n[d] for d in range(3)]
        if n[0] % 2 == 0 and q[0] == n[0] // 2:
            pw[0] = -math.pi
        P2 = sum(v * v for v in pw)
        G = 1.0 / (1.0 + pr.c * (pr.kb2 - P2))
        assert np.abs(pr.conv_L(mode) - G * mode).max() < 1e-12
        assert np.abs(pr.apply_L(mode) - pr.c * (pr.kb2 - P2) * mode).max() < 1e-12


@pytest.mark.parametrize("split,periodic", [((2, 1, 1), (0, 1, 1)), ((2, 1, 1), (1, 1, 1)),
                                            ((1, 1, 1), (0, 1, 1))])
def test_decomposed_laplacian_near_an_interface_matches_brute_force(split, periodic):
    """A narrow Gaussian packet straddling the subdomain interface (or the
    grid edge, for wrap removal): within t voxels of the edge, the decomposed
    Laplacian (FFT convolution per subdomain + edge corrections) equals the
    infinite-grid band-limited Laplacian computed as a direct sum with l(m).
    A transposed, mis-signed or mis-indexed correction block fails this by O(1)."""
    N, t = 128, 8
    shape = (N, 1, 1)
    x = np.arange(N, dtype=np.float64)
    centre = (N / 2 - 0.5) if split[0] == 2 else 3.0
    sig = 2.0
    f = np.exp(-((x - centre) ** 2) / (2 * sig * sig)) * np.exp(0.8j * (x - centre))
    pr = O.MBSProblem(shape, split, periodic, t, np.ones(shape), 1.0, (0, 0, 0), 0.0,
                      k2=np.full(shape, 1.0 + 0.1j))
    lap = (pr.apply_A(f.reshape(shape)) / pr.c - pr.k2 * f.reshape(shape)).ravel()
    # infinite grid, zero outside [0, N) (non-periodic), or N-periodic images for a periodic axis
    ref = np.zeros(N, np.complex128)
    for i in range(N):
        if periodic[0]:
            m = (i - x.astype(int)) % N
            m = np.where(m > N // 2, m - N, m)
            ref[i] = np.sum(O.laplacian_kernel_infinite(m) * f)
        else:
            ref[i] = np.sum(O.laplacian_kernel_infinite(i - x.astype(int)) * f)
    if split[0] == 2:
        win = slice(N // 2 - t, N // 2 + t)
    else:
        win = slice(0, t)
    err = np.abs(lap[win] - ref[win]).max() / np.abs(ref[win]).max()
    assert err < 5e-3, err


# ---------------------------------------------------------------------------
# fixed point and convergence (Eq. 6, Sec. 2 guarantee, Sec. 3.1 stop rule)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,split,periodic", CASES[:4])
def test_converged_iteration_equals_dense_lu(shape, split, periodic):
    k2 = O.wavenumber_squared(_medium(shape), 2 * math.pi / 4, (2, 2, 2), 0.3)
    S = np.zeros(shape, np.complex128)
    S[3, 4, 5] = 1.0
    S[6, 1, 2] = 0.5 - 0.25j
    pr = O.MBSProblem(shape, split, periodic, 4, None, None, k2=k2)
    res = pr.solve(S, tol=1e-13, max_iter=20000)
    assert res.converged
    psi = O.dense_solve(shape, split, periodic, 4, k2, S)
    assert np.linalg.norm(res.x - psi) / np.linalg.norm(psi) < 1e-10
    # monotone residual (Sec. 2; Fig. 6d) above the round-off floor
    r = res.rho
    for a, b in zip(r, r[1:]):
        if a > 1e-12 * r[0]:
            assert b <= a * (1 + 1e-12)


def test_homogeneous_absorbing_periodic_equals_spectral_solution():
    shape = (16, 12, 8)
    k2 = (2 * math.pi / 5) ** 2 * (1 + 0.05j)
    S = np.zeros(shape, np.complex128)
    S[5, 6, 3] = 1.0
    pr = O.MBSProblem(shape, (1, 1, 1), (1, 1, 1), 2, None, None, k2=np.full(shape, k2))
    res = pr.solve(S, tol=1e-13, max_iter=20000)
    ref = O.spectral_solve_homogeneous(S, k2)
    assert np.linalg.norm(res.x - ref) / np.linalg.norm(ref) < 1e-10


def test_operator_norms_dense():
    """||V|| <= 0.95 (the choice of c, Eq. 9 with the triangle inequality) and
    the iteration matrix I - alpha Gamma^-1 A is non-expansive (Sec. 2)."""
    shape, split, periodic = (16, 8, 8), (2, 1, 1), (0, 1, 0)
    pr = O.MBSProblem(shape, split, periodic, 4, _medium(shape), 2 * math.pi / 4, (2, 2, 2), 0.2)
    N = int(np.prod(shape))
    Lap = O.dense_laplacian(shape, split, periodic, 4)
    A = pr.c * (Lap + np.diag(pr.k2.ravel()))
    # L: the per-subdomain periodic convolution only (block-diagonal circulants)
    blocks = [O.dense_axis_laplacian(shape[d] // split[d], 1, 1, 4) for d in range(3)]
    for d in range(3):
        blocks[d] = np.kron(np.eye(split[d]), blocks[d])
    I3 = [np.eye(s) for s in shape]
    Lp = (np.kron(np.kron(blocks[0], I3[1]), I3[2]) + np.kron(np.kron(I3[0], blocks[1]), I3[2])
          + np.kron(np.kron(I3[0], I3[1]), blocks[2]))
    L = pr.c * (Lp + pr.kb2 * np.eye(N))
    V = A - L
    assert np.linalg.norm(V, 2) <= 0.95 + 1e-12
    I = np.eye(N)
    Ginv = (I - V) @ np.linalg.inv(L + I)
    M = I - pr.alpha * Ginv @ A
    assert np.linalg.norm(M, 2) <= 1 + 1e-12
    # the matrix-free pieces agree with the dense ones
    x = _cplx(shape)
    assert np.abs((I - V) @ x.ravel() - pr.apply_IV(x).ravel()).max() < 1e-12 * np.abs(x).max() * 10


def test_update_norm_equals_alpha_times_residual_and_resume_is_exact():
    shape = (16, 8, 8)
    pr = O.MBSProblem(shape, (2, 1, 1), (0, 1, 1), 4, _medium(shape), 2 * math.pi / 4, (2, 2, 2), 0.2)
    S = np.zeros(shape, np.complex128)
    S[4, 4, 4] = 1.0
    y = pr.source_term(S)
    x = np.zeros(shape, np.complex128)
    for _ in range(5):
        xn, rho = pr.step(x, y)
        assert abs(np.linalg.norm(xn - x) - pr.alpha * rho) < 1e-12 * rho
        x = xn
    full = pr.solve(S, tol=0.0, max_iter=40)
    half = pr.solve(S, tol=0.0, max_iter=20)
    rest = pr.solve(S, tol=0.0, max_iter=20, x0=half.x, rho_ref=half.rho_ref)
    assert np.array_equal(rest.x, full.x)
    assert np.allclose(rest.eps, full.eps[20:], rtol=0, atol=0)


def test_stop_rule_returns_next_iterate():
    shape = (8, 8, 8)
    pr = O.MBSProblem(shape, (1, 1, 1), (1, 1, 1), 4, _medium(shape), 2 * math.pi / 4, (2, 2, 2), 0.2)
    S = np.zeros(shape, np.complex128)
    S[1, 2, 3] = 1
    res = pr.solve(S, tol=1e-3, max_iter=1000)
    assert res.converged and res.eps[-1] < 1e-3 and all(e >= 1e-3 for e in res.eps[:-1])
    assert res.iterations == len(res.eps)
    # zero source: the zero field is the exact answer
    z = pr.solve(np.zeros(shape), tol=1e-6, max_iter=10)
    assert z.iterations == 1 and np.all(z.x == 0)


# ---------------------------------------------------------------------------
# physics (Sec. 4: convergence to the analytical solution in an empty medium)
# ---------------------------------------------------------------------------
def test_point_source_matches_free_space_green_function():
    """Homogeneous n = 1, 64^3, 6 ppw, absorbing ramps on all sides: the
    converged field matches exp(i k r)/(4 pi r) between 6 and 14 voxels from
    the source (band-limiting and ramp reflections leave ~1-2 %)."""
    N, ppw = 64, 6.0
    k = 2 * math.pi / ppw
    n = np.ones((N, N, N), np.complex64)
    S = np.zeros((N, N, N), np.complex64)
    S[32, 32, 32] = 1
    pr = O.MBSProblem((N,) * 3, (1, 1, 1), (1, 1, 1), 8, n, k, (12, 12, 12), 0.5)
    res = pr.solve(S, tol=1e-6, max_iter=3000)
    assert res.converged
    i = np.arange(N) - 32
    R = np.sqrt(i[:, None, None] ** 2 + i[None, :, None] ** 2 + i[None, None, :] ** 2)
    m = (R >= 6) & (R <= 14)
    g = np.exp(1j * k * R[m]) / (4 * math.pi * R[m])
    err = np.linalg.norm(res.x[m] - g) / np.linalg.norm(g)
    assert err < 3e-2, err


def _slab_reflection(ppw):
    k = 2 * math.pi / ppw
    N = int(96 * ppw)
    W = int(24 * ppw)
    zs = W + int(8 * ppw)
    z1 = zs + int(16 * ppw)
    d = int(round(2.25 * ppw))           # 2.25 wavelengths thick
    n = np.ones((1, 1, N), np.complex64)
    n[0, 0, z1:z1 + d] = 1.5
    S = np.zeros((1, 1, N), np.complex64)
    S[0, 0, zs] = 1
    out = []
    for nn in (n, np.ones_like(n)):
        pr = O.MBSProblem((1, 1, N), (1, 1, 1), (1, 1, 1), 8, nn, k, (0, 0, W), 1.0)
        out.append(pr.solve(S, tol=1e-9, max_iter=100000).x[0, 0])
    x, x0 = out
    left = slice(W + int(2 * ppw), zs - int(2 * ppw))
    right = slice(z1 + d + int(2 * ppw), N - W - int(2 * ppw))
    r = np.mean(np.abs(x[left] - x0[left]) / np.abs(x0[left]))
    tau = np.mean(np.abs(x[right]) / np.abs(x0[right]))
    n2 = 1.5
    r12 = (1 - n2) / (1 + n2)
    e = np.exp(2j * n2 * k * d)
    r_fp = abs(r12 * (1 - e) / (1 - r12 * r12 * e))
    return r, tau, r_fp


def test_dielectric_slab_matches_fabry_perot():
    """1D slab of index 1.5 (2.25 wavelengths): the reflection amplitude
    approaches the Fabry-Perot value as sampling refines, and energy is
    conserved (|r|^2 + |tau|^2 = 1 for a lossless slab)."""
    errs = []
    for ppw in (4, 8, 16):
        r, tau, r_fp = _slab_reflection(ppw)
        errs.append(abs(r - r_fp))
        assert abs(r * r + tau * tau - 1) < 2e-3
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-2


# ---------------------------------------------------------------------------
# convergence studies of Sec. 4.2 (truncation parameter, number of subdomains)
# ---------------------------------------------------------------------------
def _line_case(N=192, seed=3):
    """A 1D line (N, 1, 1) of a smoothed random medium, n in [1, 1.5] with a
    small absorption, 6 points per wavelength, point source at N/3."""
    from mbs_inputs import smoothed_random_medium
    n = smoothed_random_medium((N, 1, 1), seed, 1.0, 1.5, 3.0) + np.complex64(0.02j)
    S = np.zeros((N, 1, 1), np.complex64)
    S[N // 3, 0, 0] = 1
    return n.astype(np.complex64), S, 2 * math.pi / 6


def test_truncation_error_decays_with_t_and_iterations_do_not_depend_on_t():
    """Sec. 4.2.1 / Fig. 7: two subdomains on a cyclic axis against the single
    periodic domain they decompose.  The error is the truncation of the
    communication and wrap blocks alone; it falls with t (squared relative
    error, the paper's measure, below 1e-3 from t = 4 on) while the iteration
    count stays the same for t >= 4."""
    n, S, k = _line_case()
    N = n.shape[0]
    ref = O.MBSProblem((N, 1, 1), (1, 1, 1), (1, 1, 1), 8, n, k).solve(S, tol=1e-10, max_iter=20000)
    assert ref.converged
    errs, iters = {}, {}
    for t in (4, 8, 16, 24):
        r = O.MBSProblem((N, 1, 1), (2, 1, 1), (1, 1, 1), t, n, k).solve(S, tol=1e-10, max_iter=20000)
        assert r.converged
        errs[t] = np.linalg.norm(r.x - ref.x) / np.linalg.norm(ref.x)
        iters[t] = r.iterations
    ts = sorted(errs)
    assert all(errs[a] > errs[b] for a, b in zip(ts, ts[1:])), errs
    assert errs[4] ** 2 < 1e-3 and errs[24] < 0.1 * errs[4], errs
    assert max(iters.values()) <= 1.02 * min(iters.values()), iters


def test_iterations_do_not_depend_on_the_number_of_subdomains():
    """Sec. 4.2.2: splitting an axis into 2, 3 or 4 subdomains leaves c (Eq. 9,
    a_d = 2 in every case) and the iteration count to a fixed tolerance the same
    to within 5 %."""
    n, S, k = _line_case()
    N = n.shape[0]
    its, cs = [], []
    for P in (2, 3, 4):
        pr = O.MBSProblem((N, 1, 1), (P, 1, 1), (1, 1, 1), 8, n, k)
        r = pr.solve(S, tol=1e-6, max_iter=20000)
        assert r.converged
        its.append(r.iterations)
        cs.append(pr.c)
    assert cs[0] == cs[1] == cs[2]
    assert max(its) <= 1.05 * min(its), its
