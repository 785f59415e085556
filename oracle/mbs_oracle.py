"""FP64 reference implementation of the modified Born series (MBS) with the
paper's domain decomposition -- TEST INFRASTRUCTURE ONLY.

Mache & Vellekoop, "Domain decomposition of the modified Born series approach
for large-scale wave propagation simulations" (arXiv 2410.02395).

This module is the oracle that the HIP path is compared against.  It is plain,
slow and written to be checked against the paper by eye: numpy arithmetic in
complex128 / float64, the library FFT of ``scipy.fft`` as the only primitive,
and the steps of the method in the paper's order and notation.  It shares no
code, table or constant with the GPU library.  Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import it.

Notation (paper, Sec. 2):
  Helmholtz equation (Eq. 1)      (nabla^2 + k^2) psi = -S
  operator form (Eq. 2)           A x = y,  A = c (nabla^2 + k^2),  y = -c S
  splitting                        A = L + V,  L = c (nabla^2 + k_b^2),
                                   V = c (k^2 - k_b^2)   (+ decomposition terms, Sec. 3)
  iteration (Eq. 6)               x <- x - alpha (I-V) (x - (L+I)^-1 [y + (I-V) x])
  scaling (Eq. 4 / Eq. 9)         c = -0.95 i / (||k^2 - k_b^2||_inf + sum_d a_d ||A12||)
The paper writes the background wavenumber as k_0; here it is ``kb2`` = k_b^2,
while ``k_vac`` is the vacuum wavenumber (radians per voxel) of the medium.

Readings of points the paper leaves open (each also listed in the design notes):
  * k_b^2 is the midpoint of the range of Re k^2 (the paper only calls k_0 the
    background wavenumber); ``kb_rule="vacuum"`` selects k_b^2 = k_vac^2.
  * ||A12|| in Eq. 9 is the largest singular value of the unscaled t x t
    correction block C (Sec. 3 defines the operator norm that way).
  * the "infinite domain" kernel of Fig. 4 is the band-limited (sinc)
    second-derivative kernel l(m), and only the nearest periodic images are
    corrected (Sec. 3: one t x t block per edge).
  * the global residual is ||d||_2 over all subdomains divided by one global
    reference norm ||Gamma^-1 y|| (Sec. 3.1 squares and sums per-subdomain
    terms; normalising each subdomain separately is undefined where a
    subdomain holds no source).
  * the absorbing layer is a linear ramp of Im(n^2) inside the grid, 0 at
    the inner edge to ``ramp_max`` at the outermost voxel, maximum over axes.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft

__all__ = [
    "WORKERS", "laplacian_kernel_infinite", "laplacian_kernel_periodic_closed_form",
    "correction_block", "spectral_norm", "axis_flags", "absorbing_ramp",
    "wavenumber_squared", "MBSProblem", "SolveResult", "dense_axis_laplacian",
    "dense_laplacian", "dense_solve", "spectral_solve_homogeneous",
]

WORKERS = int(os.environ.get("MBS_ORACLE_THREADS",
                             os.environ.get("OMP_NUM_THREADS", min(16, os.cpu_count() or 1))))


# --------------------------------------------------------------------------
# kernels of the Laplacian (Sec. 2 Eq. 5 and Sec. 3 Fig. 4)
# --------------------------------------------------------------------------
def laplacian_kernel_infinite(m) -> np.ndarray:
    """l(m): 1D kernel of the Fourier Laplacian on the infinite unit grid.

    Eq. 5 applies the Laplacian as the symbol -p^2 (angular-spectrum kernel).
    On an unbounded grid with unit spacing its kernel is the inverse
    discrete-time Fourier transform of -p^2 over [-pi, pi]:
        l(0) = -pi^2/3,   l(m) = 2 (-1)^(m+1) / m^2   (m != 0).
    """
    m = np.asarray(m, dtype=np.float64)
    out = np.empty_like(m)
    zero = m == 0
    out[zero] = -math.pi ** 2 / 3.0
    mm = m[~zero]
    sign = np.where(np.mod(np.abs(mm), 2) == 1, 1.0, -1.0)  # (-1)^(m+1)
    out[~zero] = 2.0 * sign / (mm * mm)
    return out


def laplacian_kernel_periodic_closed_form(n: int) -> np.ndarray:
    """l_n(m), m = 0..n-1: kernel of the Laplacian that an n-point FFT
    convolution applies (the periodic images of l, Fig. 2d).

    Closed form of the spectral second-derivative matrix on a periodic grid
    (band-limited trigonometric interpolant; for even n the Nyquist mode
    p = -pi contributes -pi^2):
      even n: l_n(0) = -(pi^2/3)(1 + 2/n^2),
              l_n(m) = 2 (-1)^(m+1) (pi/n)^2 / sin^2(pi m/n)
      odd n:  l_n(0) = -(pi^2/3)(1 - 1/n^2),
              l_n(m) = 2 (-1)^(m+1) (pi/n)^2 cos(pi m/n) / sin^2(pi m/n)
    """
    m = np.arange(n, dtype=np.float64)
    out = np.empty(n, dtype=np.float64)
    if n % 2 == 0:
        out[0] = -(math.pi ** 2 / 3.0) * (1.0 + 2.0 / (n * n))
    else:
        out[0] = -(math.pi ** 2 / 3.0) * (1.0 - 1.0 / (n * n))
    mm = m[1:]
    sign = np.where(np.mod(mm, 2) == 1, 1.0, -1.0)
    s2 = np.sin(math.pi * mm / n) ** 2
    if n % 2 == 0:
        out[1:] = 2.0 * sign * (math.pi / n) ** 2 / s2
    else:
        out[1:] = 2.0 * sign * (math.pi / n) ** 2 * np.cos(math.pi * mm / n) / s2
    return out


def correction_block(t: int) -> np.ndarray:
    """C (t x t, real): the truncated communication block A12 of Sec. 3.

    Fig. 4: a column of A12 is the infinite-domain kernel response to a point
    source minus the periodic-subdomain response.  The difference that lies
    within t voxels of the shared edge is l at the distance between a voxel
    among the first t of a subdomain (index a) and a voxel among the last t
    of the previous one (index n-t+b): distance a + t - b.
        C[a, b] = l(a + t - b),   a, b in [0, t).
    The same block (transposed for the other edge, negated) removes the
    subdomain's own wrap-around (Sec. 3: off-diagonal of V_ss = -(A12 + A12^T)).
    """
    a = np.arange(t)[:, None]
    b = np.arange(t)[None, :]
    return laplacian_kernel_infinite(a + t - b)


def spectral_norm(C: np.ndarray) -> float:
    """Largest singular value (the operator norm of Sec. 3)."""
    return float(np.linalg.norm(C, 2))


def axis_flags(periodic: Sequence[int], split: Sequence[int]) -> Tuple[int, int, int]:
    """a_d of Eq. 9: 0 for a periodic axis with one subdomain (no correction),
    1 for a single subdomain with wrap-around removal only, 2 when the axis is
    split (communication plus wrap-around removal)."""
    out = []
    for p, P in zip(periodic, split):
        if P >= 2:
            out.append(2)
        elif p:
            out.append(0)
        else:
            out.append(1)
    return tuple(out)


# --------------------------------------------------------------------------
# medium (Eq. 1 wavenumber, thin absorbing layer)
# --------------------------------------------------------------------------
def absorbing_ramp(shape: Sequence[int], width: Sequence[int], ramp_max: float) -> np.ndarray:
    """Im(n^2) added by the thin absorbing layer: on each side of axis d the
    outermost ``width[d]`` voxels, at depth j = 1..W counted inwards from the
    inner edge (j = W at the outermost voxel), get ramp_max * j / W; where the
    layers of several axes overlap the maximum is taken."""
    total = np.zeros(tuple(shape), dtype=np.float64)
    for d, (N, W) in enumerate(zip(shape, width)):
        if W <= 0:
            continue
        i = np.arange(N)
        prof = np.zeros(N, dtype=np.float64)
        lo = i < W
        prof[lo] = ramp_max * (W - i[lo]) / W
        hi = i >= N - W
        prof[hi] = np.maximum(prof[hi], ramp_max * (i[hi] - (N - W) + 1) / W)
        bshape = [1, 1, 1]
        bshape[d] = N
        total = np.maximum(total, prof.reshape(bshape))
    return total


def wavenumber_squared(n: np.ndarray, k_vac: float, ramp_width: Sequence[int] = (0, 0, 0),
                       ramp_max: float = 0.0) -> np.ndarray:
    """k^2(r) = k_vac^2 (n(r)^2 + i * ramp(r))  (complex128)."""
    n = np.asarray(n).astype(np.complex128)
    n2 = n * n
    if any(w > 0 for w in ramp_width) and ramp_max != 0.0:
        n2 = n2 + 1j * absorbing_ramp(n.shape, ramp_width, ramp_max)
    return (k_vac * k_vac) * n2


# --------------------------------------------------------------------------
# the solver
# --------------------------------------------------------------------------
@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    converged: bool
    eps: List[float] = field(default_factory=list)
    rho: List[float] = field(default_factory=list)
    rho_ref: float = 0.0


class MBSProblem:
    """The decomposed MBS operators for one medium on one global grid.

    Fields are global C-order arrays (N0, N1, N2); subdomain s occupies the
    block [s_d n_d, (s_d + 1) n_d) along each axis (equal sizes, Sec. 4)."""

    def __init__(self, shape, split, periodic, t, n, k_vac, ramp_width=(0, 0, 0), ramp_max=0.0,
                 alpha=0.75, kb_rule="midrange", k2=None):
        self.shape = tuple(int(s) for s in shape)
        self.split = tuple(int(p) for p in split)
        self.periodic = tuple(int(p) for p in periodic)
        self.t = int(t)
        self.alpha = float(alpha)
        for N, P in zip(self.shape, self.split):
            if P < 1 or N % P != 0:
                raise ValueError("each axis must split into equal subdomains")
        self.sub = tuple(N // P for N, P in zip(self.shape, self.split))
        self.a = axis_flags(self.periodic, self.split)
        for d in range(3):
            if self.a[d] > 0 and not (1 <= self.t <= self.sub[d] // 2):
                raise ValueError("need 1 <= t <= n_d/2 on corrected axes")

        if k2 is None:
            k2 = wavenumber_squared(n, k_vac, ramp_width, ramp_max)
        self.k2 = np.asarray(k2, dtype=np.complex128)
        if np.any(self.k2.imag < 0):
            raise ValueError("gain medium: Im k^2 < 0")  # passive media only
        if kb_rule == "midrange":
            self.kb2 = 0.5 * (float(self.k2.real.min()) + float(self.k2.real.max()))
        elif kb_rule == "vacuum":
            self.kb2 = float(k_vac) ** 2
        else:
            raise ValueError(kb_rule)
        # Eq. 4 / Eq. 9
        self.K = float(np.max(np.abs(self.k2 - self.kb2)))
        self.C = correction_block(self.t)
        self.normC = spectral_norm(self.C)
        denom = self.K + sum(self.a) * self.normC
        if denom == 0.0:
            raise ValueError("degenerate scaling: ||k^2 - k_b^2|| + sum a_d ||A12|| = 0")
        self.c = -0.95j / denom
        # (I - V) restricted to its diagonal: 1 - c (k^2 - k_b^2)
        self.B = 1.0 - self.c * (self.k2 - self.kb2)
        # Fourier coordinates of one subdomain (Nyquist bin at p = -pi)
        p = [2.0 * math.pi * np.fft.fftfreq(nd) for nd in self.sub]
        self.p2 = (p[0][:, None, None] ** 2 + p[1][None, :, None] ** 2
                   + p[2][None, None, :] ** 2)
        # (L_ss + I)^-1 symbol: 1 / (1 + c (k_b^2 - |p|^2))     (Eq. 5, Eq. 6)
        self.G = 1.0 / (1.0 + self.c * (self.kb2 - self.p2))

    # -- helpers ----------------------------------------------------------
    def _blocks(self, z):
        P0, P1, P2 = self.split
        n0, n1, n2 = self.sub
        return z.reshape(P0, n0, P1, n1, P2, n2)

    def source_term(self, S) -> np.ndarray:
        """y = -c S (Eq. 2)."""
        return -self.c * np.asarray(S, dtype=np.complex128)

    # -- operators --------------------------------------------------------
    def corr_axis(self, z: np.ndarray, d: int) -> np.ndarray:
        """Off-diagonal Laplacian terms of the decomposed V along axis d
        (divided by c), following the five steps of Sec. 3.1:
          1. edge corrections from the first/last t voxels of each line:
             C h_s (h_s = last t values) and C^T l_s (l_s = first t values);
          2. transfer them to the neighbouring subdomain;
          4. subtract the subdomain's own corrections (wrap-around removal);
          5. add the ones arriving from the neighbours.
        Neighbours are cyclic on a periodic split axis and absent at the edge
        of a non-periodic grid.  Reads only the unmodified z."""
        P, n, t = self.split[d], self.sub[d], self.t
        zz = np.moveaxis(z, d, -1)
        lead = zz.shape[:-1]
        zz = zz.reshape(lead + (P, n))
        h = zz[..., n - t:]
        l = zz[..., :t]
        Ch = h @ self.C.T          # (C h_s)[a]  = sum_b C[a,b] h_s[b]
        CTl = l @ self.C           # (C^T l_s)[a] = sum_b C[b,a] l_s[b]
        corr = np.zeros_like(zz)
        corr[..., :t] -= Ch
        corr[..., n - t:] -= CTl
        if P >= 2:
            corr[..., 1:, :t] += Ch[..., :-1, :]           # from s-1
            corr[..., :-1, n - t:] += CTl[..., 1:, :]       # from s+1
            if self.periodic[d]:
                corr[..., 0, :t] += Ch[..., P - 1, :]
                corr[..., P - 1, n - t:] += CTl[..., 0, :]
        corr = corr.reshape(lead + (P * n,))
        return np.moveaxis(corr, -1, d)

    def apply_IV(self, z: np.ndarray) -> np.ndarray:
        """(I - V) z = B z - c * corr(z): diagonal scattering potential (step 3)
        plus the edge terms of every corrected axis."""
        out = self.B * z
        for d in range(3):
            if self.a[d] > 0:
                out -= self.c * self.corr_axis(z, d)
        return out

    def conv_L(self, w: np.ndarray) -> np.ndarray:
        """(L + I)^-1 w = F^-1 [G F w] per subdomain (Sec. 3.1)."""
        wb = self._blocks(np.asarray(w, dtype=np.complex128))
        Wf = sfft.fftn(wb, axes=(1, 3, 5), workers=WORKERS)
        Wf *= self.G[None, :, None, :, None, :]
        out = sfft.ifftn(Wf, axes=(1, 3, 5), workers=WORKERS)
        return out.reshape(self.shape)

    def apply_L(self, x: np.ndarray) -> np.ndarray:
        """L x = c F^-1 [(k_b^2 - |p|^2) F x] per subdomain (Eq. 5, Eq. 8)."""
        xb = self._blocks(np.asarray(x, dtype=np.complex128))
        Xf = sfft.fftn(xb, axes=(1, 3, 5), workers=WORKERS)
        Xf *= (self.c * (self.kb2 - self.p2))[None, :, None, :, None, :]
        return sfft.ifftn(Xf, axes=(1, 3, 5), workers=WORKERS).reshape(self.shape)

    def apply_A(self, x: np.ndarray) -> np.ndarray:
        """A x = L x + V x = L x + x - (I - V) x."""
        return self.apply_L(x) + x - self.apply_IV(x)

    # -- iteration (Eq. 6) ------------------------------------------------
    def residual_vector(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        """d = (I-V)(x - (L+I)^-1[y + (I-V)x]) = -Gamma^-1 (y - A x)."""
        v = self.conv_L(y + self.apply_IV(x))
        return self.apply_IV(x - v)

    def step(self, x: np.ndarray, y: np.ndarray) -> Tuple[np.ndarray, float]:
        """One iteration of Eq. 6; returns x_{n+1} and rho_n = ||d_n||_2."""
        v = self.conv_L(y + self.apply_IV(x))
        u = x - v
        d = self.apply_IV(u)
        return x - self.alpha * d, float(np.linalg.norm(d))

    def reference_norm(self, y: np.ndarray) -> float:
        """||Gamma^-1 y|| = ||(I-V)(L+I)^-1 y||."""
        return float(np.linalg.norm(self.apply_IV(self.conv_L(y))))

    def relative_residual(self, x: np.ndarray, S: np.ndarray) -> float:
        y = self.source_term(S)
        return float(np.linalg.norm(self.residual_vector(x, y))) / self.reference_norm(y)

    def solve(self, S: np.ndarray, tol: float = 1e-6, max_iter: int = 1000,
              x0: Optional[np.ndarray] = None, rho_ref: Optional[float] = None) -> SolveResult:
        """Iterate Eq. 6 from x0 (default 0).  The residual of x_n is computed
        in iteration n; when eps_n = rho_n / rho_ref < tol the iterate x_{n+1}
        is returned with iterations = n + 1.  ``tol = 0`` runs exactly
        ``max_iter`` iterations."""
        y = self.source_term(S)
        x = np.zeros(self.shape, np.complex128) if x0 is None else np.asarray(x0, np.complex128).copy()
        res = SolveResult(x=x, iterations=0, converged=False)
        if rho_ref is None and x0 is not None:
            rho_ref = self.reference_norm(y)
        for it in range(max_iter):
            x, rho = self.step(x, y)
            if rho_ref is None:
                rho_ref = rho
            eps = rho / rho_ref if rho_ref > 0 else 0.0
            res.rho.append(rho)
            res.eps.append(eps)
            res.iterations = it + 1
            if eps < tol:
                res.converged = True
                break
        res.x = x
        res.rho_ref = float(rho_ref if rho_ref is not None else 0.0)
        return res


# --------------------------------------------------------------------------
# dense mode: the decomposed operator written out entry by entry (tiny grids)
# --------------------------------------------------------------------------
def dense_axis_laplacian(N: int, P: int, periodic: int, t: int) -> np.ndarray:
    """Global 1D matrix of the decomposed Laplacian along one axis (Eq. 7-8,
    Fig. 5): a periodic circulant l_n per subdomain (the FFT convolution),
    minus the own wrap-around corner blocks (C at rows [0,t) x columns
    [n-t,n), C^T at rows [n-t,n) x columns [0,t)), plus the truncated
    communication blocks to the neighbouring subdomains."""
    n = N // P
    a = axis_flags([periodic], [P])[0]
    ln = laplacian_kernel_periodic_closed_form(n)
    D = np.zeros((N, N), dtype=np.float64)
    i = np.arange(n)
    circ = ln[(i[:, None] - i[None, :]) % n]
    for s in range(P):
        D[s * n:(s + 1) * n, s * n:(s + 1) * n] = circ
    if a == 0:
        return D
    C = correction_block(t)
    for s in range(P):
        o = s * n
        D[o:o + t, o + n - t:o + n] -= C
        D[o + n - t:o + n, o:o + t] -= C.T
        if P >= 2:
            sp = s - 1
            if sp >= 0 or periodic:
                sp %= P
                D[o:o + t, sp * n + n - t:sp * n + n] += C
            sn = s + 1
            if sn < P or periodic:
                sn %= P
                D[o + n - t:o + n, sn * n:sn * n + t] += C.T
    return D


def dense_laplacian(shape, split, periodic, t) -> np.ndarray:
    """Sum over axes of the 1D matrices (the Fourier Laplacian is a sum of
    one-dimensional operators), C-order flattening."""
    mats = [dense_axis_laplacian(shape[d], split[d], periodic[d], t) for d in range(3)]
    I = [np.eye(s) for s in shape]
    return (np.kron(np.kron(mats[0], I[1]), I[2])
            + np.kron(np.kron(I[0], mats[1]), I[2])
            + np.kron(np.kron(I[0], I[1]), mats[2]))


def dense_solve(shape, split, periodic, t, k2: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Direct LU solve of (Lap + diag k^2) psi = -S (Eq. 1 with the
    decomposed, truncated Laplacian)."""
    Lap = dense_laplacian(shape, split, periodic, t).astype(np.complex128)
    M = Lap + np.diag(np.asarray(k2, np.complex128).ravel())
    psi = np.linalg.solve(M, -np.asarray(S, np.complex128).ravel())
    return psi.reshape(shape)


def spectral_solve_homogeneous(S: np.ndarray, k2: complex) -> np.ndarray:
    """Periodic homogeneous medium: (nabla^2 + k^2) psi = -S has the one-shot
    spectral solution psi = F^-1 [ F S / (|p|^2 - k^2) ]."""
    shape = S.shape
    p = [2.0 * math.pi * np.fft.fftfreq(nd) for nd in shape]
    p2 = p[0][:, None, None] ** 2 + p[1][None, :, None] ** 2 + p[2][None, None, :] ** 2
    return np.fft.ifftn(np.fft.fftn(np.asarray(S, np.complex128)) / (p2 - k2))
