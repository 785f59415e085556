"""Seeded generators for media, sources and request streams.

Conventions (shared by every consumer):
  * arrays are C-order ``[x][y][z]`` (z contiguous), complex64;
  * a voxel has unit size, so a wavenumber is in radians per voxel;
  * the vacuum wavenumber of a workload is ``k_vac = 2*pi/ppw`` (ppw = points
    per wavelength); the method turns it into ``k^2`` itself.

Random media follow one recipe: white N(0,1) noise from a seeded
``torch.Generator`` on the device that will hold the medium (the CPU stream
and the GPU stream of one seed differ; every comparison hands the same
returned array to both sides), a periodic separable Gaussian filter of
standard deviation ``sigma = ppw/2`` voxels (so the autocorrelation of the
smoothed field is ``exp(-r^2/lambda^2)``, a one-wavelength correlation), then a
min-max rescale to [0, 1] and ``n = n_min + (n_max - n_min) * u``.  The
filtering may run on a GPU for large grids; the returned array is what both
sides of any comparison consume.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

Shape = Tuple[int, int, int]


# --------------------------------------------------------------------------
# media
# --------------------------------------------------------------------------
def sphere_medium(shape: Shape, radius: float, n_sphere: complex,
                  n_background: complex = 1.0,
                  center: Optional[Sequence[float]] = None) -> np.ndarray:
    """Homogeneous background with one sphere; voxel centres with
    ``|r - center| <= radius`` belong to the sphere.  ``center`` defaults to
    ``(N0/2, N1/2, N2/2)`` in voxel-index coordinates."""
    if center is None:
        center = [s / 2 for s in shape]
    i0, i1, i2 = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape],
                             indexing="ij", sparse=True)
    r2 = (i0 - center[0]) ** 2 + (i1 - center[1]) ** 2 + (i2 - center[2]) ** 2
    n = np.full(shape, n_background, dtype=np.complex64)
    n[r2 <= radius * radius] = n_sphere
    return n


def _gauss_taps(sigma: float) -> np.ndarray:
    half = max(1, int(math.ceil(4.0 * sigma)))
    x = np.arange(-half, half + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


def smoothed_random_medium(shape: Shape, seed: int, n_min: float, n_max: float,
                           sigma: float, device: str = "cpu") -> np.ndarray | torch.Tensor:
    """Seeded smoothed-noise medium rescaled to ``[n_min, n_max]`` (real index).

    Returns a numpy complex64 array when ``device == "cpu"``, else a complex64
    torch tensor on ``device`` (large grids are generated where they are used).
    """
    gen = torch.Generator(device=device).manual_seed(int(seed))
    u = torch.randn(shape, generator=gen, dtype=torch.float32, device=device)
    taps = _gauss_taps(sigma)
    half = (len(taps) - 1) // 2
    for axis in range(3):
        if shape[axis] == 1:
            continue
        acc = torch.zeros_like(u)
        for j, w in enumerate(taps):
            acc.add_(torch.roll(u, shifts=j - half, dims=axis), alpha=float(w))
        u = acc
        del acc
    lo = u.min()
    hi = u.max()
    u = (u - lo) / (hi - lo)
    n = (n_min + (n_max - n_min) * u).to(torch.complex64)
    del u
    if device == "cpu":
        return n.numpy()
    return n


# --------------------------------------------------------------------------
# sources
# --------------------------------------------------------------------------
def point_source(shape: Shape, pos: Sequence[int], amplitude: complex = 1.0) -> np.ndarray:
    s = np.zeros(shape, dtype=np.complex64)
    s[tuple(int(p) for p in pos)] = amplitude
    return s


def plane_source(shape: Shape, z: int, amplitude: complex = 1.0) -> np.ndarray:
    """Uniform source on the plane ``[:, :, z]`` (radiates towards +z and -z)."""
    s = np.zeros(shape, dtype=np.complex64)
    s[:, :, int(z)] = amplitude
    return s


def gaussian_beam_source(shape: Shape, z: int, waist: float,
                         center: Optional[Sequence[float]] = None) -> np.ndarray:
    """Flat-phase Gaussian amplitude ``exp(-rho^2/waist^2)`` on the plane z."""
    if center is None:
        center = (shape[0] / 2, shape[1] / 2)
    x = np.arange(shape[0], dtype=np.float64)[:, None] - center[0]
    y = np.arange(shape[1], dtype=np.float64)[None, :] - center[1]
    s = np.zeros(shape, dtype=np.complex64)
    s[:, :, int(z)] = np.exp(-(x * x + y * y) / (waist * waist)).astype(np.complex64)
    return s


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    """A solve: grid, decomposition, medium/source recipe and stop rule."""
    name: str
    shape: Shape
    split: Shape
    periodic: Shape
    t: int
    ppw: float
    ramp_width: Shape
    ramp_max: float
    alpha: float
    tol: float
    max_iter: int
    medium: Dict
    source: Dict

    @property
    def k_vac(self) -> float:
        return 2.0 * math.pi / self.ppw

    @property
    def voxels(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]


WORKLOADS: Dict[str, Workload] = {
    # 64^3 single domain, periodic axes with absorbing ramps; sphere R=10, n=1.5
    "plain64": Workload(
        "plain64", (64, 64, 64), (1, 1, 1), (1, 1, 1), 8, 4.0, (8, 8, 8), 0.2,
        0.75, 1e-6, 2000,
        medium=dict(kind="sphere", radius=10.0, n_sphere=1.5),
        source=dict(kind="point", pos=(16, 32, 32))),
    # 256^3 single domain, smoothed random medium n in [1, 1.5], beam at z=20
    "plain256": Workload(
        "plain256", (256, 256, 256), (1, 1, 1), (1, 1, 1), 8, 4.0, (16, 16, 16), 0.2,
        0.75, 1e-4, 5000,
        medium=dict(kind="random", seed=2, n_min=1.0, n_max=1.5),
        source=dict(kind="beam", z=20, waist_wavelengths=8.0)),
    # 512^3 as 2x2x2 subdomains of 256^3, non-periodic (wrap removal everywhere)
    "dd512": Workload(
        "dd512", (512, 512, 512), (2, 2, 2), (0, 0, 0), 8, 4.0, (16, 16, 16), 0.2,
        0.75, 1e-4, 20000,
        medium=dict(kind="random", seed=3, n_min=1.0, n_max=1.5),
        source=dict(kind="beam", z=20, waist_wavelengths=8.0)),
    # 1024^3 as one domain (periodic axes with 32-voxel ramps), the same medium recipe and
    # source as dd1024: the undecomposed case for context
    "plain1024": Workload(
        "plain1024", (1024, 1024, 1024), (1, 1, 1), (1, 1, 1), 8, 4.0, (32, 32, 32), 0.2,
        0.75, 1e-4, 200,
        medium=dict(kind="random", seed=4, n_min=1.0, n_max=1.5),
        source=dict(kind="plane", z=40)),
    # 1024^3 as 2x2x2 subdomains of 512^3; planar source; 32-voxel ramps
    "dd1024": Workload(
        "dd1024", (1024, 1024, 1024), (2, 2, 2), (0, 0, 0), 8, 4.0, (32, 32, 32), 0.2,
        0.75, 1e-4, 200,
        medium=dict(kind="random", seed=4, n_min=1.0, n_max=1.5),
        source=dict(kind="plane", z=40)),
}


def workload(name: str, **overrides) -> Workload:
    """Look up a named workload, optionally replacing fields (e.g. a smaller
    ``shape`` with the same recipe for a test)."""
    w = WORKLOADS[name]
    return dataclasses.replace(w, **overrides) if overrides else w


def workload_inputs(w: Workload, device: str = "cpu"):
    """Return ``(n, S)``: the medium and the source of a workload (complex64).

    ``n`` is a numpy array on the CPU or a torch tensor on ``device``; ``S`` is
    always a numpy array (sources are sparse and cheap)."""
    m = w.medium
    if m["kind"] == "sphere":
        n = sphere_medium(w.shape, m["radius"], m["n_sphere"])
        if device != "cpu":
            n = torch.from_numpy(n).to(device)
    elif m["kind"] == "random":
        n = smoothed_random_medium(w.shape, m["seed"], m["n_min"], m["n_max"],
                                   sigma=w.ppw / 2.0, device=device)
    elif m["kind"] == "uniform":
        n = np.full(w.shape, m["n"], dtype=np.complex64)
        if device != "cpu":
            n = torch.from_numpy(n).to(device)
    else:
        raise ValueError(m["kind"])
    s = w.source
    if s["kind"] == "point":
        S = point_source(w.shape, s["pos"])
    elif s["kind"] == "plane":
        S = plane_source(w.shape, s["z"])
    elif s["kind"] == "beam":
        S = gaussian_beam_source(w.shape, s["z"], s["waist_wavelengths"] * w.ppw)
    else:
        raise ValueError(s["kind"])
    return n, S


def source_tensor(w: "Workload", device: str) -> torch.Tensor:
    """The workload's source built directly as a complex64 tensor on ``device``
    (same values as ``workload_inputs``; avoids a host copy of large grids)."""
    s = w.source
    S = torch.zeros(w.shape, dtype=torch.complex64, device=device)
    if s["kind"] == "point":
        S[tuple(int(p) for p in s["pos"])] = 1.0
    elif s["kind"] == "plane":
        S[:, :, int(s["z"])] = 1.0
    elif s["kind"] == "beam":
        S[:, :, int(s["z"])] = torch.from_numpy(
            gaussian_beam_source((w.shape[0], w.shape[1], 1), 0, s["waist_wavelengths"] * w.ppw)[:, :, 0]
        ).to(device)
    else:
        raise ValueError(s["kind"])
    return S


# --------------------------------------------------------------------------
# serving request stream
# --------------------------------------------------------------------------
SERVING_EDGES = (64, 96, 128, 192, 256)


def poisson_requests(count: int = 200, rate_hz: float = 20.0, seed: int = 5,
                     edges: Sequence[int] = SERVING_EDGES) -> List[dict]:
    """Seeded Poisson stream of mixed-size solve requests.

    Each request: arrival time (s), cubic edge drawn uniformly from ``edges``,
    ppw ~ U[3, 6], medium seed ``1000 + i`` (n in [1.0, 1.4], one-wavelength
    correlation), point or Gaussian-beam source with probability 1/2, ramp
    width ``max(8, round(2*ppw))`` voxels per side, tolerance 1e-4.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        edge = int(rng.choice(np.asarray(edges)))
        ppw = float(rng.uniform(3.0, 6.0))
        beam = bool(rng.random() < 0.5)
        ramp = max(8, int(round(2 * ppw)))
        if beam:
            src = dict(kind="beam", z=ramp + 4, waist_wavelengths=min(8.0, edge / (4 * ppw)))
        else:
            src = dict(kind="point", pos=(edge // 4, edge // 2, edge // 2))
        wl = Workload(
            f"req{i}", (edge, edge, edge), (1, 1, 1), (1, 1, 1), 8, ppw, (ramp, ramp, ramp), 0.2,
            0.75, 1e-4, 20000,
            medium=dict(kind="random", seed=1000 + i, n_min=1.0, n_max=1.4),
            source=src)
        out.append(dict(id=i, arrival=t, workload=wl))
    return out
