"""Seeded synthetic image pairs for PSF matching.

This module only *makes inputs*: star fields rendered with Gaussian PSFs, sky,
Gaussian noise, variance maps, bad-pixel masks and a stamp list taken from the
known source catalogue.  It holds none of the matching method's arithmetic
(no kernel basis, no convolution with the basis, no least squares), so the
FP64 oracle and the HIP path can both consume it without sharing any of the
method.

Workloads stand in for the Pan-STARRS GPC1 data the paper analyses (Sections 3
and 6), which is not available: sizes, PSF widths, source densities and mask
fractions follow the workload definitions in :data:`WORKLOADS`.

Conventions (shared with the C interface):
  * images are float32, row-major, ``img[y, x]`` with x the fast axis;
  * masks are uint8, non-zero = masked; masked pixels hold NaN in image and
    variance planes so that any leak of a masked value is visible;
  * stamp centres are int32 ``(x, y)`` pairs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

SEED_BASE = 19010999


@dataclasses.dataclass(frozen=True)
class PsfField:
    """A Gaussian PSF whose width and ellipticity may vary across the field.

    sigma(x) = sigma_lo + (sigma_hi - sigma_lo) * x / (W - 1)
    e(y)     = e_max * y / (H - 1)           (e = 1 - b/a)
    The major axis lies at angle ``theta`` (radians); the area is preserved,
    sigma_a * sigma_b = sigma**2.
    """

    sigma_lo: float
    sigma_hi: float
    e_max: float = 0.0
    theta: float = 0.0

    def params(self, x: np.ndarray, y: np.ndarray, W: int, H: int):
        fx = x / max(W - 1, 1)
        fy = y / max(H - 1, 1)
        sig = self.sigma_lo + (self.sigma_hi - self.sigma_lo) * fx
        e = self.e_max * fy
        sa = sig / np.sqrt(1.0 - e)
        sb = sig * np.sqrt(1.0 - e)
        return sa, sb


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    width: int
    height: int
    n_sources: int
    ref_psf: PsfField
    sci_psf: PsfField
    mask_frac: float
    kernel_half: int
    sigmas: Tuple[float, ...]
    degrees: Tuple[int, ...]
    spatial_order: int
    n_stamps: int
    stamp_half: int
    flux_lo: float = 1e3
    flux_hi: float = 1e5
    sky: float = 100.0
    saturation: float = 5000.0
    variable_frac: float = 0.0
    cov_half: int = 10          # half-size of the reported covariance pseudo-matrix
    patch: int = 64             # side of the constant-kernel patches

    @property
    def n_basis(self) -> int:
        return sum((d + 1) * (d + 2) // 2 for d in self.degrees)

    @property
    def n_spatial(self) -> int:
        s = self.spatial_order
        return (s + 1) * (s + 2) // 2

    @property
    def n_unknowns(self) -> int:
        return self.n_basis * self.n_spatial + 1

    @property
    def pixels(self) -> int:
        return self.width * self.height


ISIS_SIGMAS = (0.7, 1.5, 3.0)
ISIS_DEGREES = (6, 4, 2)

WORKLOADS: Dict[str, Workload] = {
    # Plain method, CPU-seconds scale.
    "cfg0": Workload("cfg0", 512, 512, 200, PsfField(1.5, 1.5), PsfField(2.2, 2.2),
                     0.0, 10, ISIS_SIGMAS, ISIS_DEGREES, 0, 50, 20),
    # Plain FP32 GPU path with a spatially varying science PSF and a 10% mask.
    "cfg1": Workload("cfg1", 2048, 2048, 2000, PsfField(1.2, 1.2), PsfField(1.4, 2.6, 0.2),
                     0.10, 10, ISIS_SIGMAS, ISIS_DEGREES, 2, 100, 20),
    # Detector-chip-sized pair (GPC1 chip), 15% mask, 25x25 kernel, order 3.
    "cfg2": Workload("cfg2", 4846, 4868, 8000, PsfField(1.2, 1.2), PsfField(1.4, 2.6, 0.2),
                     0.15, 12, ISIS_SIGMAS, ISIS_DEGREES, 3, 400, 24),
}


def workload_seed(cfg_index: int, pair: int = 0) -> int:
    return SEED_BASE + 1000 * cfg_index + pair


def _render(W: int, H: int, xs, ys, fluxes, psf: PsfField, theta: float) -> np.ndarray:
    """Sum of pixel-sampled elliptical Gaussians (float64), each rendered in a
    window of +-6 major-axis sigmas."""
    img = np.zeros((H, W), dtype=np.float64)
    sa, sb = psf.params(xs, ys, W, H)
    c, s = math.cos(theta), math.sin(theta)
    for x0, y0, f, a, b in zip(xs, ys, fluxes, sa, sb):
        rad = int(math.ceil(6.0 * a)) + 1
        xi0, xi1 = max(int(math.floor(x0)) - rad, 0), min(int(math.floor(x0)) + rad + 1, W)
        yi0, yi1 = max(int(math.floor(y0)) - rad, 0), min(int(math.floor(y0)) + rad + 1, H)
        if xi0 >= xi1 or yi0 >= yi1:
            continue
        dx = np.arange(xi0, xi1, dtype=np.float64)[None, :] - x0
        dy = np.arange(yi0, yi1, dtype=np.float64)[:, None] - y0
        # rotate into the principal frame
        pa = c * dx + s * dy
        pb = -s * dx + c * dy
        q = (pa / a) ** 2 + (pb / b) ** 2
        img[yi0:yi1, xi0:xi1] += f / (2.0 * math.pi * a * b) * np.exp(-0.5 * q)
    return img


def _make_mask(rng: np.random.Generator, model: np.ndarray, frac: float,
               saturation: float) -> np.ndarray:
    H, W = model.shape
    mask = np.zeros((H, W), dtype=np.uint8)
    if frac <= 0:
        return mask
    sat = model > saturation
    if sat.any():
        # 1-pixel dilation of the saturated cores
        d = sat.copy()
        d[1:, :] |= sat[:-1, :]
        d[:-1, :] |= sat[1:, :]
        d[:, 1:] |= sat[:, :-1]
        d[:, :-1] |= sat[:, 1:]
        mask[d] = 1
    # contiguous blocks of bad columns until the target fraction is reached
    while mask.mean() < frac:
        w = int(rng.integers(4, 65))
        x0 = int(rng.integers(0, max(W - w, 1)))
        mask[:, x0:x0 + w] = 1
    return mask


@dataclasses.dataclass
class Pair:
    workload: Workload
    I1: np.ndarray
    V1: np.ndarray
    M1: np.ndarray
    I2: np.ndarray
    V2: np.ndarray
    M2: np.ndarray
    stamps: np.ndarray          # int32 [n, 2] (x, y)
    xs: np.ndarray
    ys: np.ndarray
    fluxes: np.ndarray
    seed: int

    @property
    def width(self) -> int:
        return self.workload.width

    @property
    def height(self) -> int:
        return self.workload.height


def select_stamps(xs, ys, fluxes, M1, M2, n_stamps: int, r: int, h: int,
                  grid: Optional[int] = None) -> np.ndarray:
    """Pick stamp centres from the known catalogue: the brightest source in each
    cell of a subregion grid whose footprint lies inside the image and away
    from masked pixels; further passes take the next-brightest per cell until
    ``n_stamps`` are found (or candidates run out)."""
    H, W = M1.shape
    if grid is None:
        grid = max(1, int(math.ceil(math.sqrt(n_stamps))))
    cx = np.clip((xs * grid / W).astype(int), 0, grid - 1)
    cy = np.clip((ys * grid / H).astype(int), 0, grid - 1)
    order = np.argsort(-fluxes, kind="stable")
    cells: Dict[Tuple[int, int], List[int]] = {}
    for k in order:
        cells.setdefault((int(cx[k]), int(cy[k])), []).append(int(k))
    bad1 = M1 != 0
    bad2 = M2 != 0
    # summed-area tables make the footprint tests O(1)
    sat1 = np.pad(bad1.astype(np.int64).cumsum(0).cumsum(1), ((1, 0), (1, 0)))
    sat2 = np.pad(bad2.astype(np.int64).cumsum(0).cumsum(1), ((1, 0), (1, 0)))

    def box_any(sat, x0, y0, x1, y1):
        return (sat[y1 + 1, x1 + 1] - sat[y0, x1 + 1] - sat[y1 + 1, x0] + sat[y0, x0]) > 0

    chosen: List[Tuple[int, int]] = []
    taken = set()
    keys = sorted(cells.keys(), key=lambda t: (t[1], t[0]))
    cursor = {k: 0 for k in keys}
    while len(chosen) < n_stamps:
        progress = False
        for key in keys:
            if len(chosen) >= n_stamps:
                break
            lst = cells[key]
            while cursor[key] < len(lst):
                k = lst[cursor[key]]
                cursor[key] += 1
                x = int(round(float(xs[k])))
                y = int(round(float(ys[k])))
                R = r + h
                if x - R < 0 or y - R < 0 or x + R >= W or y + R >= H:
                    continue
                if (x, y) in taken:
                    continue
                if box_any(sat1, x - R, y - R, x + R, y + R):
                    continue
                if box_any(sat2, x - r, y - r, x + r, y + r):
                    continue
                chosen.append((x, y))
                taken.add((x, y))
                progress = True
                break
        if not progress:
            break
    return np.asarray(chosen, dtype=np.int32).reshape(-1, 2)


def make_pair(wl: Workload, seed: int, theta: Optional[float] = None,
              n_stamps: Optional[int] = None) -> Pair:
    """Render a reference (image 1, narrower PSF) / science (image 2) pair.

    Both images see the same sources (a ``variable_frac`` share have their
    science flux scaled by U[0.5, 2]), a sky of ``wl.sky`` and independent
    Gaussian noise with variance sky + signal; the variance maps hold that
    variance exactly.  Noise is drawn from ``seed + 1``.
    """
    rng = np.random.default_rng(seed)
    W, H = wl.width, wl.height
    xs = rng.uniform(0, W, wl.n_sources)
    ys = rng.uniform(0, H, wl.n_sources)
    fluxes = np.exp(rng.uniform(math.log(wl.flux_lo), math.log(wl.flux_hi), wl.n_sources))
    f2 = fluxes.copy()
    if wl.variable_frac > 0:
        var = rng.uniform(0, 1, wl.n_sources) < wl.variable_frac
        f2[var] *= rng.uniform(0.5, 2.0, int(var.sum()))
    th = float(rng.uniform(0, math.pi)) if theta is None else theta
    m1 = _render(W, H, xs, ys, fluxes, wl.ref_psf, 0.0)
    m2 = _render(W, H, xs, ys, f2, wl.sci_psf, th)
    M1 = _make_mask(rng, m1, wl.mask_frac, wl.saturation)
    M2 = _make_mask(rng, m2, wl.mask_frac, wl.saturation)
    nrng = np.random.default_rng(seed + 1)
    V1 = wl.sky + m1
    V2 = wl.sky + m2
    I1 = V1 + nrng.standard_normal((H, W)) * np.sqrt(V1)
    I2 = V2 + nrng.standard_normal((H, W)) * np.sqrt(V2)
    I1 = I1.astype(np.float32)
    I2 = I2.astype(np.float32)
    V1 = V1.astype(np.float32)
    V2 = V2.astype(np.float32)
    for I, V, M in ((I1, V1, M1), (I2, V2, M2)):
        I[M != 0] = np.nan
        V[M != 0] = np.nan
    ns = wl.n_stamps if n_stamps is None else n_stamps
    stamps = select_stamps(xs, ys, fluxes, M1, M2, ns, wl.stamp_half, wl.kernel_half)
    return Pair(wl, I1, V1, M1, I2, V2, M2, stamps, xs, ys, fluxes, seed)


def scaled(wl: Workload, name: str, width: int, height: int, n_sources: Optional[int] = None,
           n_stamps: Optional[int] = None, **kw) -> Workload:
    """A smaller workload of the same structure (for tests): source density is
    kept unless ``n_sources`` is given."""
    if n_sources is None:
        n_sources = max(1, int(round(wl.n_sources * width * height / wl.pixels)))
    if n_stamps is None:
        n_stamps = wl.n_stamps
    return dataclasses.replace(wl, name=name, width=width, height=height,
                               n_sources=n_sources, n_stamps=n_stamps, **kw)


def gaussian_noise_image(rng: np.random.Generator, W: int, H: int, var: float) -> np.ndarray:
    return (rng.standard_normal((H, W)) * math.sqrt(var)).astype(np.float32)
