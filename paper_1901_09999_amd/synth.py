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
    "pair512": Workload("pair512", 512, 512, 200, PsfField(1.5, 1.5), PsfField(2.2, 2.2),
                     0.0, 10, ISIS_SIGMAS, ISIS_DEGREES, 0, 50, 20),
    # Plain FP32 GPU path with a spatially varying science PSF and a 10% mask.
    "pair2048": Workload("pair2048", 2048, 2048, 2000, PsfField(1.2, 1.2), PsfField(1.4, 2.6, 0.2),
                     0.10, 10, ISIS_SIGMAS, ISIS_DEGREES, 2, 100, 20),
    # Detector-chip-sized pair (GPC1 chip), 15% mask, 25x25 kernel, order 3.
    "chip4846": Workload("chip4846", 4846, 4868, 8000, PsfField(1.2, 1.2), PsfField(1.4, 2.6, 0.2),
                     0.15, 12, ISIS_SIGMAS, ISIS_DEGREES, 3, 400, 24),
}


# seed index of each named workload (pair k of a workload uses
# SEED_BASE + 1000 * index + k)
SEED_INDEX: Dict[str, int] = {"pair512": 0, "pair2048": 1, "chip4846": 2, "batch64": 3, "cells200k": 4}


def workload_seed(index: int, pair: int = 0) -> int:
    return SEED_BASE + 1000 * index + pair


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


def _pick_stamps(xs, ys, fluxes, W: int, H: int, n_stamps: int, r: int, h: int,
                 grid: Optional[int], footprint_bad) -> np.ndarray:
    """Candidate walk shared by both stamp pickers: the brightest source in
    each cell of a subregion grid whose footprint lies inside the image and
    passes ``footprint_bad(x, y)`` (False = clean); further passes take the
    next-brightest per cell until ``n_stamps`` are found (or candidates run
    out)."""
    if grid is None:
        grid = max(1, int(math.ceil(math.sqrt(n_stamps))))
    cx = np.clip((xs * grid / W).astype(int), 0, grid - 1)
    cy = np.clip((ys * grid / H).astype(int), 0, grid - 1)
    order = np.argsort(-fluxes, kind="stable")
    cells: Dict[Tuple[int, int], List[int]] = {}
    for k in order:
        cells.setdefault((int(cx[k]), int(cy[k])), []).append(int(k))
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
                if footprint_bad(x, y):
                    continue
                chosen.append((x, y))
                taken.add((x, y))
                progress = True
                break
        if not progress:
            break
    return np.asarray(chosen, dtype=np.int32).reshape(-1, 2)


def select_stamps(xs, ys, fluxes, M1, M2, n_stamps: int, r: int, h: int,
                  grid: Optional[int] = None) -> np.ndarray:
    """Pick stamp centres from the known catalogue (see :func:`_pick_stamps`):
    the footprint [x-r-h, x+r+h]^2 must be clean in M1 and the stamp
    [x-r, x+r]^2 clean in M2."""
    H, W = M1.shape
    # summed-area tables make the footprint tests O(1)
    sat1 = np.pad((M1 != 0).astype(np.int64).cumsum(0).cumsum(1), ((1, 0), (1, 0)))
    sat2 = np.pad((M2 != 0).astype(np.int64).cumsum(0).cumsum(1), ((1, 0), (1, 0)))

    def box_any(sat, x0, y0, x1, y1):
        return (sat[y1 + 1, x1 + 1] - sat[y0, x1 + 1] - sat[y1 + 1, x0] + sat[y0, x0]) > 0

    def bad(x, y):
        R = r + h
        return box_any(sat1, x - R, y - R, x + R, y + R) or box_any(sat2, x - r, y - r, x + r, y + r)

    return _pick_stamps(xs, ys, fluxes, W, H, n_stamps, r, h, grid, bad)


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


# --------------------------------------------------------------------------
# Batches of independent pairs of uneven size, rendered on the GPU.

@dataclasses.dataclass(frozen=True)
class BatchSpec:
    """Many independent pairs: per pair W, H ~ U{size_lo..size_hi}; PSF widths
    of the two images ~ U[sigma_lo, sigma_hi] (the narrower image is the one
    convolved), ellipticity up to U[0, e_max]; sources at ``density`` per
    pixel; ``mask_frac`` masked; n_stamps ~ U{stamps_lo..stamps_hi}; spatial
    order ~ U{0..S_max}; a ``variable_frac`` share of variable sources."""

    n_pairs: int = 64
    size_lo: int = 1024
    size_hi: int = 6000
    sigma_lo: float = 1.0
    sigma_hi: float = 3.0
    e_max: float = 0.3
    density: float = 2000.0 / (2048 * 2048)
    mask_frac: float = 0.10
    kernel_half: int = 10
    stamp_half: int = 20
    stamps_lo: int = 50
    stamps_hi: int = 400
    S_max: int = 3
    variable_frac: float = 0.05


BATCHES: Dict[str, BatchSpec] = {"batch64": BatchSpec()}


def batch_pair_workload(spec: BatchSpec, k: int, cfg_index: int = 3) -> Workload:
    """The workload of pair k of a batch, drawn from seed 19010999 + 1000 cfg + k."""
    rng = np.random.default_rng(workload_seed(cfg_index, k))
    W = int(rng.integers(spec.size_lo, spec.size_hi + 1))
    H = int(rng.integers(spec.size_lo, spec.size_hi + 1))
    s_a, s_b = rng.uniform(spec.sigma_lo, spec.sigma_hi, 2)
    e_a, e_b = rng.uniform(0.0, spec.e_max, 2)
    lo, hi = (s_a, s_b) if s_a <= s_b else (s_b, s_a)
    n_st = int(rng.integers(spec.stamps_lo, spec.stamps_hi + 1))
    S = int(rng.integers(0, spec.S_max + 1))
    return Workload(f"pair{k}", W, H, max(1, int(round(spec.density * W * H))),
                    PsfField(lo, lo, e_a), PsfField(hi, hi, e_b), spec.mask_frac,
                    spec.kernel_half, ISIS_SIGMAS, ISIS_DEGREES, S, n_st, spec.stamp_half,
                    variable_frac=spec.variable_frac)


@dataclasses.dataclass
class DevicePair:
    """A pair whose planes live in device memory (torch tensors)."""
    workload: Workload
    I1: "object"
    V1: "object"
    M1: "object"
    I2: "object"
    V2: "object"
    M2: "object"
    stamps: np.ndarray
    xs: np.ndarray
    ys: np.ndarray
    fluxes: np.ndarray
    seed: int

    def host(self) -> Pair:
        t = lambda a: a.cpu().numpy()
        return Pair(self.workload, t(self.I1), t(self.V1), t(self.M1), t(self.I2), t(self.V2),
                    t(self.M2), self.stamps, self.xs, self.ys, self.fluxes, self.seed)


def _render_torch(torch, W, H, xs, ys, fluxes, psf: PsfField, theta: float, device):
    """Device version of :func:`_render` (float32): each source's elliptical
    Gaussian on a fixed +-6 sigma_a box, scatter-added into the image."""
    sa, sb = psf.params(xs, ys, W, H)
    rad = int(math.ceil(6.0 * float(np.max(sa)))) + 1 if len(xs) else 1
    img = torch.zeros(H * W, dtype=torch.float32, device=device)
    off = torch.arange(-rad, rad + 1, device=device)
    c, s = math.cos(theta), math.sin(theta)
    chunk = max(1, (1 << 24) // (2 * rad + 1) ** 2)
    for i0 in range(0, len(xs), chunk):
        sl = slice(i0, i0 + chunk)
        x0 = torch.as_tensor(xs[sl], dtype=torch.float64, device=device)
        y0 = torch.as_tensor(ys[sl], dtype=torch.float64, device=device)
        a = torch.as_tensor(sa[sl], dtype=torch.float64, device=device)
        b = torch.as_tensor(sb[sl], dtype=torch.float64, device=device)
        f = torch.as_tensor(fluxes[sl], dtype=torch.float64, device=device)
        px = torch.floor(x0).long()[:, None, None] + off[None, None, :]
        py = torch.floor(y0).long()[:, None, None] + off[None, :, None]
        dx = px - x0[:, None, None]
        dy = py - y0[:, None, None]
        pa = c * dx + s * dy
        pb = -s * dx + c * dy
        q = (pa / a[:, None, None]) ** 2 + (pb / b[:, None, None]) ** 2
        val = (f / (2.0 * math.pi * a * b))[:, None, None] * torch.exp(-0.5 * q)
        ok = (px >= 0) & (px < W) & (py >= 0) & (py < H)
        idx = (py * W + px)[ok]
        img.index_add_(0, idx, val[ok].to(torch.float32))
    return img.view(H, W)


def _mask_torch(torch, rng, model, frac: float, saturation: float):
    H, W = model.shape
    mask = torch.zeros((H, W), dtype=torch.bool, device=model.device)
    if frac <= 0:
        return mask.to(torch.uint8)
    sat = model > saturation
    d = sat.clone()
    d[1:, :] |= sat[:-1, :]
    d[:-1, :] |= sat[1:, :]
    d[:, 1:] |= sat[:, :-1]
    d[:, :-1] |= sat[:, 1:]
    mask |= d
    colbad = mask.float().mean(0)                       # masked share of each column
    cols = torch.zeros(W, dtype=torch.bool, device=model.device)
    frac_now = float(mask.float().mean())
    while frac_now < frac:
        w = int(rng.integers(4, 65))
        x0 = int(rng.integers(0, max(W - w, 1)))
        cols[x0:x0 + w] = True
        frac_now = float(torch.where(cols, torch.ones_like(colbad), colbad).mean())
    mask[:, cols] = True
    return mask.to(torch.uint8)


def make_pair_device(wl: Workload, seed: int, device="cuda", n_stamps: Optional[int] = None) -> DevicePair:
    """Render a pair on the GPU with torch (same recipe as :func:`make_pair`:
    sources, variable share, masks, noise, NaN in masked pixels, stamps from
    the catalogue; the random streams differ from the CPU generator's)."""
    import torch

    rng = np.random.default_rng(seed)
    W, H = wl.width, wl.height
    xs = rng.uniform(0, W, wl.n_sources)
    ys = rng.uniform(0, H, wl.n_sources)
    fluxes = np.exp(rng.uniform(math.log(wl.flux_lo), math.log(wl.flux_hi), wl.n_sources))
    f2 = fluxes.copy()
    if wl.variable_frac > 0:
        var = rng.uniform(0, 1, wl.n_sources) < wl.variable_frac
        f2[var] *= rng.uniform(0.5, 2.0, int(var.sum()))
    th = float(rng.uniform(0, math.pi))
    m1 = _render_torch(torch, W, H, xs, ys, fluxes, wl.ref_psf, 0.0, device)
    m2 = _render_torch(torch, W, H, xs, ys, f2, wl.sci_psf, th, device)
    M1 = _mask_torch(torch, rng, m1, wl.mask_frac, wl.saturation)
    M2 = _mask_torch(torch, rng, m2, wl.mask_frac, wl.saturation)
    g = torch.Generator(device=device)
    g.manual_seed(seed + 1)
    V1 = m1 + wl.sky
    V2 = m2 + wl.sky
    del m1, m2
    I1 = V1 + torch.randn((H, W), generator=g, device=device) * torch.sqrt(V1)
    I2 = V2 + torch.randn((H, W), generator=g, device=device) * torch.sqrt(V2)
    nan = torch.tensor(float("nan"), device=device)
    I1 = torch.where(M1 != 0, nan, I1)
    V1 = torch.where(M1 != 0, nan, V1)
    I2 = torch.where(M2 != 0, nan, I2)
    V2 = torch.where(M2 != 0, nan, V2)
    # footprint tests through summed-area tables on the device
    r, h = wl.stamp_half, wl.kernel_half

    def box_bad(M, R):
        sat = torch.nn.functional.pad((M != 0).to(torch.int32).cumsum(0).cumsum(1), (1, 0, 1, 0))
        Hh, Ww = M.shape
        out = torch.ones((Hh, Ww), dtype=torch.bool, device=M.device)
        if 2 * R + 1 <= min(Hh, Ww):
            y0, x0 = R, R
            box = (sat[2 * R + 1:, 2 * R + 1:] - sat[:-2 * R - 1, 2 * R + 1:]
                   - sat[2 * R + 1:, :-2 * R - 1] + sat[:-2 * R - 1, :-2 * R - 1])
            out[y0:Hh - R, x0:Ww - R] = box > 0
        return out.cpu().numpy()

    bad1 = box_bad(M1, r + h)
    bad2 = box_bad(M2, r)
    ns = wl.n_stamps if n_stamps is None else n_stamps
    stamps = _pick_stamps(xs, ys, fluxes, W, H, ns, r, h, None,
                          lambda x, y: bool(bad1[y, x]) or bool(bad2[y, x]))
    return DevicePair(wl, I1.contiguous(), V1.contiguous(), M1, I2.contiguous(), V2.contiguous(),
                      M2, stamps, xs, ys, fluxes, seed)


def make_batch_device(name: str = "batch64", log=None):
    """The pairs of batch ``name`` rendered on the GPU, each from its own
    seed: returns (workloads, device pairs)."""
    import torch

    spec = BATCHES[name]
    seed_index = SEED_INDEX[name]
    wls = [batch_pair_workload(spec, k, seed_index) for k in range(spec.n_pairs)]
    dps = []
    for k, wl in enumerate(wls):
        dps.append(make_pair_device(wl, workload_seed(seed_index, k)))
        if log and k % 16 == 15:
            torch.cuda.synchronize()
            log(f"generated {k + 1}/{len(wls)} pairs")
    return wls, dps


# --------------------------------------------------------------------------
# Single-star stamp pairs for the learned prior (one star per 64 x 64 cell).

@dataclasses.dataclass(frozen=True)
class StampSetSpec:
    """Cells of one target star each: PSF widths of the two images ~
    U[sigma_lo, sigma_hi] (the narrower image is image 1, the one convolved),
    ellipticity ~ U[0, e_max] at a random angle, S/N ~ log-U[snr_lo, snr_hi]
    with S/N = F / sqrt(F + 4 pi sigma^2 sky) for image 1, image-2 flux F
    times U[ratio_lo, ratio_hi], sub-pixel centre offsets; Poisson-many
    neighbour sources at the field density (fluxes log-U[flux_lo, flux_hi],
    same PSFs and flux ratio); sky and Gaussian noise of variance sky +
    signal, no masks."""

    n: int = 200_000
    side: int = 64
    sigma_lo: float = 1.0
    sigma_hi: float = 3.0
    e_max: float = 0.3
    snr_lo: float = 20.0
    snr_hi: float = 500.0
    ratio_lo: float = 0.7
    ratio_hi: float = 1.4
    sky: float = 100.0
    neighbours: float = 2000.0 / (2048 * 2048)   # other sources per pixel (field density)
    flux_lo: float = 1e3                          # neighbour fluxes, log-uniform
    flux_hi: float = 1e5


STAMP_SETS: Dict[str, StampSetSpec] = {"cells200k": StampSetSpec()}


def _star_cells(torch, side, x0, y0, flux, sig, e, theta, device):
    """[n, side, side] pixel-sampled elliptical Gaussians (float32)."""
    n = x0.shape[0]
    sa = sig / np.sqrt(1.0 - e)
    sb = sig * np.sqrt(1.0 - e)
    t = lambda a: torch.as_tensor(a, dtype=torch.float32, device=device)[:, None, None]
    g = torch.arange(side, dtype=torch.float32, device=device)
    dx = g[None, None, :] - t(x0)
    dy = g[None, :, None] - t(y0)
    c, s = t(np.cos(theta)), t(np.sin(theta))
    pa = c * dx + s * dy
    pb = -s * dx + c * dy
    q = (pa / t(sa)) ** 2 + (pb / t(sb)) ** 2
    return t(flux / (2.0 * np.pi * sa * sb)) * torch.exp(-0.5 * q)


def make_stamp_cells(spec: StampSetSpec, n: int, seed: int, device="cuda"):
    """n cells stacked into one tall image pair [n * side, side] with the stamp
    centres at the cell centres.  Returns (planes dict, stamps int32 [n, 2],
    parameters dict of numpy arrays)."""
    import torch

    rng = np.random.default_rng(seed)
    side = spec.side
    s_a = rng.uniform(spec.sigma_lo, spec.sigma_hi, n)
    s_b = rng.uniform(spec.sigma_lo, spec.sigma_hi, n)
    sig1, sig2 = np.minimum(s_a, s_b), np.maximum(s_a, s_b)
    e1, e2 = rng.uniform(0.0, spec.e_max, n), rng.uniform(0.0, spec.e_max, n)
    th1, th2 = rng.uniform(0.0, math.pi, n), rng.uniform(0.0, math.pi, n)
    snr = np.exp(rng.uniform(math.log(spec.snr_lo), math.log(spec.snr_hi), n))
    bkg = 4.0 * math.pi * sig1 ** 2 * spec.sky
    F1 = 0.5 * (snr ** 2 + np.sqrt(snr ** 4 + 4.0 * snr ** 2 * bkg))
    ratio = rng.uniform(spec.ratio_lo, spec.ratio_hi, n)
    F2 = F1 * ratio
    cx = side // 2 + rng.uniform(-0.5, 0.5, n)
    cy = side // 2 + rng.uniform(-0.5, 0.5, n)
    m1 = _star_cells(torch, side, cx, cy, F1, sig1, e1, th1, device)
    m2 = _star_cells(torch, side, cx, cy, F2, sig2, e2, th2, device)
    # neighbours: up to 8 slots per cell, each present with the Poisson-thinned probability
    lam = spec.neighbours * side * side
    slots = 8
    present = rng.uniform(0, 1, (slots, n)) < lam / slots
    for k in range(slots):
        nx = rng.uniform(0, side, n)
        ny = rng.uniform(0, side, n)
        nf = np.exp(rng.uniform(math.log(spec.flux_lo), math.log(spec.flux_hi), n)) * present[k]
        m1 += _star_cells(torch, side, nx, ny, nf, sig1, e1, th1, device)
        m2 += _star_cells(torch, side, nx, ny, nf * ratio, sig2, e2, th2, device)
    g = torch.Generator(device=device)
    g.manual_seed(seed + 1)
    V1 = (m1 + spec.sky).reshape(n * side, side)
    V2 = (m2 + spec.sky).reshape(n * side, side)
    del m1, m2
    I1 = V1 + torch.randn(V1.shape, generator=g, device=device) * torch.sqrt(V1)
    I2 = V2 + torch.randn(V2.shape, generator=g, device=device) * torch.sqrt(V2)
    M = torch.zeros((n * side, side), dtype=torch.uint8, device=device)
    stamps = np.stack([np.full(n, side // 2), side * np.arange(n) + side // 2], 1).astype(np.int32)
    params = dict(sigma1=sig1, sigma2=sig2, e1=e1, e2=e2, snr=snr, ratio=ratio)
    return dict(I1=I1, V1=V1, M1=M, I2=I2, V2=V2, M2=M.clone()), stamps, params
