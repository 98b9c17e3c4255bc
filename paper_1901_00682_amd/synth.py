"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs (images, noise, masks, subdomain cuts, random
directions).  It holds none of the solver's arithmetic, and both the GPU path
and the CPU oracle are fed from it.

The paper's test images (natural photographs at 2048 x 2048 and 2048 x 3072),
its noise levels (Gaussian noise of variance 0.05, 20 % salt-and-pepper) and
its text mask (Sec. 5) are not available; piecewise-constant images of random
rectangles and discs stand in for them, with the same sizes and noise types.

Seeds: ``1000 * k + role`` for workload k with role 1 = image, 2 = noise,
3 = mask, 4 = random direction (finite differences).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

IMAGE, NOISE, MASK, DIRECTION = 1, 2, 3, 4


def rng_for(workload: int, role: int) -> np.random.Generator:
    return np.random.default_rng(1000 * workload + role)


def shapes(H: int, W: int, rng: np.random.Generator, ramp: float = 0.0) -> np.ndarray:
    """Piecewise-constant image: uniform background, then
    n = max(8, H*W // 16384) rectangles or discs painted in order (pixel-centre
    test); centre uniform over the image, half-size / radius
    U[0.02, 0.2] * min(H, W), rectangle aspect U[0.5, 2], value U[0, 1].
    ramp > 0 adds a seeded linear ramp of that amplitude (piecewise smooth)."""
    img = np.full((H, W), rng.uniform(0.0, 1.0))
    n = max(8, (H * W) // 16384)
    m = min(H, W)
    for _ in range(n):
        cy, cx = rng.uniform(0.0, H), rng.uniform(0.0, W)
        size = rng.uniform(0.02, 0.2) * m
        val = rng.uniform(0.0, 1.0)
        rect = rng.uniform() < 0.5
        aspect = rng.uniform(0.5, 2.0) if rect else 1.0
        hy, hx = size, size * aspect
        i0, i1 = max(0, int(np.floor(cy - hy - 1))), min(H, int(np.ceil(cy + hy + 1)))
        j0, j1 = max(0, int(np.floor(cx - hx - 1))), min(W, int(np.ceil(cx + hx + 1)))
        if i0 >= i1 or j0 >= j1:
            continue
        yy = np.arange(i0, i1)[:, None] + 0.5
        xx = np.arange(j0, j1)[None, :] + 0.5
        if rect:
            sel = (np.abs(yy - cy) <= hy) & (np.abs(xx - cx) <= hx)
        else:
            sel = (yy - cy) ** 2 + (xx - cx) ** 2 <= size * size
        img[i0:i1, j0:j1][sel] = val
    if ramp > 0.0:
        a, b = rng.uniform(-1.0, 1.0, size=2)
        yy = np.linspace(-0.5, 0.5, H)[:, None]
        xx = np.linspace(-0.5, 0.5, W)[None, :]
        img = img + ramp * (a * yy + b * xx)
    return img


def gaussian(shape, sd: float, rng: np.random.Generator) -> np.ndarray:
    """Additive N(0, sd^2) noise (not clipped)."""
    return rng.normal(0.0, sd, size=shape)


def salt_and_pepper(img: np.ndarray, density: float, rng: np.random.Generator) -> np.ndarray:
    """Replace a `density` fraction of pixels by 0 or 1 with equal probability."""
    out = img.copy()
    hit = rng.uniform(size=img.shape) < density
    salt = rng.uniform(size=img.shape) < 0.5
    out[hit & salt] = 1.0
    out[hit & ~salt] = 0.0
    return out


def stroke_mask(H: int, W: int, frac: float, rng: np.random.Generator, width: int = 3) -> np.ndarray:
    """Random polylines of the given width until at least `frac` of the pixels
    are missing.  Returns uint8, 1 = observed, 0 = missing (the set D)."""
    missing = np.zeros((H, W), bool)
    r = width / 2.0
    while missing.mean() < frac:
        nseg = int(rng.integers(2, 6))
        y, x = rng.uniform(0, H), rng.uniform(0, W)
        for _ in range(nseg):
            ang = rng.uniform(0, 2 * np.pi)
            length = rng.uniform(0.05, 0.3) * min(H, W)
            y2, x2 = y + length * np.sin(ang), x + length * np.cos(ang)
            steps = int(np.ceil(length / 0.5)) + 1
            for t in np.linspace(0.0, 1.0, steps):
                cy, cx = y + t * (y2 - y), x + t * (x2 - x)
                i0, i1 = max(0, int(cy - r)), min(H, int(cy + r) + 1)
                j0, j1 = max(0, int(cx - r)), min(W, int(cx + r) + 1)
                if i0 < i1 and j0 < j1:
                    missing[i0:i1, j0:j1] = True
            y, x = y2, x2
            if missing.mean() >= frac:
                break
    return (~missing).astype(np.uint8)


def floor_cuts(n: int, parts: int) -> np.ndarray:
    """Cuts floor(k n / parts), k = 0..parts."""
    return np.array([(k * n) // parts for k in range(parts + 1)], dtype=np.int32)


def tile_cuts(n: int, tile: int) -> np.ndarray:
    """Cuts at multiples of `tile` plus a ragged remainder."""
    c = list(range(0, n, tile)) + [n]
    return np.array(c, dtype=np.int32)


@dataclass
class Case:
    """One synthetic problem: data, cuts and solver settings."""

    name: str
    f: np.ndarray                 # float32 image (the GPU input; the oracle gets it widened)
    alpha: float
    row_cuts: np.ndarray
    col_cuts: np.ndarray
    fidelity: str = "L2"
    inner: str = "FISTA"
    mask: np.ndarray | None = None
    clean: np.ndarray | None = None
    n_outer: int = 100
    n_inner: int = 10
    tau: float = 50.0
    sigma: float = 0.01
    tau0: float = 10.0
    sigma0: float = 1.0 / 80.0
    gamma: float = 1.0 / 400.0
    extra: dict = field(default_factory=dict)


def rof_case(name, H, W, ny, nx, alpha, sd, n_outer, n_inner, workload, ramp=0.0) -> Case:
    clean = shapes(H, W, rng_for(workload, IMAGE), ramp=ramp)
    f = (clean + gaussian((H, W), sd, rng_for(workload, NOISE))).astype(np.float32)
    return Case(name, f, alpha, floor_cuts(H, ny), floor_cuts(W, nx), clean=clean.astype(np.float32),
                n_outer=n_outer, n_inner=n_inner)


def config1() -> Case:
    """ROF, 64 x 64, 2 x 2 subdomains of 32 x 32, noise sd 0.05, alpha 10,
    100 outer x 10 inner."""
    return rof_case("rof64_2x2", 64, 64, 2, 2, 10.0, 0.05, 100, 10, workload=1)


def config2(size: int = 2048, tile: int = 128, n_outer: int = 500) -> Case:
    """ROF, 2048 x 2048, 16 x 16 subdomains of 128 x 128, noise sd 0.1, alpha 8,
    500 outer x 5 inner (size 8192 gives the 64 x 64 DRAM-regime variant)."""
    k = size // tile
    return rof_case(f"rof{size}_{k}x{k}", size, size, k, k, 8.0, 0.1, n_outer, 5, workload=2)


def config3(H: int = 2000, W: int = 3000, ny: int = 13, nx: int = 20, n_outer: int = 1000) -> Case:
    """TV-L1 denoising + inpainting, 3000 x 2000 (W x H), 20 x 13 uneven
    subdomains, salt-and-pepper density 0.3, stroke mask with >= 10 % missing,
    f = 0 on the missing set, alpha 1.5, local accelerated primal-dual, 5 inner."""
    clean = shapes(H, W, rng_for(3, IMAGE))
    noisy = salt_and_pepper(clean, 0.3, rng_for(3, NOISE))
    mask = stroke_mask(H, W, 0.10, rng_for(3, MASK))
    f = np.where(mask == 1, noisy, 0.0).astype(np.float32)
    return Case("tvl1_inpaint", f, 1.5, floor_cuts(H, ny), floor_cuts(W, nx), fidelity="L1", inner="CP2",
                mask=mask, clean=clean.astype(np.float32), n_outer=n_outer, n_inner=5)


def config4(n_images: int = 64, lo: int = 256, hi: int = 1024, tile: int = 128, n_outer: int = 500):
    """Batch of n_images ROF problems: side lengths U{lo..hi} (independent, so
    non-square), noise sd U[0.05, 0.2], alpha U[4, 16], subdomains cut at
    multiples of `tile` with ragged remainders, 5 inner."""
    rng = rng_for(4, IMAGE)
    cases = []
    for b in range(n_images):
        H, W = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        sd = float(rng.uniform(0.05, 0.2))
        alpha = float(rng.uniform(4.0, 16.0))
        clean = shapes(H, W, rng)
        f = (clean + gaussian((H, W), sd, rng)).astype(np.float32)
        cases.append(Case(f"batch{b}", f, alpha, tile_cuts(H, tile), tile_cuts(W, tile),
                          clean=clean.astype(np.float32), n_outer=n_outer, n_inner=5))
    return cases


def config5(n_images: int = 16, size: int = 512, grid: int = 4, n_outer: int = 200):
    """Batch of ROF problems for differentiation: g clean, f = g + N(0, 0.1^2),
    alpha 8, 4 x 4 subdomains, 200 outer x 5 inner."""
    cases = []
    for b in range(n_images):
        clean = shapes(size, size, np.random.default_rng(5000 + 10 * b + IMAGE))
        f = (clean + gaussian((size, size), 0.1, np.random.default_rng(5000 + 10 * b + NOISE))).astype(np.float32)
        cases.append(Case(f"diff{b}", f, 8.0, floor_cuts(size, grid), floor_cuts(size, grid),
                          clean=clean.astype(np.float32), n_outer=n_outer, n_inner=5))
    return cases


def cv_case(size: int = 2048, tile: int = 128, n_outer: int = 500, n_inner: int = 5) -> Case:
    """Convex Chan-Vese segmentation (stand-in for the 2048 x 2048 test image of
    the segmentation experiment): the piecewise-constant shapes image plus noise
    sd 0.05, subdomains of `tile` x `tile`, alpha 10, c1 = 0.6, c2 = 0.1, outer
    tau = 1, tau sigma = 1/2, local primal-dual tau0 = 10, tau0 sigma0 = 1/8,
    gamma = 1/(8 tau)."""
    k = size // tile
    clean = shapes(size, size, rng_for(6, IMAGE))
    f = (clean + gaussian((size, size), 0.05, rng_for(6, NOISE))).astype(np.float32)
    return Case(f"cv{size}_{k}x{k}", f, 10.0, floor_cuts(size, k), floor_cuts(size, k), fidelity="CV",
                inner="CP2", clean=clean.astype(np.float32), n_outer=n_outer, n_inner=n_inner, tau=1.0,
                sigma=0.5, gamma=1.0 / 8.0, extra={"c1": 0.6, "c2": 0.1})
