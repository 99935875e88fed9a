"""Seeded synthetic porous images (inputs only).

This module draws the binary voxel images, inlet masks and outlet masks that
both the HIP path and the CPU checker consume. It holds none of the method's
arithmetic: no distance transform, no invasion, no trapping.

Every image is ``uint8`` in C order with shape ``(X, Y, Z)`` (x slowest); a
nonzero voxel is pore space, zero is solid (the paper's Boolean ``image`` with
void = True, Section 2.1). The paper's own images (the 2D images of Figures
2-10 and the 250^3 "blobs" volume of Figure 4) are not available, so these
generators stand in for them with the structures the paper describes: a
Boolean model of overlapping spheres, a dense packing of non-overlapping
spheres, and Gaussian-blurred noise thresholded at a target porosity
("blobs").

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "overlapping_spheres",
    "poisson_disks",
    "sphere_packing",
    "blurred_noise",
    "face_mask",
    "config_image",
    "batch_specs",
    "image_for_spec",
    "sha256",
    "ImageSpec",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def face_mask(shape, axis: int = 0, index: int = 0) -> np.ndarray:
    """uint8 mask with the full face ``index`` of ``axis`` set (e.g. x = 0)."""
    m = np.zeros(shape, dtype=np.uint8)
    sl = [slice(None)] * len(shape)
    sl[axis] = index
    m[tuple(sl)] = 1
    return m


# ---------------------------------------------------------------------------
# Boolean model of overlapping balls (integer centres).
# ---------------------------------------------------------------------------
def overlapping_spheres(shape=(64, 64, 64), r2: int = 16, porosity: float = 0.65,
                        seed: int = 0, margin: int | None = None) -> np.ndarray:
    """Solid = union of digital balls {|v - c|^2 <= r2} with integer centres
    drawn uniformly in the box extended by ``margin`` on every side, added one
    at a time until the pore fraction first drops to ``porosity`` or below."""
    X, Y, Z = shape
    r = int(math.isqrt(r2))
    if margin is None:
        margin = r
    rng = _rng(seed)
    img = np.ones(shape, dtype=np.uint8)
    n = X * Y * Z
    n_solid = 0
    o = np.arange(-r, r + 1)
    ball = (o[:, None, None] ** 2 + o[None, :, None] ** 2 + o[None, None, :] ** 2) <= r2
    target = (1.0 - porosity) * n
    while n_solid < target:
        c = rng.integers(low=-margin, high=np.array(shape) + margin, size=3)
        lo = c - r
        hi = c + r + 1
        a0 = np.maximum(lo, 0)
        a1 = np.minimum(hi, shape)
        if np.any(a1 <= a0):
            continue
        b = ball[a0[0] - lo[0]:a1[0] - lo[0], a0[1] - lo[1]:a1[1] - lo[1], a0[2] - lo[2]:a1[2] - lo[2]]
        view = img[a0[0]:a1[0], a0[1]:a1[1], a0[2]:a1[2]]
        newly = int(np.count_nonzero(view[b]))
        view[b] = 0
        n_solid += newly
    return img


def poisson_disks(L: int = 500, r: float = 12.0, porosity: float = 0.6, seed: int = 12,
                  scale: int = 1) -> np.ndarray:
    """One 2D geometry of overlapping solid disks, rasterised at ``scale``
    pixels per unit length: (1, L*scale, L*scale) uint8. Disk centres are a
    Poisson process over the box extended by r on every side, with intensity
    -ln(porosity) / (pi r^2), so the expected pore fraction is ``porosity``;
    a pixel is solid when its centre ((i + 0.5) / scale) lies in a disk. The
    geometry depends only on (L, r, porosity, seed), so images at several
    scales show the same structure at different resolutions."""
    rng = _rng(seed)
    lam = -math.log(porosity) / (math.pi * r * r)
    n = int(rng.poisson(lam * (L + 2 * r) ** 2))
    centres = rng.uniform(-r, L + r, size=(n, 2))
    m = L * scale
    img = np.ones((m, m), dtype=np.uint8)
    pos = (np.arange(m) + 0.5) / scale
    for cy, cx in centres:
        y0, y1 = max(int((cy - r) * scale) - 1, 0), min(int((cy + r) * scale) + 2, m)
        x0, x1 = max(int((cx - r) * scale) - 1, 0), min(int((cx + r) * scale) + 2, m)
        if y0 >= y1 or x0 >= x1:
            continue
        dy = pos[y0:y1, None] - cy
        dx = pos[None, x0:x1] - cx
        img[y0:y1, x0:x1][dy * dy + dx * dx <= r * r] = 0
    return img[None]


# ---------------------------------------------------------------------------
# Dense packing of (nearly) non-overlapping spheres with lognormal radii.
# ---------------------------------------------------------------------------
def _pack_positions(radii: np.ndarray, L: float, rng: np.random.Generator,
                    tol: float, max_iter: int) -> tuple[np.ndarray, float]:
    """Collective rearrangement in a periodic box: random start, then repeated
    pairwise overlap removal (each overlapping pair is pushed apart along its
    centre line by its overlap) until the largest overlap is below ``tol``.
    Returns the positions and the largest remaining overlap."""
    n = radii.shape[0]
    pos = rng.uniform(0.0, L, size=(n, 3))
    rsum = radii[:, None] + radii[None, :]
    iu = np.triu_indices(n, 1)
    worst = float("inf")
    for it in range(max_iter):
        d = pos[:, None, :] - pos[None, :, :]
        d -= L * np.round(d / L)
        dist = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        ov = rsum - dist
        np.fill_diagonal(ov, -1.0)
        worst = float(ov[iu].max()) if n > 1 else 0.0
        if worst < tol:
            break
        mask = ov > 0
        with np.errstate(invalid="ignore", divide="ignore"):
            unit = np.where(mask[..., None], d / np.maximum(dist, 1e-9)[..., None], 0.0)
        # push each sphere by half of each overlap it takes part in (slight
        # over-relaxation speeds the jammed phase up)
        push = 0.55 * np.where(mask, ov, 0.0)
        disp = np.einsum("ij,ijk->ik", push, unit)
        # a tiny random jiggle prevents exact cycles in jammed configurations
        disp += rng.normal(0.0, 0.01, size=disp.shape) * (it % 50 == 49)
        pos = np.mod(pos + disp, L)
    return pos, worst


def sphere_packing(shape=(200, 200, 200), porosity: float = 0.40, r_mean: float = 12.0,
                   r_sd: float = 3.0, seed: int = 0, tol: float = 0.5,
                   max_iter: int = 4000, r_min: float = 1.5) -> tuple[np.ndarray, dict]:
    """Random packing of spheres with lognormal radii (mean ``r_mean``, sd
    ``r_sd`` voxels) in a periodic cubic box, rasterised as |v - c|^2 <= r^2
    with periodic wrap. Spheres are drawn until their total volume reaches the
    solid fraction ``1 - porosity``; the packer then removes overlaps until the
    largest is below ``tol`` voxels. If it cannot (the target is beyond the
    jamming density), the remaining overlap is accepted and recorded."""
    X, Y, Z = shape
    if not (X == Y == Z):
        raise ValueError("sphere_packing needs a cubic box")
    L = float(X)
    rng = _rng(seed)
    s2 = math.log(1.0 + (r_sd / r_mean) ** 2)
    mu = math.log(r_mean) - 0.5 * s2
    target = (1.0 - porosity) * L ** 3
    radii = []
    vol = 0.0
    while vol < target:
        r = float(rng.lognormal(mu, math.sqrt(s2)))
        r = max(r, r_min)
        r = min(r, 0.45 * L)
        radii.append(r)
        vol += 4.0 / 3.0 * math.pi * r ** 3
    radii = np.array(radii)
    pos, worst = _pack_positions(radii, L, rng, tol, max_iter)
    img = np.ones(shape, dtype=np.uint8)
    for (cx, cy, cz), r in zip(pos, radii):
        R = int(math.floor(r)) + 1
        ix = np.arange(int(math.floor(cx)) - R, int(math.floor(cx)) + R + 2)
        iy = np.arange(int(math.floor(cy)) - R, int(math.floor(cy)) + R + 2)
        iz = np.arange(int(math.floor(cz)) - R, int(math.floor(cz)) + R + 2)
        dx2 = (ix - cx) ** 2
        dy2 = (iy - cy) ** 2
        dz2 = (iz - cz) ** 2
        inside = (dx2[:, None, None] + dy2[None, :, None] + dz2[None, None, :]) <= r * r
        sub = img[np.ix_(ix % X, iy % Y, iz % Z)]
        sub[inside] = 0
        img[np.ix_(ix % X, iy % Y, iz % Z)] = sub
    info = {"n_spheres": int(radii.shape[0]), "max_overlap": worst,
            "porosity": float(img.mean())}
    return img, info


# ---------------------------------------------------------------------------
# Gaussian-blurred noise thresholded at a target porosity ("blobs").
# ---------------------------------------------------------------------------
def blurred_noise(shape=(512, 512, 512), sigma: float = 6.0, porosity: float = 0.55,
                  seed: int = 0) -> np.ndarray:
    """N(0, 1) float32 noise, periodic Gaussian blur of width ``sigma`` voxels
    (applied in Fourier space), pore = the floor(porosity * N) smallest values
    (a threshold at the empirical quantile)."""
    import scipy.fft as sfft

    rng = _rng(seed)
    a = rng.standard_normal(size=shape, dtype=np.float32)
    F = sfft.rfftn(a, workers=-1)
    del a
    freqs = [np.fft.fftfreq(n).astype(np.float32) for n in shape[:-1]]
    freqs.append(np.fft.rfftfreq(shape[-1]).astype(np.float32))
    c = np.float32(-2.0 * math.pi ** 2 * sigma ** 2)
    g = [np.exp(c * f * f) for f in freqs]
    F *= g[0][:, None, None]
    F *= g[1][None, :, None]
    F *= g[2][None, None, :]
    b = sfft.irfftn(F, s=shape, workers=-1).astype(np.float32, copy=False)
    del F
    n = b.size
    k = int(math.floor(porosity * n))
    if k <= 0:
        return np.zeros(shape, dtype=np.uint8)
    if k >= n:
        return np.ones(shape, dtype=np.uint8)
    flat = b.reshape(-1)
    t = np.partition(flat, k - 1)[k - 1]
    return (b <= t).astype(np.uint8)


# ---------------------------------------------------------------------------
# The named workloads.
# ---------------------------------------------------------------------------
@dataclass
class ImageSpec:
    kind: str            # "spheres" | "packing" | "noise"
    L: int
    porosity: float
    seed: int
    sigma: float = 6.0
    r_mean: float = 12.0
    r_sd: float = 3.0
    extra: dict = field(default_factory=dict)


def image_for_spec(s: ImageSpec) -> np.ndarray:
    shape = (s.L, s.L, s.L)
    if s.kind == "spheres":
        return overlapping_spheres(shape, porosity=s.porosity, seed=s.seed)
    if s.kind == "packing":
        img, info = sphere_packing(shape, porosity=s.porosity, r_mean=s.r_mean,
                                   r_sd=s.r_sd, seed=s.seed, max_iter=1500)
        s.extra.update(info)
        return img
    if s.kind == "noise":
        return blurred_noise(shape, sigma=s.sigma, porosity=s.porosity, seed=s.seed)
    raise ValueError(s.kind)


def config_image(name: str, seed: int = 0) -> np.ndarray:
    """The three single-image workloads:
    ``spheres64``  64^3 overlapping balls of radius 4, porosity 0.65;
    ``packing200`` 200^3 packing, lognormal radii mean 12 sd 3, porosity ~0.40;
    ``noise512``   512^3 blurred noise, sigma 6, porosity 0.55."""
    if name == "spheres64":
        return overlapping_spheres((64, 64, 64), r2=16, porosity=0.65, seed=seed)
    if name == "packing200":
        img, _ = sphere_packing((200, 200, 200), porosity=0.40, r_mean=12.0, r_sd=3.0, seed=seed)
        return img
    if name == "noise512":
        return blurred_noise((512, 512, 512), sigma=6.0, porosity=0.55, seed=seed)
    raise ValueError(name)


def batch_specs(n: int = 96, lo: int = 32, hi: int = 192) -> list[ImageSpec]:
    """Uneven-size batch: image i has seed i, side uniform in [lo, hi], even i
    a sphere packing (radii scaled with the side), odd i blurred noise with
    sigma 2 + 4 (L - lo) / (hi - lo); porosity uniform in [0.35, 0.70]."""
    out = []
    for i in range(n):
        rng = _rng(i)
        L = int(rng.integers(lo, hi + 1))
        phi = float(rng.uniform(0.35, 0.70))
        if i % 2 == 0:
            rm = max(3.0, 12.0 * L / 200.0)
            out.append(ImageSpec("packing", L, phi, i, r_mean=rm, r_sd=rm / 4.0))
        else:
            sg = 2.0 + 4.0 * (L - lo) / float(hi - lo)
            out.append(ImageSpec("noise", L, phi, i, sigma=sg))
    return out


# ---------------------------------------------------------------------------
# Serving stream: many blurred-noise requests up to 768^3, generated on the
# device (the host FFT of a 768^3 volume takes seconds per image).
# ---------------------------------------------------------------------------
def serve_specs(n: int = 256, lo: int = 64, hi: int = 768, seed0: int = 1000) -> list[ImageSpec]:
    """Request j has seed seed0 + j, side round(exp(U[ln lo, ln hi])) (log-
    uniform), porosity U[0.45, 0.65], blurred noise of sigma 6."""
    out = []
    for j in range(n):
        rng = _rng(seed0 + j)
        L = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        phi = float(rng.uniform(0.45, 0.65))
        out.append(ImageSpec("noise", L, phi, seed0 + j, sigma=6.0))
    return out


def blurred_noise_device(shape, sigma: float, porosity: float, seed: int, device):
    """The blurred-noise recipe of ``blurred_noise`` computed with torch on a
    device: N(0, 1) float32 noise from torch's generator seeded with ``seed``,
    periodic Gaussian blur in Fourier space, pore = values at or below the
    ``porosity`` quantile of 2^21 sampled values. Returns a uint8 device
    tensor (1 = pore). Not bit-identical to ``blurred_noise`` (another
    generator); used where the host generator is too slow."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    a = torch.randn(tuple(shape), generator=g, device=device, dtype=torch.float32)
    F = torch.fft.rfftn(a)
    del a
    c = -2.0 * math.pi ** 2 * sigma ** 2
    fz = torch.fft.fftfreq(shape[0], device=device)
    fy = torch.fft.fftfreq(shape[1], device=device)
    fx = torch.fft.rfftfreq(shape[2], device=device)
    F *= torch.exp(c * fz * fz)[:, None, None]
    F *= torch.exp(c * fy * fy)[None, :, None]
    F *= torch.exp(c * fx * fx)[None, None, :]
    b = torch.fft.irfftn(F, s=tuple(shape))
    del F
    n = b.numel()
    idx = torch.randint(0, n, (1 << 21,), generator=g, device=device)
    t = torch.quantile(b.reshape(-1)[idx], porosity)
    return (b <= t).to(torch.uint8)
