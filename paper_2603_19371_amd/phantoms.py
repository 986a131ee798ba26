"""Seeded synthetic image pairs with a known true displacement field.

The paper's data sets (brain MRI, lung CT, abdominal MR/CT) are not available;
these generators stand in for them with volumes of the same shapes and of a
similar structure.  Every pair is built as

    F = F0 + noise_F,   M = F0 o (Id + t)^-1 + noise_M

so that M o (Id + t) = F0 and the true field is ``t``.  The inverse map is
found by the fixed-point iteration w(y) = -t(y + w(y)).

This module holds no arithmetic of the registration method: resampling here is
scipy's (``map_coordinates``, ``gaussian_filter``, ``zoom``), and nothing here
is imported by the GPU library or by the oracle except as input data.  All
randomness comes from ``numpy.random.default_rng(seed)``; arrays are produced
in float64 and returned as float32 [z][y][x] volumes and [3][z][y][x] fields
(component 0/1/2 = displacement along x/y/z, voxel units).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage as ndi


@dataclass
class Phantom:
    F: np.ndarray                 # fixed image, float32 [z][y][x]
    M: np.ndarray                 # moving image, float32 [z][y][x]
    t: np.ndarray                 # true field, float32 [3][z][y][x]
    labels: np.ndarray | None = None   # uint8 label map of F (when defined)
    meta: dict = field(default_factory=dict)


def _grid(shape):
    return np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape],
                       indexing="ij")


def _smooth_field(rng, shape, sigma, max_disp, coarse=1):
    """Random field: N(0,1) per component, Gaussian-smoothed (sigma voxels),
    scaled so that max_x ||t(x)||_2 = max_disp.  For large volumes the noise is
    drawn on a grid ``coarse`` times smaller and linearly upsampled."""
    cshape = tuple(max(2, s // coarse) for s in shape)
    t = rng.standard_normal((3,) + cshape)
    for c in range(3):
        t[c] = ndi.gaussian_filter(t[c], sigma / coarse, mode="reflect")
    if coarse > 1:
        t = np.stack([ndi.zoom(t[c], [s / cs for s, cs in zip(shape, cshape)],
                               order=1, mode="nearest", grid_mode=True)
                      for c in range(3)])
    mag = np.sqrt((t ** 2).sum(0)).max()
    return t * (max_disp / mag)


def _coords(shape, disp):
    """Array-axis sample coordinates of x + disp(x); disp is [3] in x,y,z order."""
    zz, yy, xx = _grid(shape)
    return np.stack([zz + disp[2], yy + disp[1], xx + disp[0]])


def invert_field(t, iters=50, coarse=1):
    """w with (Id + t) o (Id + w) = Id, by w <- -t(Id + w).  With coarse > 1
    the iteration runs on a grid subsampled by ``coarse`` and is upsampled."""
    shape = t.shape[1:]
    if coarse > 1:
        tc = np.stack([ndi.zoom(t[c], 1.0 / coarse, order=1, mode="nearest",
                                grid_mode=True) for c in range(3)]) / coarse
        wc = invert_field(tc, iters, 1) * coarse
        return np.stack([ndi.zoom(wc[c], [s / cs for s, cs in
                                          zip(shape, wc.shape[1:])],
                                  order=1, mode="nearest", grid_mode=True)
                         for c in range(3)])
    w = np.zeros_like(t)
    for _ in range(iters):
        cr = _coords(shape, w)
        w = -np.stack([ndi.map_coordinates(t[c], cr, order=1, mode="nearest")
                       for c in range(3)])
    return w


def _resample(img, disp, order=1):
    return ndi.map_coordinates(img, _coords(img.shape, disp), order=order,
                               mode="nearest")


# --------------------------------------------------------------- blobs (32^3)
def blobs(shape=(32, 32, 32), seed=0, n_blobs=20, sigma_range=(2.0, 6.0),
          amp_range=(0.2, 1.0), noise=0.01, field_sigma=4.0, max_disp=2.0):
    """Sum of isotropic Gaussian blobs (centres uniform in the volume) plus
    N(0, noise^2); the moving image is the blob image under the inverse of a
    smoothed random field (field_sigma, max_disp voxels)."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    cen = rng.uniform(0, 1, (n_blobs, 3)) * np.array(shape)
    sig = rng.uniform(*sigma_range, n_blobs)
    amp = rng.uniform(*amp_range, n_blobs)
    t = _smooth_field(rng, shape, field_sigma, max_disp)
    w = invert_field(t)

    def render(zz, yy, xx):
        out = np.zeros_like(zz)
        for c, s, a in zip(cen, sig, amp):
            d2 = (zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2
            out += a * np.exp(-d2 / (2 * s * s))
        return out

    zz, yy, xx = _grid(shape)
    F0 = render(zz, yy, xx)
    M0 = render(zz + w[2], yy + w[1], xx + w[0])   # blobs are analytic
    F = F0 + noise * rng.standard_normal(shape)
    M = M0 + noise * rng.standard_normal(shape)
    return Phantom(F.astype(np.float32), M.astype(np.float32),
                   t.astype(np.float32), None,
                   dict(kind="blobs", seed=seed, shape=shape))


# ------------------------------------------------------ brain (160x192x224)
BRAIN_LEVELS = (0.15, 0.30, 0.45, 0.60, 0.75, 0.90)


def brain(shape=(160, 192, 224), seed=0, n_classes=6, class_sigma=8.0,
          pv_sigma=0.7, noise=0.01, field_sigma=8.0, max_disp=6.0):
    """Brain-MRI-like volume: an ellipsoidal head mask (semi-axes 0.42 of the
    shape) filled with ``n_classes`` tissue classes, each the argmax region of
    independently smoothed noise, with piecewise-constant intensities, light
    partial-volume blur and additive noise."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    coarse = 4 if min(shape) >= 64 else 1
    cshape = tuple(max(2, s // coarse) for s in shape)
    fields = rng.standard_normal((n_classes,) + cshape)
    for k in range(n_classes):
        fields[k] = ndi.gaussian_filter(fields[k], class_sigma / coarse,
                                        mode="reflect")
    if coarse > 1:
        fields = np.stack([ndi.zoom(fields[k], [s / cs for s, cs in
                                                zip(shape, cshape)],
                                    order=1, mode="nearest", grid_mode=True)
                           for k in range(n_classes)])
    lab = np.argmax(fields, axis=0).astype(np.uint8) + 1
    zz, yy, xx = _grid(shape)
    ctr = [(s - 1) / 2 for s in shape]
    ax = [0.42 * s for s in shape]
    inside = (((zz - ctr[0]) / ax[0]) ** 2 + ((yy - ctr[1]) / ax[1]) ** 2 +
              ((xx - ctr[2]) / ax[2]) ** 2) <= 1.0
    del zz, yy, xx
    lab[~inside] = 0
    table = np.array((0.0,) + BRAIN_LEVELS[:n_classes])
    F0 = ndi.gaussian_filter(table[lab], pv_sigma, mode="constant")
    t = _smooth_field(rng, shape, field_sigma, max_disp, coarse=coarse)
    w = invert_field(t, iters=30, coarse=coarse)
    M0 = _resample(F0, w, order=1)
    F = F0 + noise * rng.standard_normal(shape)
    M = M0 + noise * rng.standard_normal(shape)
    return Phantom(F.astype(np.float32), M.astype(np.float32),
                   t.astype(np.float32), lab,
                   dict(kind="brain", seed=seed, shape=shape))


# -------------------------------------------------------------- lung (384^3)
def lung(shape=(384, 384, 384), seed=0, field_sigma=8.0, max_disp=6.0,
         n_chains=24, chain_len=80):
    """Lung-CT-like volume in HU: air (-1000) outside an elliptical body of
    soft tissue (+40), two dark lobes (-850) and a tree of vessels (random-walk
    chains of Gaussian blobs, up to +400) inside the lobes; clipped to
    [-1000, 400] and min-max normalised to [0, 1]."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    nz, ny, nx = shape
    zz, yy, xx = _grid(shape)
    body = (((zz - nz / 2) / (0.46 * nz)) ** 2 + ((yy - ny / 2) / (0.36 * ny)) ** 2
            + ((xx - nx / 2) / (0.46 * nx)) ** 2) <= 1.0
    hu = np.full(shape, -1000.0)
    hu[body] = 40.0
    lobes = []
    for side in (-1, 1):
        c = np.array([nz * 0.5, ny * 0.5, nx * (0.5 + side * 0.2)])
        a = np.array([0.36 * nz, 0.26 * ny, 0.17 * nx])
        lobe = (((zz - c[0]) / a[0]) ** 2 + ((yy - c[1]) / a[1]) ** 2 +
                ((xx - c[2]) / a[2]) ** 2) <= 1.0
        hu[lobe] = -850.0
        lobes.append((c, a, lobe))
    del zz, yy, xx
    vessel = np.zeros(shape)
    scale = min(shape) / 384.0
    for c, a, lobe in lobes:
        for _ in range(n_chains):
            p = c + (rng.uniform(-0.5, 0.5, 3) * a)
            d = rng.standard_normal(3)
            d /= np.linalg.norm(d)
            rad = rng.uniform(1.5, 3.0) * scale + 0.6
            for _ in range(chain_len):
                ip = np.round(p).astype(int)
                if np.any(ip < 0) or np.any(ip >= np.array(shape)) or not lobe[tuple(ip)]:
                    break
                r = int(np.ceil(3 * rad))
                lo = np.maximum(ip - r, 0)
                hi = np.minimum(ip + r + 1, np.array(shape))
                gz, gy, gx = [np.arange(lo[k], hi[k], dtype=np.float64)
                              for k in range(3)]
                d2 = ((gz[:, None, None] - p[0]) ** 2 + (gy[None, :, None] - p[1]) ** 2
                      + (gx[None, None, :] - p[2]) ** 2)
                stamp = np.exp(-d2 / (2 * rad * rad))
                sl = tuple(slice(lo[k], hi[k]) for k in range(3))
                np.maximum(vessel[sl], stamp, out=vessel[sl])
                d = d + 0.35 * rng.standard_normal(3)
                d /= np.linalg.norm(d)
                p = p + d * max(1.0, 1.5 * rad)
                rad = max(0.6, rad * 0.985)
    inl = lobes[0][2] | lobes[1][2]
    hu = np.where(inl, hu + vessel * (400.0 - hu), hu)
    del vessel, inl
    hu = np.clip(hu, -1000.0, 400.0)
    F0 = (hu - hu.min()) / (hu.max() - hu.min())
    del hu
    F0 = ndi.gaussian_filter(F0, 0.7, mode="nearest")
    coarse = 4 if min(shape) >= 64 else 1
    t = _smooth_field(rng, shape, field_sigma, max_disp, coarse=coarse)
    w = invert_field(t, iters=30, coarse=coarse)
    M0 = _resample(F0, w, order=1)
    del w
    noise = 0.005
    F = F0 + noise * rng.standard_normal(shape)
    M = M0 + noise * rng.standard_normal(shape)
    return Phantom(F.astype(np.float32), M.astype(np.float32),
                   t.astype(np.float32), None,
                   dict(kind="lung", seed=seed, shape=shape))


# ------------------------------------------- abdomen, cross-modal (MR -> CT)
# class intensities of the two modalities, normalised to [0, 1]:
# background, fat, muscle and soft tissue, liver, spleen, kidney, bone
ABDOMEN_CT = (0.0, 0.33, 0.52, 0.57, 0.55, 0.60, 0.92)
ABDOMEN_MR = (0.0, 0.88, 0.30, 0.42, 0.62, 0.72, 0.12)


def abdomen(shape=(192, 160, 192), seed=0, field_sigma=8.0, max_disp=6.0,
            pv_sigma=0.7, noise=0.01, bias=0.15, texture=0.08):
    """Abdomen-like cross-modal pair: one label map (an elliptical trunk with
    a subcutaneous fat shell, liver, spleen, two kidneys and a vertebral
    column, each ellipsoid jittered by the seed) rendered twice with
    different class intensities, plus one smooth tissue texture common to
    both.  The fixed image is the CT-like rendering;
    the moving image is the MR-like rendering (a smooth multiplicative bias
    field as well) warped by the inverse of the true field.  Axis 0 (z) runs
    head to foot, axis 1 (y) front to back, axis 2 (x) right to left."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    nz, ny, nx = shape
    zz, yy, xx = _grid(shape)
    zn, yn, xn = zz / nz - 0.5, yy / ny - 0.5, xx / nx - 0.5
    del zz, yy, xx

    def ell(c, a):
        c = np.asarray(c) + rng.uniform(-0.02, 0.02, 3)
        a = np.asarray(a) * rng.uniform(0.92, 1.08, 3)
        return (((zn - c[0]) / a[0]) ** 2 + ((yn - c[1]) / a[1]) ** 2 +
                ((xn - c[2]) / a[2]) ** 2) <= 1.0

    lab = np.zeros(shape, np.uint8)
    trunk = ((yn / 0.40) ** 2 + (xn / 0.46) ** 2) <= 1.0
    inner = ((yn / 0.34) ** 2 + (xn / 0.40) ** 2) <= 1.0
    lab[trunk] = 1
    lab[inner] = 2
    lab[ell((-0.12, -0.02, -0.18), (0.22, 0.20, 0.20)) & inner] = 3   # liver
    lab[ell((-0.14, 0.08, 0.24), (0.12, 0.09, 0.08)) & inner] = 4    # spleen
    for side in (-1, 1):                                               # kidneys
        lab[ell((0.05, 0.18, side * 0.15), (0.10, 0.05, 0.05)) & inner] = 5
    spine = (((yn - 0.24) / 0.06) ** 2 + (xn / 0.06) ** 2) <= 1.0
    lab[spine & inner] = 6
    del zn, yn, xn, trunk, inner, spine
    coarse = 4 if min(shape) >= 64 else 1
    # tissue texture: one smooth random pattern inside the body, shared by
    # both renderings (it belongs to the anatomy, not to the modality)
    tex = texture * _smooth_field(rng, shape, 2.0, 1.0, coarse=1)[0] * (lab > 0)
    ct = ndi.gaussian_filter(np.array(ABDOMEN_CT)[lab] + tex, pv_sigma, mode="constant")
    mr = ndi.gaussian_filter(np.array(ABDOMEN_MR)[lab] + tex, pv_sigma, mode="constant")
    del tex
    b = _smooth_field(rng, shape, 16.0, 1.0, coarse=coarse)[0]
    mr = mr * (1.0 + bias * b)
    del b
    t = _smooth_field(rng, shape, field_sigma, max_disp, coarse=coarse)
    w = invert_field(t, iters=30, coarse=coarse)
    M0 = _resample(mr, w, order=1)
    del w, mr
    F = ct + noise * rng.standard_normal(shape)
    M = M0 + noise * rng.standard_normal(shape)
    return Phantom(F.astype(np.float32), M.astype(np.float32),
                   t.astype(np.float32), lab,
                   dict(kind="abdomen", seed=seed, shape=shape))


# ------------------------------------------------------- uneven-size batch
BATCH_SHAPES = ((96, 96, 96),) * 4 + ((128, 160, 128),) * 4 + \
               ((160, 192, 224),) * 4 + ((192, 160, 256),) * 4


def batch(seed=0, shapes=BATCH_SHAPES):
    """Brain-style pairs of uneven shapes (16 pairs, 73,007,104 voxels)."""
    return [brain(s, seed=seed * 1000 + i) for i, s in enumerate(shapes)]


def to_bf16_rne(a: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(a)
    if nan.any():
        r[nan] = 0x7FC0
    return r


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint32) << 16).view(np.float32)
