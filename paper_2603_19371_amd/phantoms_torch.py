"""Seeded brain-like pairs generated with torch on the device.

The same recipe as ``phantoms.brain`` (tissue classes as the argmax regions of
smoothed noise inside an ellipsoidal head, piecewise-constant intensities,
partial-volume blur, additive noise; the moving image is the fixed one under
the inverse of a smoothed random field found by fixed-point iteration), built
from torch's device random stream so that thousands of full-size pairs can be
made in seconds (the training set of the learned initializer).  A given seed
gives the same pair on a given device type; the stream differs from numpy's,
so ``phantoms.brain(seed)`` and ``brain(seed)`` here are different pairs of
the same kind.

This module holds no arithmetic of the registration method: it only makes
input data (resampling here is torch's ``grid_sample`` / ``interpolate``).
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as TF

BRAIN_LEVELS = (0.15, 0.30, 0.45, 0.60, 0.75, 0.90)


def _gauss_taps(sigma: float, device):
    R = max(1, int(math.ceil(3.0 * sigma)))
    k = torch.arange(-R, R + 1, dtype=torch.float32, device=device)
    w = torch.exp(-k * k / (2.0 * sigma * sigma))
    return w / w.sum(), R


def _smooth(v: torch.Tensor, sigma: float, edge: bool) -> torch.Tensor:
    """Separable Gaussian of every channel of v [C][Z][Y][X]; edge: the border
    value is extended, else zeros."""
    w, R = _gauss_taps(sigma, v.device)
    x = v[:, None]
    for axis in range(3):
        shape = [1, 1, 1, 1, 1]
        shape[2 + axis] = 2 * R + 1
        pad = [0, 0, 0, 0, 0, 0]
        pad[2 * (2 - axis)] = pad[2 * (2 - axis) + 1] = R
        x = TF.pad(x, pad, mode="replicate" if edge else "constant")
        x = TF.conv3d(x, w.view(shape))
    return x[:, 0]


def _upsample(v: torch.Tensor, shape) -> torch.Tensor:
    return TF.interpolate(v[None], size=tuple(shape), mode="trilinear",
                          align_corners=False)[0]


def _sample(v: torch.Tensor, disp: torch.Tensor) -> torch.Tensor:
    """v [C][Z][Y][X] at x + disp(x) (disp [3][Z][Y][X], x/y/z components,
    voxel units), trilinear, clamped at the border."""
    Z, Y, X = v.shape[1:]
    dev = v.device
    zz, yy, xx = torch.meshgrid(torch.arange(Z, device=dev, dtype=torch.float32),
                                torch.arange(Y, device=dev, dtype=torch.float32),
                                torch.arange(X, device=dev, dtype=torch.float32),
                                indexing="ij")
    gx = (xx + disp[0]) * (2.0 / max(X - 1, 1)) - 1.0
    gy = (yy + disp[1]) * (2.0 / max(Y - 1, 1)) - 1.0
    gz = (zz + disp[2]) * (2.0 / max(Z - 1, 1)) - 1.0
    grid = torch.stack([gx, gy, gz], dim=-1)[None]
    return TF.grid_sample(v[None], grid, mode="bilinear", padding_mode="border",
                          align_corners=True)[0]


def _random_field(g, cshape, shape, sigma, max_disp, coarse):
    dev = g.device
    t = torch.randn((3,) + tuple(cshape), generator=g, device=dev)
    t = _smooth(t, sigma / coarse, edge=True)
    t = _upsample(t, shape) if coarse > 1 else t
    return t * (max_disp / t.square().sum(0).sqrt().max())


def _invert(t: torch.Tensor, iters: int, coarse: int) -> torch.Tensor:
    """w with (Id + t) o (Id + w) = Id by w <- -t(Id + w), on a grid coarsened
    by ``coarse`` (values scaled accordingly) and upsampled back."""
    shape = t.shape[1:]
    tc = TF.avg_pool3d(t[None], coarse)[0] / coarse if coarse > 1 else t
    w = torch.zeros_like(tc)
    for _ in range(iters):
        w = -_sample(tc, w)
    return _upsample(w, shape) * coarse if coarse > 1 else w


@torch.no_grad()
def brain(shape=(160, 192, 224), seed=0, device="cuda", n_classes=6, class_sigma=8.0,
          pv_sigma=0.7, noise=0.01, field_sigma=8.0, max_disp=6.0):
    """Returns (F, M, t): float32 device tensors [Z][Y][X], [Z][Y][X] and the
    true field [3][Z][Y][X]."""
    shape = tuple(int(s) for s in shape)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    coarse = 4 if min(shape) >= 64 else 1
    cshape = tuple(max(2, s // coarse) for s in shape)
    f = torch.randn((n_classes,) + cshape, generator=g, device=device)
    f = _smooth(f, class_sigma / coarse, edge=True)
    if coarse > 1:
        f = _upsample(f, shape)
    lab = f.argmax(0) + 1
    del f
    dev = lab.device
    axes = [torch.arange(s, device=dev, dtype=torch.float32) for s in shape]
    zz, yy, xx = torch.meshgrid(*axes, indexing="ij")
    ctr = [(s - 1) / 2 for s in shape]
    ax = [0.42 * s for s in shape]
    inside = (((zz - ctr[0]) / ax[0]) ** 2 + ((yy - ctr[1]) / ax[1]) ** 2 +
              ((xx - ctr[2]) / ax[2]) ** 2) <= 1.0
    del zz, yy, xx
    lab = torch.where(inside, lab, torch.zeros_like(lab))
    table = torch.tensor((0.0,) + BRAIN_LEVELS[:n_classes], device=dev)
    F0 = _smooth(table[lab][None], pv_sigma, edge=False)
    t = _random_field(g, cshape, shape, field_sigma, max_disp, coarse)
    w = _invert(t, 30, coarse)
    M0 = _sample(F0, w)[0]
    F0 = F0[0]
    F = F0 + noise * torch.randn(shape, generator=g, device=device)
    M = M0 + noise * torch.randn(shape, generator=g, device=device)
    return F.contiguous(), M.contiguous(), t.contiguous()
