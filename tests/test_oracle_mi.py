"""Pins of the oracle's mutual-information similarity (Sec. 2.2: minimise
(log2 B - MI)^2), against pieces that do not come from the oracle.

* The Parzen window is scipy's cubic B-spline basis element; the joint
  histogram a numpy product W_F^T W_M / N of the per-voxel window weights,
  MI = sum p log2(p / (p_F p_M)) by numpy.
* The gradient N dr/du (r = log2 B - MI) against fourth-order central
  differences of that numpy MI, one warped value at a time, with every
  sample point away from the trilinear kinks.
* Invariances: MI does not change when F is mapped affinely or M scaled by a
  positive factor (the bin coordinates are the same), and never exceeds
  log2 B.
* A whole forced attempt against the recomposition (residual log2 B - MI,
  scipy Gaussian, per-voxel solve, compositive update).
"""
import numpy as np
import pytest
from scipy import interpolate

import test_oracle_attempt as toa

B = 16
_BETA = interpolate.BSpline.basis_element([0.0, 1.0, 2.0, 3.0, 4.0], extrapolate=False)


def beta(t):
    v = _BETA(np.asarray(t, dtype=np.float64) + 2.0)
    return np.nan_to_num(v, nan=0.0)


def _coords(v, lo, hi, bins=B):
    return 1.0 + (bins - 3) * (v - lo) / (hi - lo)


def _ranges(F, M):
    return (F.min(), F.max(), min(M.min(), 0.0), max(M.max(), 0.0))


def _weights(vh, bins=B):
    return beta(vh[..., None] - np.arange(bins))          # (..., bins)


def _mi(F, Mw, rng_, bins=B):
    """MI in bits; Mw may carry leading batch axes."""
    flo, fhi, mlo, mhi = rng_
    WF = _weights(_coords(F.reshape(-1), flo, fhi, bins), bins)          # (N, B)
    WM = _weights(_coords(Mw.reshape(Mw.shape[:-3] + (-1,)), mlo, mhi, bins), bins)
    N = WF.shape[0]
    p = np.einsum("na,...nb->...ab", WF, WM) / N
    pa = p.sum(-1, keepdims=True)
    pb = p.sum(-2, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(p > 0, p * np.log2(p / (pa * pb)), 0.0)
    return t.sum((-2, -1)), p


def test_bspline_window_matches_scipy(orc):
    for t in np.linspace(-2.5, 2.5, 41):
        assert abs(orc.bspline3(t) - beta(t)) < 1e-15
        h = 1e-6
        fd = (beta(t + h) - beta(t - h)) / (2 * h)
        assert abs(orc.dbspline3(t) - fd) < 1e-6


def test_histogram_and_mi_match_numpy(orc):
    F, M, u0 = toa._pair()
    L, g, h = orc.mi_loss_grad(F, M, u0, bins=B, with_hist=True)
    mi, p = _mi(F, toa._warp(M, u0), _ranges(F, M))
    np.testing.assert_allclose(h, p, rtol=0, atol=1e-15)
    assert abs(-L - mi) < 1e-12
    assert 0.0 < mi <= np.log2(B)


def test_mi_invariances(orc):
    F, M, u0 = toa._pair()
    L0 = orc.mi_loss_grad(F, M, u0, bins=B, with_grad=False)
    L1 = orc.mi_loss_grad(3.0 * F - 1.5, M, u0, bins=B, with_grad=False)
    L2 = orc.mi_loss_grad(F, 2.5 * M, u0, bins=B, with_grad=False)
    assert abs(L0 - L1) < 1e-12 and abs(L0 - L2) < 1e-12


def _fd_mi_gradient(F, M, u, h=toa.H_FD):
    """N d(log2 B - MI)/du by fourth-order differences of the numpy MI."""
    shape = F.shape
    N = int(np.prod(shape))
    assert toa._kink_distance(u) > 4 * h
    rng_ = _ranges(F, M)
    Mw = toa._warp(M, u).reshape(N)
    zz, yy, xx = toa._grid(shape)
    base = np.stack([xx + u[0], yy + u[1], zz + u[2]]).reshape(3, N)
    flat = np.arange(N)
    g = np.empty((3, N))
    from scipy import ndimage as ndi
    for c in range(3):
        vals = []
        for t in (-2 * h, -h, h, 2 * h):
            p = base.copy()
            p[c] += t
            mj = ndi.map_coordinates(M, p[::-1], order=1, mode="grid-constant", cval=0.0)
            batch = np.broadcast_to(Mw, (N, N)).copy()
            batch[flat, flat] = mj
            vals.append(-_mi(F, batch.reshape((N,) + shape), rng_)[0])
        a, b, c2, d = vals
        g[c] = N * (a - 8 * b + 8 * c2 - d) / (12 * h)
    return g.reshape((3,) + shape)


def test_mi_gradient_matches_finite_differences(orc):
    F, M, u0 = toa._pair()
    _, g = orc.mi_loss_grad(F, M, u0, bins=B)
    ref = _fd_mi_gradient(F, M, u0)
    scale = np.abs(ref).max()
    assert scale > 1e-2
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-6 * scale)


def test_mi_attempt_matches_recomposition(orc):
    F, M, u0 = toa._pair()
    p = toa._params(orc, similarity=3, mi_bins=B)
    lam = 1.0
    pr = orc.Pair(F, M, p).begin(u0, lambda0=lam)
    mi0, _ = _mi(F, toa._warp(M, u0), _ranges(F, M))
    assert abs(pr.state.loss + mi0) < 1e-12
    gs = toa._smooth(_fd_mi_gradient(F, M, u0))
    np.testing.assert_allclose(pr.gs, gs, rtol=0, atol=1e-6 * np.abs(gs).max())
    d = toa._damped_step(gs, np.log2(B) - mi0, lam)
    ut = toa._compose(u0, d)
    assert np.abs(ut - u0).max() > 1e-2
    assert pr.attempt(force=1)
    np.testing.assert_allclose(pr.u, ut, rtol=0, atol=1e-8)
    mi1, _ = _mi(F, toa._warp(M, ut), _ranges(F, M))
    assert abs(pr.state.loss + mi1) < 1e-9
