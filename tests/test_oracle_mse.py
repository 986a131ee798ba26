"""Pins of the oracle's squared-error similarity and of its Demons step
(Sec. 2.2: the MSE is already a squared loss; Sec. 2.3, eq. demons), against
pieces that do not come from the oracle.

* The loss against numpy's mean of (F - M o (Id + u))^2, the warp by scipy's
  ``map_coordinates``.
* The gradient N dr/du of the scalar residual r = sqrt(MSE) against
  fourth-order central differences of sqrt(MSE) (sample points away from the
  trilinear kinks), and its closed form at identical images (r = 0: g = 0).
* The Demons step against ``numpy.linalg.solve`` of the damped per-voxel
  Gauss-Newton system (n n^T + lambda I) du = r_x n (the form the paper
  derives eq. demons from by Sherman-Morrison), with n the derivative of the
  trilinear interpolant by central differences of ``map_coordinates``.
* Whole forced attempts of both (LM on the MSE residual; the smoothed Demons
  step) against the recomposition with scipy's Gaussian and the compositive
  update.
"""
import numpy as np
import pytest
from scipy import ndimage as ndi

import test_oracle_attempt as toa


def _mse(F, Mw):
    return ((F - Mw) ** 2).mean(axis=(-3, -2, -1))


def _fd_sqrt_mse_gradient(F, M, u, h=toa.H_FD):
    """N d sqrt(MSE)/du by fourth-order differences (one warped value at a
    time, as the LNCC differences of the attempt pins)."""
    shape = F.shape
    N = int(np.prod(shape))
    assert toa._kink_distance(u) > 4 * h
    Mw = toa._warp(M, u).reshape(N)
    zz, yy, xx = toa._grid(shape)
    base = np.stack([xx + u[0], yy + u[1], zz + u[2]]).reshape(3, N)
    g = np.empty((3, N))
    d0 = F.reshape(N) - Mw
    S = (d0 ** 2).sum()
    for c in range(3):
        vals = []
        for t in (-2 * h, -h, h, 2 * h):
            p = base.copy()
            p[c] += t
            mj = ndi.map_coordinates(M, p[::-1], order=1, mode="grid-constant", cval=0.0)
            # only voxel j's term changes when u_j moves
            Sj = S - d0 ** 2 + (F.reshape(N) - mj) ** 2
            vals.append(np.sqrt(Sj / N))
        a, b, c2, d = vals
        g[c] = N * (a - 8 * b + 8 * c2 - d) / (12 * h)
    return g.reshape((3,) + shape)


def _trilinear_derivative(M, u, h=1e-5):
    zz, yy, xx = toa._grid(M.shape)
    base = np.stack([zz + u[2], yy + u[1], xx + u[0]])
    out = []
    for axis in (2, 1, 0):       # x, y, z components
        p, q = base.copy(), base.copy()
        p[axis] += h
        q[axis] -= h
        out.append((ndi.map_coordinates(M, p, order=1, mode="grid-constant", cval=0.0) -
                    ndi.map_coordinates(M, q, order=1, mode="grid-constant", cval=0.0)) /
                   (2 * h))
    return np.stack(out)


def test_mse_loss_and_gradient(orc):
    F, M, u0 = toa._pair()
    L, g = orc.mse_loss_grad(F, M, u0)
    assert abs(L - _mse(F, toa._warp(M, u0))) < 1e-14
    ref = _fd_sqrt_mse_gradient(F, M, u0)
    scale = np.abs(ref).max()
    assert scale > 1e-2
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-7 * scale)


def test_mse_identical_images_give_zero(orc):
    F, _, _ = toa._pair()
    L, g = orc.mse_loss_grad(F, F, np.zeros((3,) + F.shape))
    assert L == 0.0 and not np.any(g)


def test_demons_step_is_the_damped_gauss_newton_solve(orc):
    F, M, u0 = toa._pair()
    lam = 0.3
    du = orc.demons_step(F, M, u0, lam)
    r = F - toa._warp(M, u0)
    n = _trilinear_derivative(M, u0)
    nv = np.moveaxis(n, 0, -1).reshape(-1, 3)
    A = nv[:, :, None] * nv[:, None, :] + lam * np.eye(3)[None]
    ref = np.linalg.solve(A, (r.reshape(-1)[:, None] * nv)[:, :, None])[:, :, 0]
    ref = np.moveaxis(ref.reshape(F.shape + (3,)), -1, 0)
    np.testing.assert_allclose(du, ref, rtol=0, atol=1e-8 * np.abs(ref).max())


def test_mse_attempt_matches_recomposition(orc):
    """LM on the squared error: r = sqrt(MSE) of the accepted field, the
    smoothed N dr/du, the per-voxel solve, the compositive update; the
    candidate's loss is its MSE."""
    F, M, u0 = toa._pair()
    p = toa._params(orc, similarity=1)
    lam = 1.0
    pr = orc.Pair(F, M, p).begin(u0, lambda0=lam)
    L0 = _mse(F, toa._warp(M, u0))
    assert abs(pr.state.loss - L0) < 1e-14
    gs = toa._smooth(_fd_sqrt_mse_gradient(F, M, u0))
    np.testing.assert_allclose(pr.gs, gs, rtol=0, atol=1e-7 * np.abs(gs).max())
    d = toa._damped_step(gs, np.sqrt(L0), lam)
    ut = toa._compose(u0, d)
    assert np.abs(ut - u0).max() > 1e-2
    assert pr.attempt(force=1)
    np.testing.assert_allclose(pr.u, ut, rtol=0, atol=1e-9)
    assert abs(pr.state.loss - _mse(F, toa._warp(M, ut))) < 1e-10


def test_demons_attempt_matches_recomposition(orc):
    """The Demons step of the accepted field (per-voxel residual, global
    lambda), smoothed, integrated compositively; the candidate's MSE."""
    F, M, u0 = toa._pair()
    p = toa._params(orc, similarity=2)
    lam = 0.5
    pr = orc.Pair(F, M, p).begin(u0, lambda0=lam)
    r = F - toa._warp(M, u0)
    n = _trilinear_derivative(M, u0)
    du = r[None] * n / ((n * n).sum(0) + lam)[None]
    v = toa._smooth(du)
    ut = toa._compose(u0, v)
    assert np.abs(ut - u0).max() > 1e-2
    assert pr.attempt(force=1)
    np.testing.assert_allclose(pr.u, ut, rtol=0, atol=1e-8)
    assert abs(pr.state.loss - _mse(F, toa._warp(M, ut))) < 1e-12
