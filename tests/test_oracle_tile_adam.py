"""Pins of the oracle's pooled-Hessian step (eq. tilen) and of its Adam
comparator, against pieces that do not come from the oracle.

Pooled Hessian (Sec. 2.2, eq. tilen; the tile-size ablation of Sec. 3.2):
* the tile matrices against numpy slices of each k^3 block and a numpy
  product G G^T / count;
* the step against ``numpy.linalg.solve`` of (H_tile + lambda I) d = -r g at
  every voxel;
* k = 1 reduces to eq. tile1, and a gradient constant inside each tile gives
  the rank-1 step of eq. tile1 for every k (H_tile = g g^T there);
* a whole forced attempt with k = 2 against the recomposition of
  tests/test_oracle_attempt.py with the numpy step in place of the rank-1 one.

Adam comparator (the paper's baseline, Sec. 3: beta1 0.9, beta2 0.999):
* the direction against ``torch.optim.Adam`` stepping a float64 parameter
  with the same gradient sequence (the parameter's change is the direction);
* the first step's closed form -lr g / (|g| + eps) (bias correction makes
  mhat = g, vhat = g^2 at t = 1);
* a whole iteration against the recomposition (map_coordinates compositive
  update, the scipy LNCC, finite-difference gradient, scipy Gaussian).
"""
import numpy as np
import pytest

import test_oracle_attempt as toa


def _blocks(shape, k):
    for z0 in range(0, shape[0], k):
        for y0 in range(0, shape[1], k):
            for x0 in range(0, shape[2], k):
                yield (slice(z0, z0 + k), slice(y0, y0 + k), slice(x0, x0 + k))


@pytest.mark.parametrize("k", [2, 3, 4])
def test_tile_hessian_is_the_block_mean_of_rank1_products(orc, k):
    rng = np.random.default_rng(k)
    shape = (7, 9, 10)                       # partial blocks at every far face
    gs = rng.standard_normal((3,) + shape)
    H = orc.tile_hessian(gs, k)
    for b in _blocks(shape, k):
        G = gs[(slice(None),) + b].reshape(3, -1)
        R = G @ G.T / G.shape[1]
        h = H[b[0].start // k, b[1].start // k, b[2].start // k]
        ref = [R[0, 0], R[1, 1], R[2, 2], R[0, 1], R[0, 2], R[1, 2]]
        np.testing.assert_allclose(h, ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("k", [2, 3])
def test_tile_step_is_the_explicit_solve(orc, k):
    rng = np.random.default_rng(10 + k)
    shape = (5, 6, 7)
    gs = rng.standard_normal((3,) + shape)
    r, lam = 0.37, 0.05
    d = orc.tile_step(gs, k, r, lam)
    for b in _blocks(shape, k):
        G = gs[(slice(None),) + b].reshape(3, -1)
        A = G @ G.T / G.shape[1] + lam * np.eye(3)
        ref = np.linalg.solve(A, -r * G)
        np.testing.assert_allclose(d[(slice(None),) + b].reshape(3, -1), ref,
                                   rtol=1e-11, atol=1e-14)


def test_tile_step_special_cases(orc):
    rng = np.random.default_rng(20)
    shape = (6, 6, 8)
    gs = rng.standard_normal((3,) + shape)
    r, lam = 0.8, 0.3
    # k = 1 is eq. tile1
    np.testing.assert_allclose(orc.tile_step(gs, 1, r, lam), orc.closed_form(gs, r, lam),
                               rtol=1e-13, atol=1e-15)
    # a gradient constant on each 2^3 tile: H_tile = g g^T, so eq. tile1 again
    c = rng.standard_normal((3, 3, 3, 4))
    gc = np.repeat(np.repeat(np.repeat(c, 2, 1), 2, 2), 2, 3)
    np.testing.assert_allclose(orc.tile_step(gc, 2, r, lam), -r * gc / (
        (gc * gc).sum(0) + lam), rtol=1e-12, atol=1e-15)
    # lambda -> infinity: gradient descent -r g / lambda
    big = 1e9
    ref = -r * gs / big
    np.testing.assert_allclose(orc.tile_step(gs, 3, r, big), ref, rtol=0,
                               atol=1e-7 * np.abs(ref).max())


def test_tile_attempt_matches_recomposition(orc):
    """A forced-accept attempt with k = 2: candidate field, loss and the
    re-smoothed gradient, with the step solved by numpy on the pooled
    matrices of the smoothed gradient."""
    F, M, u0 = toa._pair()
    p = toa._params(orc, tile=2)
    lam = 1.0
    pr = orc.Pair(F, M, p).begin(u0, lambda0=lam)
    ref = toa.Recomposed(F, M, p, u0, lam)
    r = 1.0 + ref.L
    d = np.empty_like(ref.gs)
    for b in _blocks(F.shape, 2):
        G = ref.gs[(slice(None),) + b]
        Gm = G.reshape(3, -1)
        A = Gm @ Gm.T / Gm.shape[1] + lam * np.eye(3)
        d[(slice(None),) + b] = np.linalg.solve(A, -r * Gm).reshape(G.shape)
    ut = toa._compose(u0, d)
    Lc = float(toa._loss(F, toa._warp(M, ut)))
    assert np.abs(ut - u0).max() > 1e-2
    assert toa._kink_distance(ut) > 1e-3
    # the pooled step differs from the pointwise one on this pair
    assert np.abs(d - toa._damped_step(ref.gs, r, lam)).max() > 1e-2
    assert pr.attempt(force=1)
    np.testing.assert_allclose(pr.u, ut, rtol=0, atol=1e-9)
    assert abs(pr.state.loss - Lc) < 1e-12
    gs_ref = toa._smooth(toa._fd_gradient(F, M, ut))
    np.testing.assert_allclose(pr.gs, gs_ref, rtol=0, atol=1e-7 * np.abs(gs_ref).max())


def test_adam_direction_matches_torch_adam(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(30)
    shape = (3, 4, 5, 6)
    ap = orc.AdamParams(lr=0.2, beta1=0.9, beta2=0.999, eps=1e-8)
    prm = torch.zeros(shape, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([prm], lr=ap.lr, betas=(ap.beta1, ap.beta2), eps=ap.eps)
    m = np.zeros(shape)
    v = np.zeros(shape)
    for t in range(1, 5):
        g = rng.standard_normal(shape) * (0.5 + t)
        before = prm.detach().clone()
        prm.grad = torch.from_numpy(g.copy())
        opt.step()
        delta = (prm.detach() - before).numpy()
        du = orc.adam_direction(g, m, v, t, ap)
        np.testing.assert_allclose(du, delta, rtol=1e-12, atol=1e-15)


def test_adam_first_step_closed_form(orc):
    rng = np.random.default_rng(31)
    g = rng.standard_normal((3, 2, 3, 4))
    ap = orc.AdamParams(lr=0.3)
    du = orc.adam_direction(g, np.zeros_like(g), np.zeros_like(g), 1, ap)
    np.testing.assert_allclose(du, -0.3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_iterations_match_recomposition(orc):
    """Two iterations: the Adam directions of the smoothed gradients (from
    torch.optim.Adam), the compositive update and the new loss and smoothed
    gradient; the moments carry over between iterations."""
    torch = pytest.importorskip("torch")
    F, M, u0 = toa._pair()
    p = toa._params(orc)
    ap = orc.AdamParams(lr=0.05)
    ad = orc.AdamPair(F, M, p, ap).begin(u0)
    ref = toa.Recomposed(F, M, p, u0, 1.0)
    assert abs(ad.state.loss - ref.L) < 1e-12
    prm = torch.zeros(ref.gs.shape, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([prm], lr=ap.lr, betas=(ap.beta1, ap.beta2), eps=ap.eps)
    u, gs = u0.copy(), ref.gs
    for _ in range(2):
        before = prm.detach().clone()
        prm.grad = torch.from_numpy(gs.copy())
        opt.step()
        d = (prm.detach() - before).numpy()
        u = toa._compose(u, d)
        L = float(toa._loss(F, toa._warp(M, u)))
        assert toa._kink_distance(u) > 1e-3
        gs = toa._smooth(toa._fd_gradient(F, M, u))
        got = ad.iterate()
        np.testing.assert_allclose(ad.u, u, rtol=0, atol=1e-9)
        assert abs(got - L) < 1e-12
        np.testing.assert_allclose(ad.gs, gs, rtol=0, atol=1e-7 * np.abs(gs).max())
    assert ad.t == 2 and ad.state.n_hist == 3
