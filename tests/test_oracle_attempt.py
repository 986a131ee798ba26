"""Pins of the oracle's composition functions: begin, one attempt, register.

The attempt is rebuilt here from pieces that do not come from the oracle:

* the warp M(x + u) by scipy's ``map_coordinates`` (order 1, zero padding);
* the loss L = -mean cc by an LNCC written with scipy's ``uniform_filter``
  (zero padding, divisor w^3), the squared windowed correlation;
* the raw gradient g = N dL/du by fourth-order central differences of that
  loss, one coordinate at a time, with every sample point kept away from the
  trilinear kinks so that the differences are exact up to O(h^4);
* the smoothed gradient by scipy's ``gaussian_filter`` (zero padding,
  radius ceil(3 sigma));
* the residual r = 1 - LNCC of the accepted field (Sec. 2.2: LNCC enters
  the least-squares form as (1 - LNCC)^2);
* the damped step by ``numpy.linalg.solve`` of (g g^T + lambda I) d = -r g
  per voxel (App. A, eq. lm-local), not by the closed form of eq. tile1;
* the compositive update u~ = eps d + u o (Id + eps d) by ``map_coordinates``
  (Sec. 2.1, eq. compositive);
* the damping rule and the rejection test (eq. lambda-update, eq. rejection)
  restated from the paper with the readings the oracle takes;
* the pyramid hand-off by numpy reshape-means and torch's trilinear
  ``interpolate`` (values doubled), with lambda and the loss history
  restarted at every level.

A dropped or swapped term anywhere in the oracle's composition (r = -L in
place of 1 + L, the raw instead of the smoothed gradient after an accept, a
lambda carried across pyramid levels) changes the field or the state by far
more than the tolerances here.
"""
import math

import numpy as np
import pytest
from scipy import ndimage as ndi

SHAPE = (7, 8, 9)
W, SIGMA, EPS_CC = 3, 1.0, 1e-5
H_FD = 1e-4


def _grid(shape):
    return np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape],
                       indexing="ij")                      # z, y, x


def _warp(M, u):
    zz, yy, xx = _grid(M.shape)
    cr = np.stack([zz + u[2], yy + u[1], xx + u[0]])
    return ndi.map_coordinates(M, cr, order=1, mode="grid-constant", cval=0.0)


def _loss(F, Mw, w=W, eps=EPS_CC):
    """-mean of the windowed squared correlation; Mw may carry leading batch
    axes."""
    size = (1,) * (Mw.ndim - 3) + (w, w, w)
    uf = lambda a: ndi.uniform_filter(a, size=size, mode="constant", cval=0.0)
    Fb = np.broadcast_to(F, Mw.shape).copy()
    mf, mm = uf(Fb), uf(Mw)
    sfm = uf(Fb * Mw) - mf * mm
    sff = uf(Fb * Fb) - mf * mf
    smm = uf(Mw * Mw) - mm * mm
    cc = sfm * sfm / (sff * smm + eps)
    return -cc.mean(axis=(-3, -2, -1))


def _kink_distance(u):
    """Smallest distance of any sample coordinate x + u from an integer."""
    zz, yy, xx = _grid(u.shape[1:])
    p = np.stack([xx + u[0], yy + u[1], zz + u[2]])
    fr = p - np.floor(p)
    return float(np.minimum(fr, 1.0 - fr).min())


def _fd_gradient(F, M, u, h=H_FD):
    """g = N dL/du by fourth-order central differences.  Moving u_j along
    axis c changes only the warped value at j, so each difference re-evaluates
    the whole loss with that one value re-sampled."""
    shape = F.shape
    N = int(np.prod(shape))
    assert _kink_distance(u) > 4 * h
    Mw = _warp(M, u)
    zz, yy, xx = _grid(shape)
    base = np.stack([xx + u[0], yy + u[1], zz + u[2]]).reshape(3, N)   # x,y,z
    g = np.empty((3, N))
    flat = np.arange(N)
    for c in range(3):
        vals = []
        for t in (-2 * h, -h, h, 2 * h):
            p = base.copy()
            p[c] += t
            mj = ndi.map_coordinates(M, p[::-1], order=1, mode="grid-constant",
                                     cval=0.0)                          # (N,)
            batch = np.broadcast_to(Mw.reshape(N), (N, N)).copy()
            batch[flat, flat] = mj
            vals.append(_loss(F, batch.reshape((N,) + shape)))
        Lm2, Lm1, Lp1, Lp2 = vals
        g[c] = N * (Lm2 - 8 * Lm1 + 8 * Lp1 - Lp2) / (12 * h)
    return g.reshape((3,) + shape)


def _smooth(g, sigma=SIGMA):
    R = math.ceil(3 * sigma)
    return np.stack([ndi.gaussian_filter(g[c], sigma, mode="constant", cval=0.0,
                                         radius=R) for c in range(3)])


def _damped_step(gs, r, lam):
    """Per voxel, solve (g g^T + lambda I) d = -r g with LAPACK."""
    g = np.moveaxis(gs, 0, -1).reshape(-1, 3)
    A = g[:, :, None] * g[:, None, :] + lam * np.eye(3)[None]
    d = np.linalg.solve(A, (-r * g)[:, :, None])[:, :, 0]
    return np.moveaxis(d.reshape(gs.shape[1:] + (3,)), -1, 0)


def _compose(u, d, eps=1.0):
    zz, yy, xx = _grid(u.shape[1:])
    cr = np.stack([zz + eps * d[2], yy + eps * d[1], xx + eps * d[0]])
    return np.stack([eps * d[c] + ndi.map_coordinates(
        u[c], cr, order=1, mode="grid-constant", cval=0.0) for c in range(3)])


class Recomposed:
    """One pair advanced attempt by attempt from the pieces above."""

    def __init__(self, F, M, p, u0, lambda0):
        self.F, self.M, self.p = F, M, p
        self.u = u0.copy()
        self.L = float(_loss(F, _warp(M, self.u)))
        self.L_prev = self.L
        self.n_hist = 1
        self.lam = lambda0
        self.gs = _smooth(_fd_gradient(F, M, self.u))

    def candidate(self):
        r = 1.0 - (-self.L)                       # 1 - LNCC of the accepted field
        d = _damped_step(self.gs, r, self.lam)
        ut = _compose(self.u, d, self.p.step_eps)
        return ut, float(_loss(self.F, _warp(self.M, ut)))

    def attempt(self, force=-1):
        p = self.p
        ut, Lc = self.candidate()
        if force >= 0:
            acc = bool(force)
        elif not math.isfinite(Lc):
            acc = False
        else:
            ref = abs(self.L - self.L_prev) if self.n_hist >= 2 else 0.0
            acc = not (Lc - self.L > p.tau * ref)
        clamp = lambda v: min(max(v, p.lambda_min), p.lambda_max)
        if acc:
            self.lam = clamp((p.lambda_inc if Lc > self.L else p.lambda_dec) * self.lam)
            self.L_prev, self.L = self.L, Lc
            self.n_hist += 1
            self.u = ut
            self.gs = _smooth(_fd_gradient(self.F, self.M, ut))
        else:
            self.lam = clamp(p.lambda_inc * self.lam)
        return acc, ut, Lc


def _pair(seed=40):
    """A smooth image and a copy of it displaced by about a voxel, plus a
    starting field whose sample points all sit between 0.25 and 0.55 of a
    cell (far from the trilinear kinks)."""
    rng = np.random.default_rng(seed)
    big = ndi.gaussian_filter(rng.standard_normal((11, 12, 13)), 1.3)
    F = big[2:9, 2:10, 2:11].copy()
    M = big[1:8, 3:11, 2:11].copy() + 0.05 * rng.standard_normal(SHAPE)
    F, M = F / F.std(), M / M.std()
    u0 = 0.4 + 0.15 * np.tanh(ndi.gaussian_filter(rng.standard_normal((3,) + SHAPE),
                                                  (0, 1, 1, 1)))
    return F, M, u0


def _params(orc, **kw):
    return orc.Params(window=W, grad_sigma=SIGMA, cc_eps=EPS_CC, **kw)


def test_fd_gradient_converges():
    """The differencing itself: at two step sizes the fourth-order
    differences agree far below the tolerances used on the oracle, and the
    gradient is not trivially small."""
    F, M, u0 = _pair()
    assert _kink_distance(u0) > 0.2
    g1 = _fd_gradient(F, M, u0, 1e-4)
    g2 = _fd_gradient(F, M, u0, 2e-4)
    scale = np.abs(g1).max()
    assert scale > 1e-2
    assert np.abs(g1 - g2).max() < 1e-9 * scale


def test_begin_matches_recomposition(orc):
    """orc_begin: L(u0) and the smoothed gradient of u0 (the state an attempt
    starts from)."""
    F, M, u0 = _pair()
    pr = orc.Pair(F, M, _params(orc)).begin(u0, lambda0=2.0)
    ref = Recomposed(F, M, _params(orc), u0, 2.0)
    assert abs(pr.state.loss - ref.L) < 1e-12
    scale = np.abs(ref.gs).max()
    assert scale > 1e-2
    np.testing.assert_allclose(pr.gs, ref.gs, rtol=0, atol=1e-8 * scale)
    assert pr.state.lambda_ == 2.0 and pr.state.n_hist == 1
    assert pr.state.retries == 0 and pr.state.stalled == 0


def test_forced_accept_matches_recomposition(orc):
    """One forced-accept attempt: the candidate field, its loss, lambda and
    the smoothed gradient stored for the next attempt."""
    F, M, u0 = _pair()
    p = _params(orc)
    pr = orc.Pair(F, M, p).begin(u0, lambda0=2.0)
    ref = Recomposed(F, M, p, u0, 2.0)
    L0 = ref.L
    acc, ut, Lc = ref.attempt(force=1)
    assert acc
    step = np.abs(ut - u0).max()
    assert step > 1e-2                           # the attempt moves the field
    assert _kink_distance(ut) > 1e-3             # the FD gradient at u~ is valid
    assert pr.attempt(force=1)
    np.testing.assert_allclose(pr.u, ut, rtol=0, atol=1e-9)
    assert abs(pr.state.loss - Lc) < 1e-12
    assert abs(pr.state.loss_prev - L0) < 1e-12
    assert pr.state.lambda_ == pytest.approx(ref.lam, rel=1e-15)
    scale = np.abs(ref.gs).max()
    np.testing.assert_allclose(pr.gs, ref.gs, rtol=0, atol=1e-7 * scale)


def test_forced_reject_keeps_field_and_gradient(orc):
    """A rejected candidate leaves u and the smoothed gradient bit for bit,
    raises lambda by mu+, and still reports the candidate's loss."""
    F, M, u0 = _pair()
    p = _params(orc)
    pr = orc.Pair(F, M, p).begin(u0, lambda0=2.0)
    u_before, gs_before = pr.u.copy(), pr.gs.copy()
    L_before = pr.state.loss
    ref = Recomposed(F, M, p, u0, 2.0)
    _, Lc = ref.candidate()
    assert not pr.attempt(force=0)
    assert np.array_equal(pr.u, u_before)
    assert np.array_equal(pr.gs, gs_before)
    assert pr.state.loss == L_before
    assert pr.state.lambda_ == 4.0 and pr.state.retries == 1
    assert abs(pr.state.cand_loss - Lc) < 1e-12
    # the next attempt starts from the same u with the larger lambda
    ref.lam = 4.0
    ut, Lc2 = ref.candidate()
    assert pr.attempt(force=1)
    np.testing.assert_allclose(pr.u, ut, rtol=0, atol=1e-9)
    assert abs(pr.state.loss - Lc2) < 1e-12


def test_automatic_attempts_match_recomposition(orc):
    """Several attempts with the oracle's own decisions (tau = 0, x2 / x0.5):
    the same accept flags, lambdas and fields as the recomposition."""
    F, M, u0 = _pair(41)
    p = _params(orc)
    pr = orc.Pair(F, M, p).begin(u0, lambda0=0.5)
    ref = Recomposed(F, M, p, u0, 0.5)
    seen = set()
    for _ in range(4):
        acc_ref, ut, Lc = ref.attempt()
        seen.add(acc_ref)
        assert pr.attempt() == acc_ref
        assert abs(pr.state.cand_loss - Lc) < 1e-12
        assert pr.state.lambda_ == pytest.approx(ref.lam, rel=1e-15)
        np.testing.assert_allclose(pr.u, ref.u, rtol=0, atol=1e-8)
        if _kink_distance(ref.u) < 1e-3:
            break
    assert True in seen


def test_register_matches_recomposition(orc):
    """Coarse-to-fine: each level pools the images by reshape-means, starts
    from the previous level's field upsampled by torch's trilinear interpolate
    with values doubled (the coarsest from zero), and restarts lambda and the
    loss history; forced decisions make the two runs comparable."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(42)
    shape = (8, 8, 12)
    big = ndi.gaussian_filter(rng.standard_normal((12, 12, 16)), 1.5)
    F = big[2:10, 2:10, 2:14].copy()
    M = big[1:9, 3:11, 2:14].copy()
    F, M = F / F.std(), M / M.std()
    p = orc.Params(window=3, grad_sigma=1.0)
    levels = [(2, 3), (1, 2)]
    forces = [[1, 0, 1], [1, 1]]
    u, dec = orc.register(F, M, p, levels, lambda0=1.5, forces=forces)
    assert dec == [[True, False, True], [True, True]]

    def pool(a, f):
        z, y, x = a.shape
        return a.reshape(z // f, f, y // f, f, x // f, f).mean((1, 3, 5))

    Fc, Mc = pool(F, 2), pool(M, 2)
    c = orc.Pair(Fc, Mc, p).begin(np.zeros((3,) + Fc.shape), 1.5)
    for f in forces[0]:
        c.attempt(f)
    up = torch.nn.functional.interpolate(torch.from_numpy(c.u)[None], scale_factor=2,
                                         mode="trilinear", align_corners=False)[0]
    u1 = up.numpy() * 2.0
    fine = orc.Pair(F, M, p).begin(u1, 1.5)
    assert fine.state.lambda_ == 1.5 and fine.state.n_hist == 1
    for f in forces[1]:
        fine.attempt(f)
    np.testing.assert_allclose(u, fine.u, rtol=0, atol=1e-12)
    # a run that kept the coarse level's lambda would differ
    carried = orc.Pair(F, M, p).begin(u1, c.state.lambda_)
    for f in forces[1]:
        carried.attempt(f)
    assert np.abs(carried.u - u).max() > 1e-6
