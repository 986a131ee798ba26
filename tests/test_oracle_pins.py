"""Pins of the FP64 oracle against things other than itself.

Each test ties one oracle function (O1..O9) to a library routine (scipy,
numpy, torch on the CPU), a closed form, an invariant the mathematics fixes,
or finite differences, so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage as ndi

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ O1 warp
def test_sample_matches_scipy_grid_constant(orc):
    """Trilinear sampling with zero padding equals scipy's order-1
    map_coordinates in 'grid-constant' mode (padding value 0)."""
    rng = _rng(1)
    V = rng.standard_normal((5, 6, 7))
    pts = rng.uniform(-1.7, 1.0, (400, 3)) * 0 + np.stack(
        [rng.uniform(-1.5, 7.5, 400), rng.uniform(-1.5, 6.5, 400),
         rng.uniform(-1.5, 5.5, 400)], 1)            # (x, y, z)
    ours = np.array([orc.sample(V, p) for p in pts])
    ref = ndi.map_coordinates(V, pts[:, ::-1].T, order=1, mode="grid-constant",
                              cval=0.0)
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-13)


def test_sample_derivative_finite_difference(orc):
    rng = _rng(2)
    V = rng.standard_normal((6, 6, 6))
    h = 1e-6
    for _ in range(50):
        p = rng.uniform(0.2, 4.8, 3)
        p = np.floor(p) + 0.1 + 0.8 * (p - np.floor(p))   # keep off the kinks
        _, d = orc.sample(V, p, with_grad=True)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (orc.sample(V, p + e) - orc.sample(V, p - e)) / (2 * h)
            assert abs(fd - d[c]) < 1e-8


def test_warp_integer_shift_is_exact(orc):
    """u = s (integer) samples M(x + s) bitwise, with zeros outside."""
    rng = _rng(3)
    M = rng.standard_normal((9, 10, 11))
    for s in [(1, 0, 0), (-2, 3, 1), (0, 0, -4), (12, 0, 0)]:
        u = np.zeros((3,) + M.shape)
        for c in range(3):
            u[c] = s[c]
        Mw = orc.warp(M, u)
        ref = np.zeros_like(M)
        sx, sy, sz = s
        nz, ny, nx = M.shape
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    if 0 <= x + sx < nx and 0 <= y + sy < ny and 0 <= z + sz < nz:
                        ref[z, y, x] = M[z + sz, y + sy, x + sx]
        assert np.array_equal(Mw, ref)


def test_warp_constant_image_interior(orc):
    M = np.full((8, 8, 8), 2.5)
    rng = _rng(4)
    u = rng.uniform(-0.9, 0.9, (3, 8, 8, 8))
    Mw = orc.warp(M, u)
    np.testing.assert_allclose(Mw[1:-1, 1:-1, 1:-1], 2.5, atol=1e-14)


# ------------------------------------------------------------------ O2 LNCC
@pytest.mark.parametrize("w", [1, 3, 5, 7])
def test_box_sum_matches_uniform_filter(orc, w):
    a = _rng(5).standard_normal((7, 9, 8))
    ref = ndi.uniform_filter(a, size=w, mode="constant", cval=0.0) * w ** 3
    np.testing.assert_allclose(orc.box_sum(a, w), ref, rtol=1e-12, atol=1e-12)


def test_window_stats_brute_force(orc):
    rng = _rng(6)
    F, M = rng.standard_normal((2, 6, 7, 8))
    x, y, z = 0, 3, 5
    st = orc.window_stats(F, M, 5, x, y, z)
    sl = (slice(max(z - 2, 0), z + 3), slice(max(y - 2, 0), y + 3),
          slice(max(x - 2, 0), x + 3))
    f, m = F[sl], M[sl]
    ref = [f.sum(), m.sum(), (f * f).sum(), (m * m).sum(), (f * m).sum()]
    np.testing.assert_allclose(st, ref, rtol=1e-13)


def test_lncc_identical_images_is_one(orc):
    """cc <= 1 (Cauchy-Schwarz) with equality for identical images, at every
    voxel including the zero-padded border.  With eps > 0 all three window
    moments equal var(F), so cc = var^2 / (var^2 + eps); var is taken from
    scipy's zero-padded uniform filter (divisor w^3 at every centre)."""
    F = _rng(7).standard_normal((10, 11, 12))
    m, cc = orc.lncc(F, F, 5, 0.0, with_map=True)
    assert abs(m - 1.0) < 1e-12
    assert np.all(np.abs(cc - 1.0) < 1e-12)
    eps = 1e-5
    m2, cc2 = orc.lncc(F, F, 5, eps, with_map=True)
    uf = lambda a: ndi.uniform_filter(a, 5, mode="constant", cval=0.0)
    var = uf(F * F) - uf(F) ** 2
    np.testing.assert_allclose(cc2, var ** 2 / (var ** 2 + eps), rtol=1e-10)
    assert m2 < 1.0
    assert 1.0 - m2 < 3e-5 * np.mean(1.0 / var ** 2)


def test_lncc_range_and_symmetry(orc):
    rng = _rng(8)
    F, M = rng.uniform(0, 1, (2, 9, 9, 9))
    m1, c1 = orc.lncc(F, M, 5, 1e-5, with_map=True)
    m2, c2 = orc.lncc(M, F, 5, 1e-5, with_map=True)
    np.testing.assert_allclose(c1, c2, rtol=1e-12, atol=1e-15)
    assert np.all(c1 >= 0) and np.all(c1 <= 1)


def test_lncc_affine_invariance_interior(orc):
    rng = _rng(9)
    F, M = rng.uniform(0, 1, (2, 11, 11, 11))
    _, c1 = orc.lncc(F, M, 5, 0.0, with_map=True)
    _, c2 = orc.lncc(3.0 * F + 7.0, M, 5, 0.0, with_map=True)
    _, c3 = orc.lncc(F, -0.5 * M + 2.0, 5, 0.0, with_map=True)
    i = (slice(2, -2),) * 3
    np.testing.assert_allclose(c2[i], c1[i], rtol=1e-9)
    np.testing.assert_allclose(c3[i], c1[i], rtol=1e-9)


@pytest.mark.parametrize("w", [3, 5, 7])
def test_lncc_closed_form_ramp(orc, w):
    """F = x and M = x^2 (constant along y, z): at an interior centre c the
    window moments are those of k in [-h, h]: var(F) = E k^2,
    cov(F, M) = 2 c E k^2, var(M) = 4 c^2 E k^2 + E k^4 - (E k^2)^2."""
    h = w // 2
    n = 21
    x = np.arange(n, dtype=np.float64) - 10.0
    F = np.broadcast_to(x, (n, n, n)).copy()
    M = F * F
    eps = 1e-5
    _, cc = orc.lncc(F, M, w, eps, with_map=True)
    k = np.arange(-h, h + 1, dtype=np.float64)
    v2, m4 = (k ** 2).mean(), (k ** 4).mean()
    for xi in range(h, n - h):
        c = x[xi]
        sfm, sff, smm = 2 * c * v2, v2, 4 * c * c * v2 + m4 - v2 * v2
        ref = sfm ** 2 / (sff * smm + eps)
        got = cc[10, 10, xi]
        assert abs(got - ref) < 1e-10 * max(1.0, ref), (xi, got, ref)


# ------------------------------------------------------------------ O3 grad
def _smooth_pair(shape, seed):
    rng = _rng(seed)
    F = ndi.gaussian_filter(rng.standard_normal(shape), 1.2)
    M = ndi.gaussian_filter(rng.standard_normal(shape), 1.2)
    return F / F.std(), M / M.std()


@pytest.mark.parametrize("w,eps", [(3, 1e-5), (5, 1e-5), (5, 0.0)])
def test_gradient_matches_finite_differences(orc, w, eps):
    """g_raw = N dL/du against central differences of the FP64 loss, with
    sample points kept 0.3 voxel away from the trilinear kinks."""
    shape = (7, 8, 9)
    F, M = _smooth_pair(shape, 10 + w)
    rng = _rng(11)
    u = 0.3 + 0.4 * rng.uniform(0, 1, (3,) + shape) + rng.integers(-1, 2, (3,) + shape)
    L, g = orc.loss_grad(F, M, u, w, eps)
    N = np.prod(shape)
    h = 1e-5
    worst = 0.0
    for _ in range(40):
        c = rng.integers(0, 3)
        z, y, x = [rng.integers(0, s) for s in shape]
        up, um = u.copy(), u.copy()
        up[c, z, y, x] += h
        um[c, z, y, x] -= h
        fd = (orc.loss_grad(F, M, up, w, eps, False) -
              orc.loss_grad(F, M, um, w, eps, False)) / (2 * h) * N
        err = abs(fd - g[c, z, y, x]) / max(1e-3, abs(g[c, z, y, x]))
        worst = max(worst, err)
    assert worst < 1e-6, worst


def test_gradient_zero_for_identical_images(orc):
    F, _ = _smooth_pair((8, 8, 8), 12)
    u = np.zeros((3, 8, 8, 8))
    L, g = orc.loss_grad(F, F, u, 5, 0.0)
    assert abs(L + 1.0) < 1e-12
    assert np.abs(g).max() < 1e-9


def test_grad_at_agrees_with_full_gradient(orc):
    shape = (9, 10, 11)
    F, M = _smooth_pair(shape, 13)
    u = _rng(14).uniform(-1.5, 1.5, (3,) + shape)
    _, g = orc.loss_grad(F, M, u, 5, 1e-5)
    for (z, y, x) in [(0, 0, 0), (4, 5, 6), (8, 9, 10), (2, 0, 7)]:
        np.testing.assert_allclose(orc.grad_at(F, M, u, 5, 1e-5, x, y, z),
                                   g[:, z, y, x], rtol=1e-10, atol=1e-13)


def test_point_evaluations_agree_with_volume_functions(orc):
    shape = (8, 9, 10)
    F, M = _smooth_pair(shape, 30)
    u = _rng(31).uniform(-1.5, 1.5, (3,) + shape)
    Mw = orc.warp(M, u)
    _, cc = orc.lncc(F, Mw, 5, 1e-5, with_map=True)
    g = _rng(32).standard_normal((3,) + shape)
    gs = orc.gauss(g, 1.0)
    for (z, y, x) in [(0, 0, 0), (3, 4, 5), (7, 8, 9), (0, 8, 2)]:
        assert abs(orc.cc_at(F, M, u, 5, 1e-5, x, y, z) - cc[z, y, x]) < 1e-12
        np.testing.assert_allclose(orc.gauss_at(g, 1.0, x, y, z), gs[:, z, y, x],
                                   rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------ O4 Gaussian
@pytest.mark.parametrize("sigma", [1.0, 0.7, 1.6])
def test_gauss_matches_scipy(orc, sigma):
    g = _rng(15).standard_normal((3, 8, 9, 10))
    R = orc.gauss_radius(sigma)
    assert R == math.ceil(3 * sigma)
    ref = np.stack([ndi.gaussian_filter(g[c], sigma, mode="constant", cval=0.0,
                                        radius=R) for c in range(3)])
    np.testing.assert_allclose(orc.gauss(g, sigma), ref, rtol=1e-12, atol=1e-13)


def test_gauss_keeps_constants_and_ramps_inside(orc):
    z, y, x = np.meshgrid(*[np.arange(12.0)] * 3, indexing="ij")
    g = np.stack([np.full_like(x, 3.0), 2 * x - y, z + 0.5 * x])
    out = orc.gauss(g, 1.0)
    i = (slice(None),) + (slice(3, -3),) * 3
    np.testing.assert_allclose(out[i], g[i], atol=1e-12)


def test_gauss_sigma_zero_is_identity(orc):
    g = _rng(16).standard_normal((3, 4, 5, 6))
    np.testing.assert_array_equal(orc.gauss(g, 0.0), g)


# ------------------------------------------------------------------ O5 update
def test_closed_form_equals_explicit_solve(orc):
    """eq. tile1 equals the solution of (g g^T + lambda I) d = -r g
    (App. A), both by the oracle's own elimination and numpy's LAPACK."""
    rng = _rng(17)
    gs = rng.standard_normal((3, 3, 4, 5)) * 10 ** rng.uniform(-4, 3, (1, 3, 4, 5))
    for lam in [1e-6, 0.006, 1.0, 250.0]:
        r = 0.37
        du = orc.closed_form(gs, r, lam)
        for idx in np.ndindex(3, 4, 5):
            gv = gs[(slice(None),) + idx]
            A = np.outer(gv, gv) + lam * np.eye(3)
            ref = np.linalg.solve(A, -r * gv)
            d2 = orc.explicit_solve(gv, r, lam)
            scale = np.abs(ref).max()
            # solving a system of condition (|g|^2 + lambda)/lambda loses
            # that factor of relative accuracy in the explicit solves
            tol = 1e-14 * scale * ((gv @ gv + lam) / lam) + 1e-300
            assert np.abs(du[(slice(None),) + idx] - ref).max() <= tol
            assert np.abs(d2 - ref).max() <= tol


def test_closed_form_limits_and_bound(orc):
    rng = _rng(18)
    gs = rng.standard_normal((3, 4, 4, 4))
    r = 0.8
    big = 1e10
    np.testing.assert_allclose(orc.closed_form(gs, r, big) * big, -r * gs,
                               rtol=1e-8)
    n2 = (gs ** 2).sum(0)
    np.testing.assert_allclose(orc.closed_form(gs, r, 1e-300), -r * gs / n2,
                               rtol=1e-12)
    for lam in [1e-4, 0.1, 3.0]:
        du = orc.closed_form(gs * 10 ** rng.uniform(-3, 3), r, lam)
        assert np.sqrt((du ** 2).sum(0)).max() <= r / (2 * math.sqrt(lam)) * (1 + 1e-12)
        # parallel to -g
        cos = -(du * gs).sum(0) / np.sqrt((du ** 2).sum(0) * n2)
        np.testing.assert_allclose(cos, 1.0, atol=1e-12)


# ------------------------------------------------------------------ O6 integrate
def test_integrate_additive_and_constant_field(orc):
    rng = _rng(19)
    v = rng.uniform(-0.5, 0.5, (3, 8, 8, 8))
    u = rng.standard_normal((3, 8, 8, 8))
    np.testing.assert_allclose(orc.integrate(u, v, 0.7, 0), u + 0.7 * v,
                               atol=1e-15)
    uc = np.stack([np.full((8, 8, 8), c) for c in (0.3, -1.2, 2.0)])
    out = orc.integrate(uc, v, 1.0, 1)
    i = (slice(None),) + (slice(1, -1),) * 3
    np.testing.assert_allclose(out[i], (uc + v)[i], atol=1e-13)


def test_integrate_matches_scipy_resample(orc):
    """u o (Id + eps v) resampled by scipy (order 1, zero padding)."""
    rng = _rng(20)
    shape = (6, 7, 8)
    u = rng.standard_normal((3,) + shape)
    v = rng.uniform(-1.5, 1.5, (3,) + shape)
    eps = 0.8
    zz, yy, xx = np.meshgrid(*[np.arange(s, dtype=float) for s in shape],
                             indexing="ij")
    cr = np.stack([zz + eps * v[2], yy + eps * v[1], xx + eps * v[0]])
    ref = np.stack([eps * v[c] + ndi.map_coordinates(u[c], cr, order=1,
                                                     mode="grid-constant",
                                                     cval=0.0)
                    for c in range(3)])
    np.testing.assert_allclose(orc.integrate(u, v, eps, 1), ref, atol=1e-12)


# ------------------------------------------------------------------ O7 decide
def test_decision_tables(orc):
    """Hand-built loss sequences (golden file) with the decisions and lambdas
    that eq. lambda-update and eq. rejection fix."""
    with open(os.path.join(GOLD, "decision_tables.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        p = orc.Params(**case["params"])
        st = orc.State(**case["state"])
        for step in case["steps"]:
            acc, st = orc.decide(p, st, step["cand"], step.get("force", -1))
            assert acc == step["accept"], (case["name"], step)
            assert st.lambda_ == pytest.approx(step["lambda"], rel=1e-15), (case["name"], step)
            if "stalled" in step:
                assert st.stalled == step["stalled"], (case["name"], step)


def test_run_monotone_loss_and_lambda_trajectory(orc):
    """With tau = 0 an accepted step never raises the loss; lambda follows
    lambda0 mu+^(#bad) mu-^(#good) exactly (clamps inactive)."""
    from paper_2603_19371_amd import phantoms
    ph = phantoms.blobs((16, 16, 16), seed=3)
    p = orc.Params(window=5)
    pr = orc.Pair(ph.F, ph.M, p).begin(lambda0=1.0)
    L0 = pr.state.loss
    losses = [pr.state.loss]
    n_inc = n_dec = 0
    for _ in range(25):
        before = pr.state.loss
        acc = pr.attempt()
        if acc:
            assert pr.state.loss <= before
            losses.append(pr.state.loss)
            n_dec += pr.state.loss <= before
        else:
            n_inc += 1
        assert pr.state.lambda_ == pytest.approx(2.0 ** n_inc * 0.5 ** n_dec, rel=1e-15)
    assert pr.state.loss < L0
    assert np.all(np.diff(losses) <= 0)


def test_tau_negative_always_accepts(orc):
    from paper_2603_19371_amd import phantoms
    ph = phantoms.blobs((12, 12, 12), seed=4)
    p = orc.Params(window=3, tau=-1.0, lambda_inc=1.5, lambda_dec=0.975,
                   lambda_max=math.inf)
    pr = orc.Pair(ph.F, ph.M, p).begin(lambda0=0.006)
    lam = 0.006
    prev = pr.state.loss
    for _ in range(8):
        assert pr.attempt()
        lam *= 1.5 if pr.state.loss > prev else 0.975
        prev = pr.state.loss
        assert pr.state.lambda_ == pytest.approx(lam, rel=1e-14)


# ------------------------------------------------------------------ O8 pyramid
def test_avgpool_matches_numpy(orc):
    a = _rng(21).standard_normal((8, 12, 16))
    for f in (2, 4):
        ref = a.reshape(8 // f, f, 12 // f, f, 16 // f, f).mean((1, 3, 5))
        np.testing.assert_allclose(orc.avgpool(a, f), ref, rtol=1e-13)


def test_upsample_matches_torch_interpolate(orc):
    torch = pytest.importorskip("torch")
    uc = _rng(22).standard_normal((3, 4, 5, 6))
    ref = torch.nn.functional.interpolate(
        torch.from_numpy(uc)[None], scale_factor=2, mode="trilinear",
        align_corners=False)[0].numpy() * 2.0
    np.testing.assert_allclose(orc.upsample_field(uc, (8, 10, 12)), ref,
                               rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------------ O9 folds
def test_folded_count_matches_numpy_gradient(orc):
    rng = _rng(23)
    u = ndi.gaussian_filter(rng.standard_normal((3, 9, 10, 11)), (0, 1, 1, 1)) * 6
    n, det = orc.folded_count(u, with_det=True)
    # numpy.gradient: central inside, first-order one-sided on the faces
    J = np.empty((3, 3) + u.shape[1:])
    axis_of = {0: 2, 1: 1, 2: 0}          # x, y, z -> array axis
    for c in range(3):
        for d in range(3):
            J[c, d] = np.gradient(u[c], axis=axis_of[d], edge_order=1) + (c == d)
    ref = np.linalg.det(np.moveaxis(J, (0, 1), (-2, -1)))
    np.testing.assert_allclose(det, ref, rtol=1e-10, atol=1e-10)
    assert n == int((ref <= 0).sum())
    assert 0 < n < det.size
    assert orc.folded_count(np.zeros((3, 5, 5, 5))) == 0
    x = np.arange(6.0)
    comp = np.zeros((3, 6, 6, 6))
    comp[0] = -2.0 * x          # x -> -x: det = -1 everywhere
    assert orc.folded_count(comp) == 216
