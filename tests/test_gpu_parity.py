"""GPU parity: liblmreg (through its C-ABI) against the FP64 oracle.

Every input comes from the seeded generators; every expected value comes from
the oracle on the same bytes.  Sizes span several 32x8 tiles and z-chunks with
ragged tails; the full-size cases use the 160x192x224 brain-phantom shape in
the launch configuration the benchmark times and are checked on sampled
voxels.

Tolerances (float32 kernels against the FP64 oracle):
  * warp / derivative: the trilinear weights and the 8-corner sums are FP32:
    a few ulp of max|M|  -> 4e-6 * max|M|.
  * LNCC map and loss: box sums are exact (FP32 products summed in FP64); the
    only difference is the FP32 rounding of the warped image -> cc within
    2e-6, loss within 2e-7.
  * raw gradient: the adjoint maps are stored in FP32 and the bracket
    F B(alpha) - B(alpha mu_F) + ... cancels about two digits -> 2e-5 of
    max|g|.
  * field after one attempt, and after every attempt of the oracle's own
    50-attempt config-1 trajectory restarted from the oracle's FP32-rounded
    state: 1e-4 voxel (FP32 images, and BF16 images against the oracle on the
    same BF16 values); 5e-3 voxel for BF16 images against the FP32-image
    oracle on the first attempt.  Whole free-running trajectories are not
    compared field by field: the trilinear derivative jumps at cell
    boundaries, so any two FP32/FP64 runs part ways after ~20 attempts (the
    oracle against its own FP32-rounded copy does too).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2603_19371_amd import _lib
    _lib.lib()
    return _lib


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(
        "cuda").to(dtype).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def smooth_pair(shape, seed):
    from scipy import ndimage as ndi
    rng = np.random.default_rng(seed)
    F = ndi.gaussian_filter(rng.standard_normal(shape), 1.0)
    M = ndi.gaussian_filter(rng.standard_normal(shape), 1.0)
    return (F / F.std()).astype(np.float32), (M / M.std()).astype(np.float32)


def report(name, got, ref):
    err = np.abs(got - ref)
    print(f"[{name}] max|err|={err.max():.3e} max|ref|={np.abs(ref).max():.3e}",
          flush=True)
    return err.max()


RAGGED = (20, 37, 70)


# ------------------------------------------------------------------ warp
@pytest.mark.parametrize("img", ["f32", "bf16"])
def test_warp_matches_oracle(L, orc, img):
    from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne
    rng = np.random.default_rng(1)
    F, M = smooth_pair(RAGGED, 2)
    u = rng.uniform(-3, 3, (3,) + RAGGED).astype(np.float32)
    u[:, ::3] = np.round(u[:, ::3])          # integer displacements too
    Mh = bf16_to_f32(to_bf16_rne(M)) if img == "bf16" else M
    Md = dev(Mh, torch.bfloat16 if img == "bf16" else torch.float32)
    Mw, dMw = L.warp(Md, dev(u), with_grad=True)
    rMw, rdMw = orc.warp(Mh, u, with_grad=True)
    s = np.abs(Mh).max()
    e = report("warp", host(Mw), rMw)
    assert e < 4e-6 * s, e
    e = report("dwarp", host(dMw), rdMw)
    assert e < 8e-6 * s, e


def test_warp_integer_shift_is_exact(L):
    F, M = smooth_pair(RAGGED, 3)
    for s in [(2, -1, 3), (-5, 0, 0)]:
        u = np.zeros((3,) + RAGGED, np.float32)
        for c in range(3):
            u[c] = s[c]
        Mw = host(L.warp(dev(M), dev(u)))
        ref = np.zeros_like(M)
        nz, ny, nx = M.shape
        sx, sy, sz = s
        ref[max(0, -sz):nz - max(0, sz), max(0, -sy):ny - max(0, sy),
            max(0, -sx):nx - max(0, sx)] = M[max(0, sz):nz - max(0, -sz) or None,
                                              max(0, sy):ny - max(0, -sy) or None,
                                              max(0, sx):nx - max(0, -sx) or None]
        assert np.array_equal(Mw.astype(np.float32), ref)


# ------------------------------------------------------------------ loss and gradients
# the two tilings of the stencil passes: 32 x 8 columns marching through z
# chunks, and bricks of 8 x 8 columns, 4 or 8 planes deep (the default below
# 2^20 voxels)
STENCILS = [1, 2]


@pytest.mark.parametrize("stencil", STENCILS)
@pytest.mark.parametrize("window,sigma", [(3, 1.0), (5, 0.7), (7, 1.0), (9, 1.6)])
def test_loss_and_gradients_match_oracle(L, orc, window, sigma, stencil):
    F, M = smooth_pair(RAGGED, 10 + window)
    rng = np.random.default_rng(11)
    u = (rng.uniform(-2, 2, (3,) + RAGGED)).astype(np.float32)
    ctx = L.Context(RAGGED, window=window, grad_sigma=sigma, stencil=stencil)
    loss, gr, gs, cc = ctx.loss_grad(dev(F), dev(M), dev(u), cc=True)
    rL, rg = orc.loss_grad(F, M, u, window, 1e-5)
    rMw = orc.warp(M, u)
    _, rcc = orc.lncc(F, rMw, window, 1e-5, with_map=True)
    rgs = orc.gauss(rg, sigma)
    print(f"[loss w={window} stencil={stencil}] gpu={loss:.12f} oracle={rL:.12f}",
          flush=True)
    assert abs(loss - rL) < 2e-7
    e = report("cc", host(cc), rcc)
    assert e < 2e-6, e
    gmax = np.abs(rg).max()
    e = report("g_raw", host(gr), rg)
    assert e < 2e-5 * gmax, e
    e = report("g_smooth", host(gs), rgs)
    assert e < 2e-5 * gmax, e


@pytest.mark.parametrize("stencil", STENCILS)
@pytest.mark.parametrize("window,sigma", [(5, 0.7), (9, 1.6)])
def test_compensated_fp32_sums_match_oracle(L, orc, window, sigma, stencil):
    """Box sums kept as unevaluated FP32 pairs (LMR_ACC_F32C) carry about
    twice FP32's significand, so loss and gradients meet the same bounds as
    the FP64 sums."""
    F, M = smooth_pair(RAGGED, 30 + window)
    rng = np.random.default_rng(12)
    u = (rng.uniform(-2, 2, (3,) + RAGGED)).astype(np.float32)
    ctx = L.Context(RAGGED, window=window, grad_sigma=sigma, accum=1, stencil=stencil)
    loss, gr, gs, cc = ctx.loss_grad(dev(F), dev(M), dev(u), cc=True)
    rL, rg = orc.loss_grad(F, M, u, window, 1e-5)
    rMw = orc.warp(M, u)
    _, rcc = orc.lncc(F, rMw, window, 1e-5, with_map=True)
    print(f"[loss f32c w={window}] gpu={loss:.12f} oracle={rL:.12f}", flush=True)
    assert abs(loss - rL) < 2e-7
    e = report("cc(f32c)", host(cc), rcc)
    assert e < 2e-6, e
    gmax = np.abs(rg).max()
    e = report("g_raw(f32c)", host(gr), rg)
    assert e < 2e-5 * gmax, e
    e = report("g_smooth(f32c)", host(gs), orc.gauss(rg, sigma))
    assert e < 2e-5 * gmax, e


@pytest.mark.parametrize("accum", [0, 1])
def test_deep_bricks_match_oracle(L, orc, accum):
    """The cube form with 8-plane bricks (a volume giving at least 512 of
    them; the smaller ragged volume above runs 4-plane bricks), ragged
    against the brick in every axis."""
    shape = (44, 77, 83)
    F, M = smooth_pair(shape, 77)
    rng = np.random.default_rng(13)
    u = (rng.uniform(-2, 2, (3,) + shape)).astype(np.float32)
    ctx = L.Context(shape, window=7, grad_sigma=1.0, accum=accum, stencil=2)
    loss, gr, gs, cc = ctx.loss_grad(dev(F), dev(M), dev(u), cc=True)
    rL, rg = orc.loss_grad(F, M, u, 7, 1e-5)
    _, rcc = orc.lncc(F, orc.warp(M, u), 7, 1e-5, with_map=True)
    print(f"[loss deep bricks accum={accum}] gpu={loss:.12f} oracle={rL:.12f}", flush=True)
    assert abs(loss - rL) < 2e-7
    e = report("cc(deep)", host(cc), rcc)
    assert e < 2e-6, e
    gmax = np.abs(rg).max()
    e = report("g_raw(deep)", host(gr), rg)
    assert e < 2e-5 * gmax, e
    e = report("g_smooth(deep)", host(gs), orc.gauss(rg, 1.0))
    assert e < 2e-5 * gmax, e


def test_identical_images_give_minus_one_and_zero_gradient(L):
    F, _ = smooth_pair((24, 24, 40), 12)
    u = np.zeros((3, 24, 24, 40), np.float32)
    ctx = L.Context(F.shape, window=5, cc_eps=0.0)
    loss, gr, _, _ = ctx.loss_grad(dev(F), dev(F), dev(u), smooth=False)
    assert abs(loss + 1.0) < 1e-12
    assert np.abs(host(gr)).max() < 1e-5


# ------------------------------------------------------------------ update
@pytest.mark.parametrize("compositive", [1, 0])
def test_update_matches_oracle(L, orc, compositive):
    rng = np.random.default_rng(13)
    u = rng.uniform(-2, 2, (3,) + RAGGED).astype(np.float32)
    g = (rng.standard_normal((3,) + RAGGED) * 10 ** rng.uniform(-2, 1, RAGGED)
         ).astype(np.float32)
    r, lam = 0.37, 0.05
    ctx = L.Context(RAGGED, compositive=compositive, step_eps=0.8)
    out = host(ctx.update(dev(u), dev(g), r, lam))
    ref = orc.integrate(u, orc.closed_form(g, r, lam), 0.8, compositive)
    e = report("update", out, ref)
    assert e < 2e-5, e


@pytest.mark.parametrize("sign", [-1.0, 1.0])
def test_gathers_at_volume_corners(L, orc, sign):
    """Displacements of one sign everywhere put the trilinear cell of the
    first (sign < 0) or last (sign > 0) voxel half outside the volume along
    all three axes; warp and update must still read the in-volume corner."""
    shape = (9, 10, 11)
    rng = np.random.default_rng(40)
    M = rng.uniform(0.5, 1.5, shape).astype(np.float32)
    u = np.full((3,) + shape, 0.3 * sign, np.float32)
    got = host(L.warp(dev(M), dev(u)))
    ref = orc.warp(M, u)
    e = np.abs(got - ref).max()
    assert e < 1e-6, e
    uu = rng.uniform(0.5, 1.5, (3,) + shape).astype(np.float32)
    g = np.full((3,) + shape, -sign, np.float32)      # du has the sign of `sign`
    ctx = L.Context(shape)
    out = host(ctx.update(dev(uu), dev(g), 0.4, 0.1))
    ref = orc.integrate(uu, orc.closed_form(g, 0.4, 0.1), 1.0, 1)
    e = np.abs(out - ref).max()
    assert e < 2e-6, e


@pytest.mark.parametrize("nx", [12, 11, 4])
def test_bf16_gathers_at_row_ends(L, orc, nx):
    """BF16 images: even rows of four or more elements take both corners of a
    row from one 8-byte load (clamped at the row end), odd rows one load per
    corner; displacements reach past both ends of every axis."""
    from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne
    shape = (9, 10, nx)
    rng = np.random.default_rng(41 + nx)
    M = bf16_to_f32(to_bf16_rne(rng.uniform(0.5, 1.5, shape).astype(np.float32)))
    for u in (rng.uniform(-3, 3, (3,) + shape).astype(np.float32),
              np.full((3,) + shape, 0.3, np.float32), np.full((3,) + shape, -0.3, np.float32)):
        got, dgot = L.warp(dev(M, torch.bfloat16), dev(u), with_grad=True)
        ref, dref = orc.warp(M, u, with_grad=True)
        e, de = np.abs(host(got) - ref).max(), np.abs(host(dgot) - dref).max()
        assert e < 1e-6 and de < 1e-5, (nx, e, de)


# Large enough for the LDS-staged form of the update (ragged in x, y and in
# the last z-chunk).  With the smaller gradients most steps go beyond one
# voxel, where the gather falls back to memory; with the larger none do.
STAGED = (67, 100, 330)


@pytest.mark.parametrize("scale, lam", [(1.0, 0.05), (0.1, 0.01)])
def test_staged_update_matches_oracle(L, orc, scale, lam):
    rng = np.random.default_rng(17)
    u = rng.uniform(-2, 2, (3,) + STAGED).astype(np.float32)
    g = (scale * rng.standard_normal((3,) + STAGED)).astype(np.float32)
    ctx = L.Context(STAGED, step_eps=0.8)
    out = host(ctx.update(dev(u), dev(g), 0.37, lam))
    v = orc.closed_form(g, 0.37, lam)
    far = (np.abs(0.8 * v) >= 1.0).any(axis=0).mean()
    print(f"\n[staged update] {100 * far:.1f}% of the steps beyond one voxel")
    ref = orc.integrate(u, v, 0.8, 1)
    e = report("staged update", out, ref)
    assert e < 2e-5, e
    assert (far == 0.0) if scale == 1.0 else (0.3 < far < 0.9), far


# ------------------------------------------------------------------ decision
def test_decide_probe_matches_golden_tables(L):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "decision_tables.json")
    for case in json.load(open(path))["cases"]:
        kw = dict(case["params"])
        ctx = L.Context((4, 4, 4), **{k: v for k, v in kw.items()
                                      if k not in ("window",)})
        st = dict(case["state"])
        for step in case["steps"]:
            st = ctx.decide_probe(st, step["cand"], step.get("force", -1))
            assert bool(st["accepted"]) == step["accept"], (case["name"], step)
            assert st["lambda_"] == pytest.approx(step["lambda"], rel=1e-15)
            if "stalled" in step:
                assert st["stalled"] == step["stalled"]


# ------------------------------------------------------------------ whole attempts
def _config1(seed=0):
    from paper_2603_19371_amd import phantoms
    return phantoms.blobs((32, 32, 32), seed=seed)


def _oracle_run(orc, F, M, n, params, lambda0=1.0, forces=None):
    pr = orc.Pair(F, M, params).begin(lambda0=lambda0)
    dec, lams = [], []
    for t in range(n):
        dec.append(pr.attempt(-1 if forces is None else forces[t]))
        lams.append(pr.state.lambda_)
    return pr, dec, lams


def test_begin_matches_oracle(L, orc):
    ph = _config1(0)
    ctx = L.Context(ph.F.shape, window=5)
    ctx.begin(dev(ph.F), dev(ph.M), lambda0=1.0)
    st = ctx.state()
    pr = orc.Pair(ph.F, ph.M, orc.Params(window=5)).begin(lambda0=1.0)
    assert abs(st["loss"] - pr.state.loss) < 2e-7
    assert st["lambda_"] == 1.0 and st["n_hist"] == 1
    g = host(ctx.grad())
    e = report("g_smooth(begin)", g, pr.gs)
    assert e < 2e-5 * np.abs(pr.gs).max(), e


def test_one_attempt_field_within_1e4(L, orc):
    ph = _config1(0)
    ctx = L.Context(ph.F.shape, window=5)
    ctx.begin(dev(ph.F), dev(ph.M), lambda0=1.0)
    ctx.step_forced(dev(ph.F), dev(ph.M), [1])
    pr, _, _ = _oracle_run(orc, ph.F, ph.M, 1, orc.Params(window=5), forces=[1])
    e = report("field(1 attempt)", host(ctx.field()), pr.u)
    assert e < 1e-4, e
    st = ctx.state()
    assert abs(st["loss"] - pr.state.loss) < 1e-6


def test_one_attempt_field_within_1e4_compensated_fp32(L, orc):
    ph = _config1(0)
    ctx = L.Context(ph.F.shape, window=5, accum=1)
    ctx.begin(dev(ph.F), dev(ph.M), lambda0=1.0)
    ctx.step_forced(dev(ph.F), dev(ph.M), [1])
    pr, _, _ = _oracle_run(orc, ph.F, ph.M, 1, orc.Params(window=5), forces=[1])
    e = report("field(1 attempt, f32c)", host(ctx.field()), pr.u)
    assert e < 1e-4, e
    assert abs(ctx.state()["loss"] - pr.state.loss) < 1e-6


@pytest.mark.parametrize("accum", [0, 1])
def test_abdomen_cross_modal_attempts_match_oracle(L, orc, accum):
    """Abdomen-like cross-modal pair (CT-like fixed, MR-like moving), w = 7:
    begin and three automatic attempts match the oracle within 1e-4 voxel,
    with the same decisions."""
    from paper_2603_19371_amd.phantoms import abdomen
    ph = abdomen((48, 40, 48), seed=4)
    ctx = L.Context(ph.F.shape, window=7, accum=accum)
    ctx.begin(dev(ph.F), dev(ph.M), lambda0=1.0)
    ctx.step(dev(ph.F), dev(ph.M), 3)
    pr, dec, lams = _oracle_run(orc, ph.F, ph.M, 3, orc.Params(window=7))
    st = ctx.state()
    e = report(f"field(abdomen, 3 attempts, accum={accum})", host(ctx.field()), pr.u)
    assert e < 1e-4, e
    assert st["lambda_"] == lams[-1]
    assert abs(st["loss"] - pr.state.loss) < 1e-6


def _teacher_forced(L, orc, F_or, M_or, F_gpu, M_gpu, img_dtype, n, refs, window=5,
                    accum=0):
    """Runs the oracle's own config-1 trajectory (automatic decisions) and, at
    every attempt t, restarts the GPU from the oracle's accepted state: the
    field rounded to FP32 (the library's storage), lambda and the loss
    history.  The GPU attempt (forced accept, so that the candidate is kept)
    must reproduce the candidate the oracle computes from that same FP32
    field.  ``refs`` lists (name, F, M, tol) oracle references evaluated on
    the same state.  Returns the per-attempt errors of every reference and
    the worst candidate-loss error against the first reference."""
    p = orc.Params(window=window)
    traj = orc.Pair(F_or, M_or, p).begin(lambda0=1.0)
    ctx = L.Context(F_or.shape, img_dtype=img_dtype, window=window, accum=accum)
    errs = {name: [] for name, *_ in refs}
    worst_loss = 0.0
    for t in range(n):
        u32 = traj.u.astype(np.float32)
        ctx.begin(F_gpu, M_gpu, field=dev(u32), lambda0=traj.state.lambda_)
        ctx.step_forced(F_gpu, M_gpu, [1])
        got = host(ctx.field())
        cand = ctx.state()["cand_loss"]
        for name, Fr, Mr, tol in refs:
            ref = orc.Pair(Fr, Mr, p).begin(u0=u32, lambda0=traj.state.lambda_)
            ref.attempt(force=1)
            errs[name].append(float(np.abs(got - ref.u).max()))
            if name == refs[0][0]:
                worst_loss = max(worst_loss, abs(cand - ref.state.loss))
        traj.attempt()
    for name, *_ in refs:
        e = errs[name]
        print(f"[teacher-forced {name}] max|err| first attempt {e[0]:.3e}, "
              f"worst over {n} attempts {max(e):.3e} (attempt {int(np.argmax(e))});"
              f" worst |cand loss err| {worst_loss:.3e}", flush=True)
    return errs, worst_loss


def test_teacher_forced_config1_trajectory_within_1e4(L, orc):
    """Config 1 (32^3 blobs, w=5, sigma 1, lambda0 1, x2/x0.5, tau 0, 50
    attempts).  The trajectory itself is discontinuous in its inputs (the
    trilinear derivative jumps at cell boundaries), so an FP32 run and the
    FP64 run part ways after ~20 attempts whatever the implementation; the
    field is therefore checked at every attempt of the oracle's trajectory
    from the oracle's own state."""
    ph = _config1(0)
    errs, wl = _teacher_forced(L, orc, ph.F, ph.M, dev(ph.F), dev(ph.M),
                               torch.float32, 50, [("fp32", ph.F, ph.M, 1e-4)])
    assert max(errs["fp32"]) < 1e-4
    assert wl < 1e-6


def test_teacher_forced_bf16_images(L, orc):
    """BF16 image storage.  Implementation parity: every attempt within 1e-4
    of the oracle run on the same BF16-rounded images.  Precision effect
    against the oracle on the FP32 images: within 5e-3 on the first attempt
    (lambda0 = 1); later, as lambda falls, the step's sensitivity to the
    gradient grows like r / lambda and the input quantisation shows through
    (the oracle itself shows the same difference); it is reported, not
    bounded."""
    from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne
    ph = _config1(1)
    Fr, Mr = bf16_to_f32(to_bf16_rne(ph.F)), bf16_to_f32(to_bf16_rne(ph.M))
    errs, _ = _teacher_forced(
        L, orc, ph.F, ph.M, dev(Fr, torch.bfloat16), dev(Mr, torch.bfloat16),
        torch.bfloat16, 30, [("bf16-images", Fr, Mr, 1e-4),
                             ("fp32-images", ph.F, ph.M, 5e-3)])
    assert max(errs["bf16-images"]) < 1e-4
    assert errs["fp32-images"][0] < 5e-3


def test_teacher_forced_bf16_images_compensated_fp32(L, orc):
    """The precision form with compensated FP32 box sums in place of FP64
    ones: BF16 images, FP32 field, FP64 loss reduction.  Every attempt
    within 1e-4 of the oracle on the same BF16 values; the first within
    5e-3 of the oracle on the FP32 images."""
    from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne
    ph = _config1(1)
    Fr, Mr = bf16_to_f32(to_bf16_rne(ph.F)), bf16_to_f32(to_bf16_rne(ph.M))
    errs, wl = _teacher_forced(
        L, orc, ph.F, ph.M, dev(Fr, torch.bfloat16), dev(Mr, torch.bfloat16),
        torch.bfloat16, 10, [("bf16-images f32c", Fr, Mr, 1e-4),
                             ("fp32-images f32c", ph.F, ph.M, 5e-3)], accum=1)
    assert max(errs["bf16-images f32c"]) < 1e-4
    assert errs["fp32-images f32c"][0] < 5e-3
    assert wl < 1e-6


LUNG = (384, 384, 384)


@pytest.fixture(scope="module")
def lung_full():
    """The 384^3 lung-CT-like pair of the precision-form workload (seed 0)."""
    from paper_2603_19371_amd.phantoms import lung
    return lung(LUNG, seed=0)


@pytest.mark.parametrize("accum", [0, 1])
def test_lung_precision_form(L, orc, lung_full, accum):
    """Precision form on the centred 64^3 crop of the 384^3 lung-CT-like pair
    (w = 7): BF16 images, FP32 field, FP64 loss reduction, with FP64 box sums
    (accum 0) and with compensated FP32 box sums (accum 1, the form as the
    precision configuration states it).  Implementation: every attempt of
    the oracle's trajectory restarted from the oracle's state matches the
    oracle on the same BF16 values within 1e-4.  Precision effect: the first
    attempt's distance from the FP32-image oracle is the distance between the
    oracle's own runs on the BF16 and the FP32 images (the storage format's
    effect, 7.6e-3 voxel on this crop: above the 5e-3 aimed for, and not a
    property of the kernels) within 1e-4; a free two-level run (2x/1x, 20/10
    attempts) ends within 2e-3 of the loss of the FP32-image GPU run with
    FP64 sums."""
    from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne
    c = tuple(slice(d // 2 - 32, d // 2 + 32) for d in LUNG)
    F = np.ascontiguousarray(lung_full.F[c])
    M = np.ascontiguousarray(lung_full.M[c])
    Fr, Mr = bf16_to_f32(to_bf16_rne(F)), bf16_to_f32(to_bf16_rne(M))
    errs, wl = _teacher_forced(
        L, orc, F, M, dev(Fr, torch.bfloat16), dev(Mr, torch.bfloat16),
        torch.bfloat16, 10, [(f"lung crop bf16-images accum={accum}", Fr, Mr, 1e-4),
                             (f"lung crop fp32-images accum={accum}", F, M, 5e-3)],
        window=7, accum=accum)
    assert max(errs[f"lung crop bf16-images accum={accum}"]) < 1e-4
    assert wl < 1e-6
    p = orc.Params(window=7)
    ob = orc.Pair(Fr, Mr, p).begin(lambda0=1.0)
    of = orc.Pair(F, M, p).begin(lambda0=1.0)
    ob.attempt(force=1)
    of.attempt(force=1)
    storage = float(np.abs(ob.u - of.u).max())
    gpu = errs[f"lung crop fp32-images accum={accum}"][0]
    print(f"[lung precision accum={accum}] first attempt vs the FP32-image oracle: GPU "
          f"{gpu:.3e}, oracle on the BF16 images {storage:.3e}", flush=True)
    assert abs(gpu - storage) < 1e-4
    assert storage < 2e-2
    runs = {}
    for name, Fi, Mi, dt, acc in (("bf16", Fr, Mr, torch.bfloat16, accum),
                                  ("fp32", F, M, torch.float32, 0)):
        pyr = L.Pyramid(F.shape, (2, 1), img_dtype=dt, window=7, accum=acc)
        u = host(pyr.run(dev(Fi, dt), dev(Mi, dt), [20, 10]))
        runs[name] = (u, pyr.level(1).state()["loss"])
    dL = abs(runs["bf16"][1] - runs["fp32"][1])
    du = float(np.abs(runs["bf16"][0] - runs["fp32"][0]).max())
    print(f"[lung precision accum={accum}] final loss bf16 {runs['bf16'][1]:.6f} fp32 "
          f"{runs['fp32'][1]:.6f} |dL| {dL:.2e}; field max|diff| {du:.3e}", flush=True)
    assert dL < 2e-3, dL


def test_compensated_sums_on_long_chunks(L, orc, lung_full):
    """Compensated FP32 box sums where the stencil tiles march long z-chunks
    (384^3: 96 planes a chunk, about 200 additions per running sum): the
    loss of the whole volume against the oracle within 2e-7, the cc map and
    the raw gradient on sampled voxels within 2e-6 and 2e-5 of max|g|."""
    ph = lung_full
    u = (0.5 * ph.t).astype(np.float32)
    ctx = L.Context(LUNG, window=7, accum=1)
    loss, gr, _, cc = ctx.loss_grad(dev(ph.F), dev(ph.M), dev(u), smooth=False, cc=True)
    orc.set_threads(16)
    rL = -orc.lncc(ph.F, orc.warp(ph.M, u), 7, 1e-5)
    print(f"[f32c 384^3 loss] gpu={loss:.12f} oracle={rL:.12f}", flush=True)
    assert abs(loss - rL) < 2e-7
    ccd, grd = host(cc), host(gr)
    gmax = np.abs(grd).max()
    F64, M64, u64 = (a.astype(np.float64) for a in (ph.F, ph.M, u))
    worst_cc = worst_g = 0.0
    for (z, y, x) in _samples(LUNG, 32, 9):
        ecc = abs(ccd[z, y, x] - orc.cc_at(F64, M64, u64, 7, 1e-5, x, y, z))
        eg = np.abs(grd[:, z, y, x] - orc.grad_at(F64, M64, u64, 7, 1e-5, x, y, z)).max()
        worst_cc, worst_g = max(worst_cc, ecc), max(worst_g, eg)
    print(f"[f32c 384^3 samples] cc max|err| {worst_cc:.3e}, g max|err| {worst_g:.3e} "
          f"(max|g| {gmax:.3e})", flush=True)
    assert worst_cc < 2e-6
    assert worst_g < 2e-5 * gmax


def test_force_decision_matches_forced_steps(L):
    """lmr_force_decision (a mode for later lmr_step calls) and lmr_step_forced
    (decisions per call) give the same attempts, bit for bit; a forced
    rejection leaves the field and raises lambda by mu+."""
    ph = _config1(7)
    Fd, Md = dev(ph.F), dev(ph.M)
    seq = [1, 0, 0, 1, -1, 1]
    a = L.Context(ph.F.shape, window=5)
    a.begin(Fd, Md)
    a.step_forced(Fd, Md, seq)
    b = L.Context(ph.F.shape, window=5)
    b.begin(Fd, Md)
    for d in seq:
        before = (host(b.field()), b.state())
        b.force_decision(d)
        b.step(Fd, Md, 1)
        if d == 0:
            st = b.state()
            assert np.array_equal(host(b.field()), before[0])
            assert st["accepted"] == 0
            lam_max = L.Params.make().lambda_max
            assert st["lambda_"] == min(before[1]["lambda_"] * 2.0, lam_max)
    b.force_decision(-1)
    assert np.array_equal(host(a.field()), host(b.field()))
    assert a.state() == b.state()
    with pytest.raises(L.LmrError):
        b.force_decision(2)


def test_checkpoint_resume_is_bitwise(L):
    ph = _config1(5)
    Fd, Md = dev(ph.F), dev(ph.M)
    a = L.Context(ph.F.shape, window=5)
    a.begin(Fd, Md)
    a.step(Fd, Md, 12)
    u_ck, st_ck = a.field().clone(), a.state()
    a.step(Fd, Md, 10)
    b = L.Context(ph.F.shape, window=5)
    b.begin(Fd, Md, field=u_ck, lambda0=st_ck["lambda_"])
    b.set_state(st_ck)
    b.step(Fd, Md, 10)
    assert np.array_equal(host(a.field()), host(b.field()))
    sa, sb = a.state(), b.state()
    assert sa == sb, (sa, sb)


def test_automatic_config1_run_tracks_oracle(L, orc):
    """Unforced: the GPU takes its own decisions over the 50 attempts of the
    32^3 blob configuration.  The decision rule (eq. lambda-update,
    eq. rejection) compares FP64 losses that differ between the FP32 kernels
    and the FP64 oracle by ~1e-8, so a candidate within that of the accepted
    loss may be decided differently; at most 2 of the 50 decisions may
    differ.  The fields agree within 1e-4 voxel at every attempt up to the
    first differing decision or attempt 6, whichever comes first (the
    trilinear derivative's jumps at cell boundaries part any FP32 run from
    the FP64 one: on this pair the difference reaches 1e-4 near attempt 10;
    every attempt of the trajectory is checked from the oracle's own state
    by the teacher-forced test), and the final loss within 1e-4."""
    ph = _config1(0)
    n = 50
    pr = orc.Pair(ph.F, ph.M, orc.Params(window=5)).begin(lambda0=1.0)
    ctx = L.Context(ph.F.shape, window=5)
    Fd, Md = dev(ph.F), dev(ph.M)
    ctx.begin(Fd, Md, lambda0=1.0)
    dec, gdec, errs = [], [], []
    for _ in range(n):
        dec.append(pr.attempt())
        ctx.step(Fd, Md, 1)
        gdec.append(bool(ctx.state()["accepted"]))
        errs.append(float(np.abs(host(ctx.field()) - pr.u).max()))
    mism = [t for t in range(n) if dec[t] != gdec[t]]
    first = mism[0] if mism else n
    agree = min(first, 6)
    print(f"[auto] decision mismatches {len(mism)}/{n} at {mism}; field max|err| per "
          f"attempt {['%.1e' % e for e in errs[:12]]}..., at the end {errs[-1]:.3e}",
          flush=True)
    assert len(mism) <= 2, mism
    assert max(errs[:agree]) < 1e-4
    st = ctx.state()
    assert abs(st["loss"] - pr.state.loss) < 1e-4
    assert st["attempts"] == n


def test_run_is_bitwise_deterministic(L):
    ph = _config1(2)
    outs = []
    for _ in range(2):
        ctx = L.Context(ph.F.shape, window=5)
        ctx.begin(dev(ph.F), dev(ph.M))
        ctx.step(dev(ph.F), dev(ph.M), 20)
        outs.append((host(ctx.field()), ctx.state()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


def test_fixed_image_statistics_follow_the_buffer(L):
    """The window statistics of F come from lmr_begin while the step gets the
    same buffer, and are recomputed when it gets another one: both runs are
    bitwise equal when the buffers hold the same image."""
    ph = _config1(2)
    outs = []
    for same in (True, False):
        ctx = L.Context(ph.F.shape, window=5)
        F0, Md = dev(ph.F), dev(ph.M)
        ctx.begin(F0, Md)
        ctx.step(F0 if same else dev(ph.F), Md, 10)
        outs.append((host(ctx.field()), ctx.state()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


def test_stalled_pair_is_frozen(L):
    ph = _config1(3)
    ctx = L.Context(ph.F.shape, window=5, lambda_max=4.0, max_retries=2)
    Fd, Md = dev(ph.F), dev(ph.M)
    ctx.begin(Fd, Md, lambda0=1.0)
    ctx.step_forced(Fd, Md, [0, 0, 0])          # 2, 4 (cap), 4 -> frozen
    st = ctx.state()
    assert st["stalled"] == 1 and st["lambda_"] == 4.0
    u0 = host(ctx.field())
    ctx.step(Fd, Md, 3)
    st2 = ctx.state()
    assert st2["stalled"] == 1 and st2["attempts"] == st["attempts"]
    assert np.array_equal(host(ctx.field()), u0)


def test_accepted_attempts_never_raise_the_loss(L):
    ph = _config1(4)
    ctx = L.Context(ph.F.shape, window=5)
    Fd, Md = dev(ph.F), dev(ph.M)
    ctx.begin(Fd, Md)
    prev = ctx.state()["loss"]
    for _ in range(30):
        ctx.step(Fd, Md, 1)
        st = ctx.state()
        if st["accepted"]:
            assert st["loss"] <= prev
        prev = st["loss"]


# ------------------------------------------------------------------ full size, sampled
FULL = (160, 192, 224)


@pytest.fixture(scope="module")
def brain_full():
    from paper_2603_19371_amd import phantoms
    return phantoms.brain(FULL, seed=0)


def _samples(shape, n, seed):
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (shape[0] - 1, shape[1] - 1, shape[2] - 1),
           (shape[0] // 2, 0, shape[2] - 1), (3, shape[1] - 2, 5)]
    pts += [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(n)]
    return pts


def test_full_size_loss_cc_and_gradient_samples(L, orc, brain_full):
    ph = brain_full
    u = (0.5 * ph.t).astype(np.float32)
    ctx = L.Context(FULL, window=7)
    loss, gr, _, cc = ctx.loss_grad(dev(ph.F), dev(ph.M), dev(u), smooth=False,
                                    cc=True)
    orc.set_threads(16)
    rMw = orc.warp(ph.M, u)
    rL = -orc.lncc(ph.F, rMw, 7, 1e-5)
    print(f"[full loss] gpu={loss:.12f} oracle={rL:.12f}", flush=True)
    assert abs(loss - rL) < 2e-7
    ccd, grd = host(cc), host(gr)
    gmax = np.abs(grd).max()
    F64, M64, u64 = (a.astype(np.float64) for a in (ph.F, ph.M, u))
    for (z, y, x) in _samples(FULL, 24, 5):
        assert abs(ccd[z, y, x] - orc.cc_at(F64, M64, u64, 7, 1e-5, x, y, z)) < 2e-6
        rg = orc.grad_at(F64, M64, u64, 7, 1e-5, x, y, z)
        assert np.abs(grd[:, z, y, x] - rg).max() < 2e-5 * gmax, (z, y, x)


def test_full_size_one_attempt_field_within_1e4(L, orc, brain_full):
    """One whole attempt at 160x192x224 (w=7, sigma 1) from the identity, in
    the benchmark's launch configuration, against the full FP64 oracle."""
    ph = brain_full
    orc.set_threads(16)
    ctx = L.Context(FULL, window=7)
    Fd, Md = dev(ph.F), dev(ph.M)
    ctx.begin(Fd, Md, lambda0=1.0)
    ctx.step_forced(Fd, Md, [1])
    got = host(ctx.field())
    st = ctx.state()
    pr = orc.Pair(ph.F, ph.M, orc.Params(window=7)).begin(lambda0=1.0)
    pr.attempt(force=1)
    e = report("full-size field(1 attempt)", got, pr.u)
    assert e < 1e-4, e
    assert abs(st["loss"] - pr.state.loss) < 2e-7


def test_full_size_smooth_and_update_samples(L, orc):
    rng = np.random.default_rng(21)
    g = rng.standard_normal((3,) + FULL).astype(np.float32)
    u = rng.uniform(-3, 3, (3,) + FULL).astype(np.float32)
    ctx = L.Context(FULL, window=7)
    gs = host(ctx.smooth(dev(g)))
    un = host(ctx.update(dev(u), dev(g), 0.3, 0.02))
    g64, u64 = g.astype(np.float64), u.astype(np.float64)
    for (z, y, x) in _samples(FULL, 40, 6):
        np.testing.assert_allclose(gs[:, z, y, x], orc.gauss_at(g64, 1.0, x, y, z),
                                   atol=2e-6)
        gv = g64[:, z, y, x]
        v = -0.3 * gv / (gv @ gv + 0.02)
        ref = [v[c] + orc.sample(u64[c], (x + v[0], y + v[1], z + v[2]))
               for c in range(3)]
        np.testing.assert_allclose(un[:, z, y, x], ref, atol=2e-5)


def test_full_size_attempts_properties(L, brain_full):
    """Whole attempts at full size (the benchmark's launch configuration):
    bitwise determinism, monotone accepted losses (tau = 0) and the step bound
    |du| <= r / (2 sqrt(lambda)) of the closed form."""
    ph = brain_full
    Fd, Md = dev(ph.F), dev(ph.M)
    fields = []
    for rep in range(2):
        ctx = L.Context(FULL, window=7)
        ctx.begin(Fd, Md, lambda0=1.0)
        st0 = ctx.state()
        ctx.step_forced(Fd, Md, [1])
        # from u = 0 the candidate is eps du itself: |du| <= r / (2 sqrt(lambda))
        du = ctx.field().norm(dim=0).max().item()
        assert du <= (1 + st0["loss"]) / (2 * math.sqrt(st0["lambda_"])) * (1 + 1e-5)
        prev = ctx.state()
        for _ in range(4):
            ctx.step(Fd, Md, 1)
            st = ctx.state()
            if st["accepted"]:
                assert st["loss"] <= prev["loss"]
            prev = st
        fields.append(host(ctx.field()))
    assert np.array_equal(fields[0], fields[1])
