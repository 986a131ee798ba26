"""The two tilings of the stencil passes give the same attempts.

Marching 32 x 8 columns and bricks of 8 x 8 columns (4 planes deep below
512 bricks of 8 planes, else 8) sum the same box and Gaussian terms in
different orders (FP64 or compensated FP32 sums), so the candidate fields of a
run differ only by rounding and the accept/reject decisions coincide.  Shapes
are ragged against both tilings (and against the brick edges); the oracle
parity of each form is in test_gpu_parity.py."""
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


def host(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("accum", [0, 1])
@pytest.mark.parametrize("shape,window,sigma", [((13, 9, 30), 3, 0.6),
                                                ((20, 37, 70), 7, 1.0),
                                                ((40, 48, 56), 9, 1.3),
                                                ((44, 77, 83), 7, 1.0)])
def test_cube_and_march_runs_agree(L, shape, window, sigma, accum):
    from paper_2603_19371_amd import phantoms
    ph = phantoms.brain(shape, seed=sum(shape) + window)
    F = torch.from_numpy(ph.F).cuda()
    M = torch.from_numpy(ph.M).cuda()
    runs = []
    for form in (L.LMR_STENCIL_MARCH, L.LMR_STENCIL_CUBE):
        c = L.Context(shape, window=window, grad_sigma=sigma, accum=accum, stencil=form)
        c.begin(F, M)
        states = []
        for _ in range(8):
            c.step(F, M, 1)
            states.append(c.state())
        runs.append((host(c.field()), states))
    (u0, s0), (u1, s1) = runs
    dl = max(abs(a["cand_loss"] - b["cand_loss"]) for a, b in zip(s0, s1))
    err = np.abs(u0 - u1).max()
    print(f"[march vs cube {shape} w={window} accum={accum}] max|dL|={dl:.3e} "
          f"max|du|={err:.3e}", flush=True)
    # the FP32 maps, gradients and fields round differently, and the
    # candidates drift apart by about 1e-7 voxel per attempt
    for a, b in zip(s0, s1):
        assert a["accepted"] == b["accepted"], (a, b)
    assert dl < 2e-7, dl
    assert err < 1e-5, err


def test_auto_form_switches_at_the_size_limit(L):
    """Below 2^20 voxels AUTO is the cube form, above it the march: the same
    pair gives bitwise the same run as the explicit form on each side."""
    from paper_2603_19371_amd import phantoms
    for shape, form in (((64, 128, 128), L.LMR_STENCIL_CUBE),
                        ((64, 128, 129), L.LMR_STENCIL_MARCH)):
        ph = phantoms.blobs(shape, seed=3)
        F = torch.from_numpy(ph.F).cuda()
        M = torch.from_numpy(ph.M).cuda()
        out = []
        for s in (L.LMR_STENCIL_AUTO, form):
            c = L.Context(shape, window=5, stencil=s)
            c.begin(F, M)
            c.step(F, M, 2)
            out.append((host(c.field()), c.state()))
        assert out[0][1] == out[1][1]
        assert np.array_equal(out[0][0], out[1][0]), shape
