"""lmr_loss_grad_noalloc (the entry point for callers that cannot allocate)
against lmr_loss_grad on the same inputs: two calls in a row on one GPU, the
second on a smaller volume, each bitwise equal to the context-based call
(same kernels, same tiling, same reduction order), and within the oracle's
tolerances of the FP64 oracle."""
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


def _pair(shape, seed):
    from paper_2603_19371_amd import phantoms
    ph = phantoms.brain(shape, seed=seed)
    u = (0.5 * ph.t).astype(np.float32)
    return ph.F, ph.M, u


@pytest.mark.parametrize("accum", [0, 1])
def test_noalloc_matches_context_call_twice(L, accum):
    import oracle
    for shape, seed in (((64, 96, 112), 3), ((24, 40, 56), 4)):
        F, M, u = _pair(shape, seed)
        Fd, Md, ud = (torch.from_numpy(a).cuda() for a in (F, M, u))
        print(f"[noalloc] shape {shape} accum {accum}", flush=True)
        loss, gr, gs, cc = L.loss_grad_noalloc(Fd, Md, ud, window=7, accum=accum, cc=True)
        ctx = L.Context(shape, window=7, accum=accum)
        rl, rgr, rgs, rcc = ctx.loss_grad(Fd, Md, ud, cc=True)
        torch.cuda.synchronize()
        assert loss.item() == rl
        assert torch.equal(gr, rgr) and torch.equal(gs, rgs) and torch.equal(cc, rcc)
        oracle.set_threads(16)
        ol = -oracle.lncc(F, oracle.warp(M, u), 7, 1e-5)
        assert abs(loss.item() - ol) < 2e-7, (loss.item(), ol)


def test_noalloc_rejects_volumes_beyond_its_workspace(L):
    shape = (128, 128, 65)   # 1,064,960 voxels > 2^20
    F = torch.zeros(shape, device="cuda")
    u = torch.zeros((3,) + shape, device="cuda")
    with pytest.raises(L.LmrError):
        L.loss_grad_noalloc(F, F, u, window=7)
