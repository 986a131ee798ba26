"""The device phantom generator of the learned initializer's training set,
run on the CPU: determinism, value ranges and the built-in inverse."""
import pytest

torch = pytest.importorskip("torch")


def test_brain_pairs_are_seeded_and_well_formed():
    from paper_2603_19371_amd import phantoms_torch as P
    sh = (64, 64, 80)
    F, M, t = P.brain(sh, seed=3, device="cpu")
    F2, M2, t2 = P.brain(sh, seed=3, device="cpu")
    F3, _, _ = P.brain(sh, seed=4, device="cpu")
    assert torch.equal(F, F2) and torch.equal(M, M2) and torch.equal(t, t2)
    assert not torch.equal(F, F3)
    assert F.shape == sh and M.shape == sh and t.shape == (3,) + sh
    assert F.dtype == torch.float32 and F.is_contiguous() and t.is_contiguous()
    assert -0.1 < float(F.min()) and float(F.max()) < 1.1
    assert abs(float(t.square().sum(0).sqrt().max()) - 6.0) < 1e-4
    # M o (Id + t) = F up to noise and resampling: far closer than M itself
    inner = (slice(6, -6),) * 3
    Mw = P._sample(M[None], t)[0]
    e_warp = float((Mw - F)[inner].square().mean().sqrt())
    e_id = float((M - F)[inner].square().mean().sqrt())
    assert e_warp < 0.6 * e_id, (e_warp, e_id)
