"""Synthetic inputs: the abdomen-like cross-modal pair (the generator holds no
arithmetic of the method; these checks pin its construction)."""
import numpy as np
import pytest

from paper_2603_19371_amd import phantoms


def test_abdomen_is_seeded_and_has_every_class():
    a = phantoms.abdomen((40, 32, 40), seed=5)
    b = phantoms.abdomen((40, 32, 40), seed=5)
    c = phantoms.abdomen((40, 32, 40), seed=6)
    assert a.F.dtype == np.float32 and a.M.dtype == np.float32
    assert a.F.shape == (40, 32, 40) and a.t.shape == (3, 40, 32, 40)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.M, b.M)
    assert not np.array_equal(a.F, c.F)
    counts = np.bincount(a.labels.ravel(), minlength=7)
    assert (counts > 0).all(), counts
    assert np.sqrt((a.t ** 2).sum(0)).max() == pytest.approx(6.0, rel=1e-5)


def test_abdomen_renders_two_modalities_of_one_anatomy():
    """Class means of the fixed image follow the CT table; the moving image
    unwarped by the true field follows the MR table (up to the bias field),
    so fat is dark against liver in one and bright in the other."""
    from scipy import ndimage as ndi
    ph = phantoms.abdomen((48, 40, 48), seed=3, bias=0.0)
    lab = ph.labels
    # M o (Id + t): sample M at x + t(x) (t is [x, y, z] components)
    zz, yy, xx = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in lab.shape],
                             indexing="ij")
    Mt = ndi.map_coordinates(ph.M.astype(np.float64),
                             [zz + ph.t[2], yy + ph.t[1], xx + ph.t[0]], order=1,
                             mode="nearest")
    # (the fat shell is two or three voxels thick here: only its ordering is
    # checked, its mean is dominated by partial volume)
    for k in (2, 3):
        sel = ndi.binary_erosion(lab == k, iterations=1)
        assert sel.sum() > 20
        assert abs(ph.F[sel].mean() - phantoms.ABDOMEN_CT[k]) < 0.03
        assert abs(Mt[sel].mean() - phantoms.ABDOMEN_MR[k]) < 0.05
    fat, liver = (lab == 1), (lab == 3)
    assert ph.F[fat].mean() < ph.F[liver].mean()
    assert Mt[fat].mean() > Mt[liver].mean()


def test_abdomen_loss_falls_under_the_oracle():
    import oracle as orc
    ph = phantoms.abdomen((32, 28, 32), seed=2)
    pr = orc.Pair(ph.F, ph.M, orc.Params(window=7)).begin(lambda0=1.0)
    L0 = pr.state.loss
    for _ in range(10):
        pr.attempt()
    assert pr.state.loss < L0 - 0.05
