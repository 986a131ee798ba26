"""GPU parity of the coarse-to-fine pyramid against the FP64 oracle."""
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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda().to(dtype)


def host(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("img", ["f32", "bf16"])
@pytest.mark.parametrize("f", [2, 4])
def test_avgpool_matches_oracle(L, orc, img, f):
    from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne
    a = np.random.default_rng(1).uniform(0, 1, (24, 40, 72)).astype(np.float32)
    if img == "bf16":
        a = bf16_to_f32(to_bf16_rne(a))
    got = host(L.avgpool(dev(a, torch.bfloat16 if img == "bf16" else torch.float32), f))
    ref = orc.avgpool(a, f)
    assert np.abs(got - ref).max() < 1e-6


def test_upsample_matches_oracle(L, orc):
    uc = np.random.default_rng(2).standard_normal((3, 7, 13, 21)).astype(np.float32)
    got = host(L.upsample_field(dev(uc)))
    ref = orc.upsample_field(uc, (14, 26, 42))
    assert np.abs(got - ref).max() < 2e-6


def test_pyramid_run_with_oracle_decisions(L, orc):
    """A short 3-level registration (factors 4/2/1) with the oracle's
    decisions replayed: final field within 1e-4 voxel."""
    from paper_2603_19371_amd import phantoms
    ph = phantoms.brain((32, 40, 48), seed=3)
    levels = [(4, 4), (2, 3), (1, 2)]
    p = orc.Params(window=5)
    u_ref, dec = orc.register(ph.F, ph.M, p, levels, lambda0=1.0)
    flat = [int(d) for lv in dec for d in lv]
    pyr = L.Pyramid(ph.F.shape, (4, 2, 1), window=5)
    out = pyr.run(dev(ph.F), dev(ph.M), [n for _, n in levels], lambda0=1.0,
                  decisions=flat)
    err = np.abs(host(out) - u_ref).max()
    print(f"[pyramid] max|err|={err:.3e}", flush=True)
    assert err < 1e-4, err
    for l, (_, n) in enumerate(levels):
        assert pyr.level(l).state()["attempts"] == n


def test_pyramid_graph_replays_match_eager_runs(L):
    """The attempts of each level as one replayed HIP graph give the same
    fields and states, bit for bit, as the kernel-by-kernel enqueue, over
    repeated runs with other device work in between."""
    from paper_2603_19371_amd import phantoms
    ph = phantoms.brain((32, 40, 48), seed=4)
    F, M = dev(ph.F), dev(ph.M)
    iters = [12, 8, 5]
    eager = L.Pyramid(ph.F.shape, (4, 2, 1), window=5)
    eager.use_graphs(False)
    ref = host(eager.run(F, M, iters))
    ref_states = [eager.level(l).state() for l in range(3)]
    graph = L.Pyramid(ph.F.shape, (4, 2, 1), window=5)
    for rep in range(3):
        out = graph.run(F, M, iters)
        _ = (torch.ones(1000, device="cuda") * rep).sum().item()
        assert np.array_equal(host(out), ref), rep
        assert [graph.level(l).state() for l in range(3)] == ref_states, rep


def test_sampled_kernel_timing_keeps_the_graph_sequence(L):
    """With kernel timing open at stride 4 on the fine level, the sampled
    attempts run eagerly between their events and the others as graph
    launches: the same fields and states bit for bit, and one timed attempt
    in four (a ragged last chunk included)."""
    from paper_2603_19371_amd import phantoms
    ph = phantoms.brain((32, 40, 48), seed=5)
    F, M = dev(ph.F), dev(ph.M)
    iters = [6, 4, 11]
    eager = L.Pyramid(ph.F.shape, (4, 2, 1), window=5)
    eager.use_graphs(False)
    ref = host(eager.run(F, M, iters))
    ref_states = [eager.level(l).state() for l in range(3)]
    pyr = L.Pyramid(ph.F.shape, (4, 2, 1), window=5)
    fine = pyr.level(2)
    fine.profile_start(max_attempts=100, stride=4)
    for rep in range(2):
        out = pyr.run(F, M, iters)
        assert np.array_equal(host(out), ref), rep
        assert [pyr.level(l).state() for l in range(3)] == ref_states, rep
    prof = fine.profile_stop()
    # attempts 0, 4, 8 of the first run; the count goes on across runs
    # (22 attempts in all: 0, 4, ..., 20)
    assert all(v["count"] == 6 and v["avg_ms"] > 0 for v in prof.values()), prof


@pytest.mark.parametrize("shape", [(9, 10, 11), (20, 37, 70), (1, 16, 24)])
def test_folded_count_is_bit_exact(L, orc, shape):
    """The count is an integer decided in FP64 with the oracle's operation
    order: it must equal the oracle's count exactly."""
    from scipy import ndimage as ndi
    rng = np.random.default_rng(sum(shape))
    u = ndi.gaussian_filter(rng.standard_normal((3,) + shape), (0, 1, 1, 1)) * 5
    u = u.astype(np.float32)
    ctx = L.Context(shape)
    n, det = ctx.folded_count(dev(u), with_det=True)
    rn, rdet = orc.folded_count(u.astype(np.float64), with_det=True)
    assert n == rn
    assert 0 < n < int(np.prod(shape)) or shape[0] == 1
    np.testing.assert_allclose(host(det), rdet, rtol=1e-6, atol=1e-6)
    assert ctx.folded_count(dev(np.zeros((3,) + shape, np.float32))) == 0
