"""Batched persistent form: equivalence with per-pair runs and graph replays,
and parity with the FP64 oracle at the shapes of the 16-pair workload."""
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(20, 37, 70), (32, 32, 32), (24, 40, 48)]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2603_19371_amd import _lib
    _lib.lib()
    return _lib


@pytest.fixture(scope="module")
def pairs():
    from paper_2603_19371_amd import phantoms
    out = []
    for i, sh in enumerate(SHAPES):
        ph = phantoms.brain(sh, seed=100 + i) if i != 1 else phantoms.blobs(sh, seed=5)
        out.append((torch.from_numpy(ph.F).cuda(), torch.from_numpy(ph.M).cuda()))
    return out


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("accum", [0, 1])
def test_batch_matches_per_pair_runs(L, pairs, accum):
    """Every pair of the batch follows exactly (bitwise) the run of a
    stand-alone context: these small pairs run on 4-plane bricks in both,
    with the same bricks and the same reduction order; with either box-sum
    accumulator."""
    n = 6
    ref = []
    for (F, M), sh in zip(pairs, SHAPES):
        c = L.Context(sh, window=5, accum=accum)
        c.begin(F, M)
        c.step(F, M, n)
        ref.append((host(c.field()), c.state()))
    b = L.Batch(SHAPES, window=5, accum=accum)
    b.begin([F for F, _ in pairs], [M for _, M in pairs])
    b.step(n, graph=True)
    b.sync()
    for i, (u_ref, st_ref) in enumerate(ref):
        v = b.pair(i)
        assert v.state() == st_ref, (i, v.state(), st_ref)
        assert np.array_equal(host(v.field()), u_ref), i


def test_mixed_batch_matches_per_pair_runs(L):
    """A small pair (bricks) and a pair above 2^20 voxels (marching tiles,
    the staged update) in one persistent launch: each follows its stand-alone
    run bit for bit."""
    from paper_2603_19371_amd import phantoms
    shapes = [(24, 40, 48), (40, 64, 420)]
    imgs = []
    for i, sh in enumerate(shapes):
        ph = phantoms.brain(sh, seed=60 + i)
        imgs.append((torch.from_numpy(ph.F).cuda(), torch.from_numpy(ph.M).cuda()))
    ref = []
    for (F, M), sh in zip(imgs, shapes):
        c = L.Context(sh, window=7)
        c.begin(F, M)
        c.step(F, M, 4)
        ref.append((host(c.field()), c.state()))
    b = L.Batch(shapes, window=7)
    b.begin([F for F, _ in imgs], [M for _, M in imgs])
    b.step(4, graph=True)
    b.sync()
    for i, (u_ref, st_ref) in enumerate(ref):
        assert b.pair(i).state() == st_ref, (i, b.pair(i).state(), st_ref)
        assert np.array_equal(host(b.pair(i).field()), u_ref), i


@pytest.mark.parametrize("accum", [0, 1])
def test_phase_launches_match_persistent_kernel(L, accum):
    """One launch per phase (blocks_per_cu = -1) computes the same items as
    the persistent kernel: identical states and fields, bit for bit, on a
    batch of brick and marching pairs, eager and replayed."""
    from paper_2603_19371_amd import phantoms
    shapes = [(20, 37, 70), (40, 64, 420), (32, 32, 32)]
    Fs, Ms = [], []
    for i, sh in enumerate(shapes):
        ph = phantoms.brain(sh, seed=80 + i)
        Fs.append(torch.from_numpy(ph.F).cuda())
        Ms.append(torch.from_numpy(ph.M).cuda())
    ref = L.Batch(shapes, window=7, accum=accum)
    ref.set_config(0, 16, 0)  # the persistent kernel
    ph_ = L.Batch(shapes, window=7, accum=accum)
    ph_.set_config(0, 16, -1)
    assert ph_.config()["blocks_per_cu"] == -1
    for b in (ref, ph_):
        b.begin(Fs, Ms)
        b.step(2, graph=False)
        b.step(3, graph=True)
        b.sync()
    for i in range(len(shapes)):
        assert ph_.pair(i).state() == ref.pair(i).state(), i
        assert np.array_equal(host(ph_.pair(i).field()), host(ref.pair(i).field())), i


def test_batch_matches_staged_per_pair_run(L):
    """A pair large enough for the per-pair LDS-staged update kernel: the
    batched kernel's memory gathers give the same field bit for bit."""
    from paper_2603_19371_amd import phantoms
    sh = (67, 100, 330)
    ph = phantoms.brain(sh, seed=7)
    F, M = torch.from_numpy(ph.F).cuda(), torch.from_numpy(ph.M).cuda()
    c = L.Context(sh, window=5, stencil=L.LMR_STENCIL_MARCH)
    c.begin(F, M)
    c.step(F, M, 3)
    ref, st_ref = host(c.field()), c.state()
    b = L.Batch([sh], window=5)
    b.begin([F], [M])
    b.step(3, graph=False)
    b.sync()
    assert b.pair(0).state() == st_ref
    assert np.array_equal(host(b.pair(0).field()), ref)


@pytest.mark.parametrize("blocks_per_cu", [-1, 0])
def test_graph_replays_match_eager_steps(L, pairs, blocks_per_cu):
    """Replayed steps equal eager steps, in the per-phase launches (the
    default) and in the persistent kernel."""
    Fs, Ms = [F for F, _ in pairs], [M for _, M in pairs]
    eager = L.Batch(SHAPES, window=5)
    graph = L.Batch(SHAPES, window=5)
    eager.set_config(0, 16, blocks_per_cu)
    graph.set_config(0, 16, blocks_per_cu)
    eager.begin(Fs, Ms)
    graph.begin(Fs, Ms)
    for rep in range(3):
        eager.step(2, graph=False)
        eager.sync()
        graph.step(2, graph=True)
        graph.sync()
        # the program's own work between replays
        _ = (torch.ones(1000, device="cuda") * rep).sum().item()
        for i in range(len(SHAPES)):
            assert graph.pair(i).state() == eager.pair(i).state(), (rep, i)
            assert np.array_equal(host(graph.pair(i).field()),
                                  host(eager.pair(i).field())), (rep, i)


def test_launch_not_co_resident_fails_fast(L, pairs):
    """A launch whose grid is not all on the GPU gives up at its first barrier
    within milliseconds (LMR_EBUSY, not the 0.25 s barrier timeout), leaves
    every pair as the last completed launch left it, and the batch steps on
    afterwards.  The absent block is simulated (lmr_batch_test_residency:
    block 0 starts 4 ms late): the GPU is never actually contended, and every
    wait of the kernel is bounded."""
    Fs, Ms = [F for F, _ in pairs], [M for _, M in pairs]
    b = L.Batch(SHAPES, window=5)
    b.set_config(0, 16, 0)  # the persistent kernel
    b.begin(Fs, Ms)
    b.step(2, graph=False)
    b.sync()
    before = [(host(b.pair(i).field()), b.pair(i).state()) for i in range(len(SHAPES))]
    b.test_residency(1)
    t0 = time.perf_counter()
    b.step(3, graph=False)
    status = b.sync_status()
    dt = time.perf_counter() - t0
    print(f"[co-residency] status={status} after {dt * 1e3:.2f} ms", flush=True)
    assert status == L.LMR_EBUSY
    assert dt < 0.1, dt
    for i, (u, st) in enumerate(before):
        assert b.pair(i).state() == st, i
        assert np.array_equal(host(b.pair(i).field()), u), i
    b.test_residency(0)
    b.step(2, graph=True)
    assert b.sync_status() == 0
    ref = L.Batch(SHAPES, window=5)
    ref.begin(Fs, Ms)
    ref.step(4, graph=False)
    ref.sync()
    for i in range(len(SHAPES)):
        assert b.pair(i).state() == ref.pair(i).state(), i
        assert np.array_equal(host(b.pair(i).field()), host(ref.pair(i).field())), i


def test_autotuner_and_cache(L, pairs, tmp_path):
    Fs, Ms = [F for F, _ in pairs], [M for _, M in pairs]
    b = L.Batch(SHAPES, window=5)
    cache = os.path.join(tmp_path, "tune.txt")
    ms = b.tune(Fs, Ms, cache_path=cache, iters=2)
    cfg = b.config()
    assert ms > 0 and os.path.exists(cache)
    b2 = L.Batch(SHAPES, window=5)
    ms2 = b2.tune(Fs, Ms, cache_path=cache, iters=2)     # read from the cache
    assert b2.config() == cfg and ms2 == pytest.approx(ms)
    b2.begin(Fs, Ms)
    b2.step(3)
    b2.sync()
    for i in range(len(SHAPES)):
        assert b2.pair(i).state()["attempts"] == 3


CONFIG4 = [(96, 96, 96), (128, 160, 128), (160, 192, 224), (192, 160, 256)]


@pytest.fixture(scope="module")
def config4():
    """One brain-like pair of each shape of the 16-pair workload, and the FP64
    oracle's begin and first automatic attempt on each (w = 7, sigma 1)."""
    import oracle
    from paper_2603_19371_amd import phantoms
    oracle.set_threads(16)
    out = []
    for i, sh in enumerate(CONFIG4):
        ph = phantoms.brain(sh, seed=100 + i)
        pr = oracle.Pair(ph.F, ph.M, oracle.Params(window=7)).begin(lambda0=1.0)
        acc = pr.attempt()
        out.append((ph, pr, acc))
        print(f"[config4 oracle] {sh}: accepted {acc}, loss {pr.state.loss:.9f}",
              flush=True)
    return out


@pytest.mark.parametrize("tuned", [False, True])
def test_batch_config4_shapes_match_oracle(L, config4, tuned):
    """The four shapes advance together (graph replay), with the default
    configuration and with the autotuner's choice.  After one automatic
    attempt every pair has the oracle's decision and lambda, its loss within
    2e-7, its field within 1e-4 voxel and the smoothed gradient of its
    accepted field within 2e-5 of max|g|, element by element."""
    Fs = [torch.from_numpy(ph.F).cuda() for ph, _, _ in config4]
    Ms = [torch.from_numpy(ph.M).cuda() for ph, _, _ in config4]
    b = L.Batch(CONFIG4, window=7)
    if tuned:
        b.tune(Fs, Ms, iters=1)
    print(f"[config4] tiling {b.config()}", flush=True)
    b.begin(Fs, Ms)
    b.step(1, graph=True)
    b.sync()
    for i, (ph, pr, acc) in enumerate(config4):
        v = b.pair(i)
        st = v.state()
        assert bool(st["accepted"]) == acc, i
        assert st["lambda_"] == pr.state.lambda_, i
        assert abs(st["loss"] - pr.state.loss) < 2e-7, (i, st["loss"], pr.state.loss)
        u = host(v.field()).astype(np.float64)
        eu = float(np.abs(u - pr.u).max())
        gs = host(v.grad()).astype(np.float64)
        eg = float(np.abs(gs - pr.gs).max())
        gmax = float(np.abs(pr.gs).max())
        print(f"[config4 {CONFIG4[i]} tuned={tuned}] field max|err| {eu:.3e}, "
              f"g_smooth max|err| {eg:.3e} (max|g| {gmax:.3e})", flush=True)
        assert eu < 1e-4, (i, eu)
        assert eg < 2e-5 * gmax, (i, eg)


def test_unsupported_gaussian_radius_is_rejected(L):
    with pytest.raises(L.LmrError):
        L.Batch(SHAPES, window=5, grad_sigma=2.0)
