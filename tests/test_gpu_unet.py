"""U-Net of the learned initializer: HIP forward/backward (BF16 MFMA, FP32
accumulation) against the FP64 oracle, the optimizer step, and accumulation.

Layer by layer (element by element).  Each of the 15 convolutions runs alone
on BF16 inputs that the oracle sees exactly; the GPU accumulates in FP32, the
oracle in FP64.  The recursive FP32 sum of K products errs by at most about
K 2^-24 of the sum of their magnitudes, far less in practice (errors are
random, ~sqrt(K) 2^-24); with K up to 27 x 192 (forward, input gradient) the
bound taken is 1e-5 of the oracle's sum of |products| at every output, and
1e-4 for the weight and bias gradients, which sum over every voxel of a
level (K up to 860,160); a BF16-stored output (input gradient) adds its own
rounding, 2^-8 of its value.  A wrong tap, index or transposed operand moves
an output by the order of its value, hundreds of times these bounds.  The
shapes give several rows per chunk of the weight-gradient kernel
(72 x 64 x 8: 4,608 level-0 rows; 80 x 96 x 112, the network's real size:
7,680).

Whole network, two comparisons per case.
  Implementation parity: the oracle rounds every activation and activation
  gradient it stores to BF16, where the GPU stores them in BF16, and keeps its
  arithmetic in FP64.  What remains is FP32 accumulation on the GPU against
  FP64 in the oracle, which flips the BF16 rounding of a small fraction of the
  stored values by one unit (2^-8 relative) and those flips propagate through
  the later layers; on the seeded cases the output differs by up to 3.0e-3
  (8 x 24 x 72) and the per-layer gradients by up to 7.2e-3 in relative L2.
  Bounds: output relative L2 <= 5e-3, per-layer gradient relative L2
  <= 1.5e-2 and cosine >= 0.9999, an order of magnitude below what a wrong
  index or a missing term gives (the element-wise layer test below is the
  strict check of each kernel).
  Precision effect: against the plain FP64 oracle (no storage rounding) the
  BF16 storage itself shows, growing with depth and with the few voxels of
  the coarsest level: reported, and bounded at output relative L2 <= 2e-2,
  gradient cosine >= 0.995, relative L2 <= 0.1."""
import numpy as np
import pytest

from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(16, 16, 24), (8, 24, 72)]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2603_19371_amd import _lib
    _lib.lib()
    return _lib


def bf(a):
    return bf16_to_f32(to_bf16_rne(np.asarray(a, np.float32))).astype(np.float64)


def make_case(shape, seed):
    from oracle import unet
    rng = np.random.default_rng(seed)
    params = unet.init_params(seed=seed)
    params = [(bf(W), np.float32(rng.normal(0, 0.05, b.shape)).astype(np.float64))
              for W, b in params]
    F = rng.uniform(0, 1, shape).astype(np.float32)
    M = rng.uniform(0, 1, shape).astype(np.float32)
    target = (rng.standard_normal((3,) + shape) * 0.05).astype(np.float32)
    return params, F, M, target


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def unflat(v, layers):
    out = []
    for ci, co, _, off in layers:
        W = v[off:off + 27 * ci * co].reshape(27, ci, co)
        b = v[off + 27 * ci * co:off + 27 * ci * co + co]
        out.append((W, b))
    return out


def oracle_run(params, F, M, target, rnd=None):
    from oracle import unet
    x = np.stack([bf(F), bf(M)], axis=-1)
    out, acts = unet.forward(params, x, rnd=rnd)
    t = target.transpose(1, 2, 3, 0).astype(np.float64)
    loss, dout = unet.mse(out, t)
    grads, _ = unet.backward(params, acts, rnd(dout) if rnd else dout, rnd=rnd)
    return out.transpose(3, 0, 1, 2), loss, grads


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def cosine(a, b):
    a, b = a.ravel(), b.ravel()
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))


def test_layer_table_matches_oracle(L):
    from oracle import unet
    layers = L.unet_layers()
    assert [(ci, co, r) for ci, co, r, _ in layers] == list(unet.LAYERS)
    assert L.unet_param_count() == sum(27 * ci * co + co for ci, co, _ in unet.LAYERS)


def _compare(tag, out, loss, g, ref):
    out_o, loss_o, grads_o = ref
    e_out = rel_l2(out, out_o)
    e_loss = abs(loss - loss_o) / loss_o
    print(f"\n[unet {tag}] out rel-L2 {e_out:.2e}  loss rel {e_loss:.2e}")
    worst_cos, worst_rel = 1.0, 0.0
    for li, ((gw, gb), (ow, ob)) in enumerate(zip(g, grads_o)):
        c, r, rb = cosine(gw, ow), rel_l2(gw, ow), rel_l2(gb, ob)
        print(f"  layer {li:2d}: dW cos {c:.6f} rel-L2 {r:.2e}  db rel-L2 {rb:.2e}")
        worst_cos, worst_rel = min(worst_cos, c), max(worst_rel, r, rb)
    return e_out, e_loss, worst_cos, worst_rel


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_backward_match_oracle(L, shape):
    params, F, M, target = make_case(shape, seed=sum(shape))
    net = L.UNet(shape)
    net.set_params(torch.from_numpy(flat(params)).cuda())
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = net.forward(torch.from_numpy(F).cuda(), torch.from_numpy(M).cuda())
    net.backward(torch.from_numpy(target).cuda(), loss=loss)
    g = unflat(net.grads().cpu().numpy().astype(np.float64), L.unet_layers())
    out, loss = out.cpu().numpy(), loss.item()
    # implementation parity: the oracle stores in BF16 where the GPU does
    e_out, e_loss, cos, rel = _compare(f"{shape} bf16-storage oracle", out, loss, g,
                                       oracle_run(params, F, M, target, rnd=bf))
    assert e_out <= 5e-3 and e_loss <= 2e-3, (e_out, e_loss)
    assert cos >= 0.9999 and rel <= 1.5e-2, (cos, rel)
    # precision effect: the plain FP64 oracle
    e_out, e_loss, cos, rel = _compare(f"{shape} fp64 oracle", out, loss, g,
                                       oracle_run(params, F, M, target))
    assert e_out <= 2e-2 and e_loss <= 2e-2, (e_out, e_loss)
    assert cos >= 0.995 and rel <= 0.1, (cos, rel)


LEVEL = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0]   # resolution level of each layer


def _bits(a):
    """BF16 bits (round to nearest even) of a float array, as int16."""
    return to_bf16_rne(np.asarray(a, np.float32)).view(np.int16)


@pytest.mark.parametrize("shape,layers", [((72, 64, 8), tuple(range(15))),
                                          ((80, 96, 112), (1, 12, 13))])
def test_each_layer_matches_oracle_elementwise(L, shape, layers):
    from oracle import unet
    params, _, _, _ = make_case(shape, seed=31)
    net = L.UNet(shape)
    net.set_params(torch.from_numpy(flat(params)).cuda())
    rng = np.random.default_rng(32)
    for l in layers:
        ci, co, relu = unet.LAYERS[l]
        dims = tuple(s >> LEVEL[l] for s in shape)
        n = int(np.prod(dims))
        ldx, ldz = (ci + 3) // 4 * 4, (co + 3) // 4 * 4
        x = bf(rng.uniform(-1.0, 1.0, (n, ci)))
        dz = bf(rng.standard_normal((n, co)) * 0.1)
        xp = np.zeros((n, ldx))
        xp[:, :ci] = x
        dzp = np.zeros((n, ldz))
        dzp[:, :co] = dz
        y, dx, dW, db = net.layer_probe(l, torch.from_numpy(_bits(xp)).cuda(),
                                        torch.from_numpy(_bits(dzp)).cuda())
        torch.cuda.synchronize()
        y = y.cpu().numpy().astype(np.float64)
        dx = bf16_to_f32(dx.cpu().numpy().view(np.uint16)).astype(np.float64)
        dW = dW.cpu().numpy().astype(np.float64)
        db = db.cpu().numpy().astype(np.float64)
        W, b = params[l]
        X = x.reshape(dims + (ci,))
        D = dz.reshape(dims + (co,))
        yr = unet.conv(X, W, b)
        if relu:
            yr = np.maximum(yr, 0.0)
        ya = unet.conv(np.abs(X), np.abs(W), np.abs(b))
        dxr, dWr, dbr = unet.conv_backward(X, W, D)
        dxa, dWa, dba = unet.conv_backward(np.abs(X), np.abs(W), np.abs(D))
        yr, ya = yr.reshape(n, co), ya.reshape(n, co)
        dxr, dxa = dxr.reshape(n, ci), dxa.reshape(n, ci)
        ry = np.abs(y - yr) / np.maximum(ya, 1e-30)
        rx = (np.abs(dx - dxr) - 2.0 ** -8 * np.abs(dxr)) / np.maximum(dxa, 1e-30)
        rw = np.abs(dW - dWr) / np.maximum(dWa, 1e-30)
        rb = np.abs(db - dbr) / np.maximum(dba, 1e-30)
        print(f"[unet layer {l:2d} {dims}] y {ry.max():.2e}  dx {max(rx.max(), 0):.2e}  "
              f"dW {rw.max():.2e}  db {rb.max():.2e}  (of sum |products|)", flush=True)
        assert ry.max() <= 1e-5, (l, ry.max())
        assert rx.max() <= 1.01e-5, (l, rx.max())
        assert rw.max() <= 1e-4, (l, rw.max())
        assert rb.max() <= 1e-4, (l, rb.max())


def test_pooled_input_matches_oracle(L):
    """pool=1: images of twice the network size are average-pooled first."""
    from oracle import unet
    shape = SHAPES[0]
    params, _, _, _ = make_case(shape, seed=3)
    rng = np.random.default_rng(4)
    big = tuple(2 * s for s in shape)
    F = rng.uniform(0, 1, big).astype(np.float32)
    M = rng.uniform(0, 1, big).astype(np.float32)
    x = np.stack([bf(unet.pool(F[..., None].astype(np.float64))[..., 0]),
                  bf(unet.pool(M[..., None].astype(np.float64))[..., 0])], axis=-1)
    out_o = unet.forward(params, x, rnd=bf)[0].transpose(3, 0, 1, 2)
    net = L.UNet(shape)
    net.set_params(torch.from_numpy(flat(params)).cuda())
    out = net.forward(torch.from_numpy(F).cuda(), torch.from_numpy(M).cuda(), pool=True)
    e = rel_l2(out.cpu().numpy(), out_o)
    print(f"\n[unet pooled] out rel-L2 {e:.2e}")
    assert e <= 3e-3, e


def test_accumulate_doubles_gradients_exactly(L):
    shape = SHAPES[0]
    params, F, M, target = make_case(shape, seed=7)
    net = L.UNet(shape)
    net.set_params(torch.from_numpy(flat(params)).cuda())
    Fd, Md, td = (torch.from_numpy(a).cuda() for a in (F, M, target))
    net.forward(Fd, Md)
    net.backward(td)
    g1 = net.grads().cpu()
    net.backward(td, accumulate=True)
    g2 = net.grads().cpu()
    assert torch.equal(g2, g1 * 2)


def test_adam_step_follows_its_definition(L):
    """One step of Adam (bias-corrected first and second moments) applied to
    the gradients the network reports, recomputed in FP64."""
    shape = SHAPES[0]
    params, F, M, target = make_case(shape, seed=9)
    net = L.UNet(shape)
    p0 = flat(params)
    net.set_params(torch.from_numpy(p0).cuda())
    Fd, Md, td = (torch.from_numpy(a).cuda() for a in (F, M, target))
    lr, b1, b2, eps, gs = 1e-3, 0.9, 0.999, 1e-8, 0.5
    m = np.zeros_like(p0, dtype=np.float64)
    v = np.zeros_like(p0, dtype=np.float64)
    p = p0.astype(np.float64)
    for t in (1, 2):
        net.forward(Fd, Md)
        net.backward(td)
        g = net.grads().cpu().numpy().astype(np.float64) * gs
        net.adam(lr, b1, b2, eps, grad_scale=gs)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        got = net.params().cpu().numpy().astype(np.float64)
        err = np.abs(got - p).max()
        assert err <= 1e-6 * lr * 10 + 1e-7, (t, err)


def test_training_reduces_the_loss(L):
    """Adam steps through the HIP backward fit a constant displacement."""
    shape = SHAPES[0]
    params, F, M, _ = make_case(shape, seed=11)
    target = np.empty((3,) + shape, np.float32)
    target[0], target[1], target[2] = 0.05, -0.03, 0.04
    net = L.UNet(shape)
    net.set_params(torch.from_numpy(flat(params)).cuda())
    Fd, Md, td = (torch.from_numpy(a).cuda() for a in (F, M, target))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    for _ in range(60):
        net.forward(Fd, Md)
        net.backward(td, loss=loss)
        hist.append(loss.item())
        net.adam(3e-3)
    print(f"\n[unet train] loss {hist[0]:.4e} -> {hist[-1]:.4e}")
    assert hist[-1] < 0.3 * hist[0]


def test_invalid_arguments_are_rejected(L):
    with pytest.raises(L.LmrError):
        L.UNet((12, 16, 16))
    net = L.UNet((8, 8, 8))
    with pytest.raises(L.LmrError):
        net.backward(torch.zeros((3, 8, 8, 8), device="cuda"))
    with pytest.raises(L.LmrError):
        net.adam(-1.0)
