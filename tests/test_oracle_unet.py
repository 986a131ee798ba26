"""Pins of the U-Net oracle (oracle/unet.py): each operation against torch's
CPU FP64 primitives and the whole-network gradient against finite
differences."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _rng(s):
    return np.random.default_rng(s)


def _to_torch_w(w):
    # [27][cin][cout] -> [cout][cin][3][3][3]
    return torch.from_numpy(w.reshape(3, 3, 3, w.shape[1], w.shape[2]).transpose(4, 3, 0, 1, 2).copy())


def test_conv_matches_torch_conv3d():
    from oracle import unet
    x = _rng(1).standard_normal((5, 6, 7, 3))
    w = _rng(2).standard_normal((27, 3, 4))
    b = _rng(3).standard_normal(4)
    y = unet.conv(x, w, b)
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2).copy())[None]
    ref = F.conv3d(xt, _to_torch_w(w), torch.from_numpy(b), padding=1)[0].numpy()
    np.testing.assert_allclose(y, ref.transpose(1, 2, 3, 0), rtol=1e-12, atol=1e-12)


def test_conv_backward_matches_autograd():
    from oracle import unet
    x = _rng(4).standard_normal((4, 5, 6, 3))
    w = _rng(5).standard_normal((27, 3, 2))
    b = _rng(6).standard_normal(2)
    dy = _rng(7).standard_normal((4, 5, 6, 2))
    dx, dw, db = unet.conv_backward(x, w, dy)
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2).copy())[None].requires_grad_()
    wt = _to_torch_w(w).requires_grad_()
    bt = torch.from_numpy(b).requires_grad_()
    yt = F.conv3d(xt, wt, bt, padding=1)
    yt.backward(torch.from_numpy(dy.transpose(3, 0, 1, 2).copy())[None])
    np.testing.assert_allclose(dx, xt.grad[0].numpy().transpose(1, 2, 3, 0), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dw, wt.grad.numpy().transpose(2, 3, 4, 1, 0).reshape(27, 3, 2),
                               rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12)


def test_pool_and_upsample_match_torch():
    from oracle import unet
    x = _rng(8).standard_normal((4, 6, 8, 3))
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2).copy())[None]
    np.testing.assert_allclose(unet.pool(x),
                               F.avg_pool3d(xt, 2)[0].numpy().transpose(1, 2, 3, 0), rtol=1e-13)
    np.testing.assert_allclose(unet.up(x), F.interpolate(xt, scale_factor=2, mode="nearest")
                               [0].numpy().transpose(1, 2, 3, 0), rtol=0, atol=0)
    d = _rng(9).standard_normal((8, 12, 16, 3))
    # adjoint identities <P x, d'> = <x, P^T d'>, <U x, d> = <x, U^T d>
    dp = _rng(10).standard_normal((2, 3, 4, 3))
    assert abs((unet.pool(x) * dp).sum() - (x * unet.pool_backward(dp)).sum()) < 1e-11
    assert abs((unet.up(x) * d).sum() - (x * unet.up_backward(d)).sum()) < 1e-11


def test_network_gradient_matches_finite_differences():
    from oracle import unet
    params = unet.init_params(seed=1)
    x = _rng(11).uniform(0, 1, (8, 8, 8, 2))
    target = _rng(12).standard_normal((8, 8, 8, 3)) * 0.1
    out, acts = unet.forward(params, x)
    L, dout = unet.mse(out, target)
    grads, _ = unet.backward(params, acts, dout)
    rng = _rng(13)
    h = 1e-6
    worst = 0.0
    for li in (0, 3, 7, 8, 12, 14):
        w = params[li][0]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            old = w[idx]
            w[idx] = old + h
            Lp = unet.mse(unet.forward(params, x)[0], target)[0]
            w[idx] = old - h
            Lm = unet.mse(unet.forward(params, x)[0], target)[0]
            w[idx] = old
            fd = (Lp - Lm) / (2 * h)
            g = grads[li][0][idx]
            worst = max(worst, abs(fd - g) / max(1e-9, abs(g), abs(fd)))
        b = params[li][1]
        j = int(rng.integers(0, b.shape[0]))
        old = b[j]
        b[j] = old + h
        Lp = unet.mse(unet.forward(params, x)[0], target)[0]
        b[j] = old - h
        Lm = unet.mse(unet.forward(params, x)[0], target)[0]
        b[j] = old
        g = grads[li][1][j]
        fd = (Lp - Lm) / (2 * h)
        worst = max(worst, abs(fd - g) / max(1e-9, abs(g), abs(fd)))
    assert worst < 1e-5, worst


def test_storage_rounding_mode():
    """rnd is applied to stored tensors only: the identity reproduces the
    default bit for bit, and BF16 storage moves the result by the size that
    rounding 8-bit significands implies, not more."""
    from oracle import unet
    from paper_2603_19371_amd.phantoms import bf16_to_f32, to_bf16_rne

    def bf(a):
        return bf16_to_f32(to_bf16_rne(np.asarray(a, np.float32))).astype(np.float64)

    params = unet.init_params(seed=2)
    x = bf(_rng(14).uniform(0, 1, (8, 8, 16, 2)))
    t = _rng(15).standard_normal((8, 8, 16, 3)) * 0.05
    out0, acts0 = unet.forward(params, x)
    out1, acts1 = unet.forward(params, x, rnd=lambda a: a)
    assert np.array_equal(out0, out1)
    g0, _ = unet.backward(params, acts0, unet.mse(out0, t)[1])
    g1, _ = unet.backward(params, acts1, unet.mse(out1, t)[1], rnd=lambda a: a)
    assert all(np.array_equal(a[0], b[0]) for a, b in zip(g0, g1))
    outb, actsb = unet.forward(params, x, rnd=bf)
    for k in ("e1a", "p1", "e4", "f1"):
        assert np.array_equal(actsb[k], bf(actsb[k])), k
    rel = np.linalg.norm(outb - out0) / np.linalg.norm(out0)
    assert 1e-5 < rel < 3e-2, rel
