"""FP64 oracle of the learned initializer's network (a small 3D U-Net).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in double
precision; each convolution is the sum over its 27 taps of a matrix product
(a library primitive), written out without blocking or fusion.  Layouts are
channels-last: activations [z][y][x][c], weights [27][cin][cout] with tap
t = 9 (dz+1) + 3 (dy+1) + (dx+1).

Network (four levels, channels 16/32/64/128, 3x3x3 convolutions with zero
padding 1, ReLU after every convolution but the last):
  e1 = R(C(R(C(x, 2->16)), 16->16))                    at S1
  e2 = R(C(R(C(P(e1), 16->32)), 32->32))               at S1/2
  e3 = R(C(R(C(P(e2), 32->64)), 64->64))               at S1/4
  e4 = R(C(R(C(P(e3), 64->128)), 128->128))            at S1/8
  f3 = R(C(R(C([U(e4), e3], 192->64)), 64->64))        at S1/4
  f2 = R(C(R(C([U(f3), e2], 96->32)), 32->32))         at S1/2
  f1 = R(C(R(C([U(f2), e1], 48->16)), 16->16))         at S1
  out = C(f1, 16->3)                                    at S1
with P the 2x2x2 average pooling, U the x2 nearest-neighbour upsampling and
[a, b] channel concatenation.  The output is a displacement field (x, y, z
components, in voxels of S1).
"""
from __future__ import annotations

import numpy as np

# (cin, cout, relu) of the 15 convolutions, in evaluation order
LAYERS = [(2, 16, True), (16, 16, True), (16, 32, True), (32, 32, True),
          (32, 64, True), (64, 64, True), (64, 128, True), (128, 128, True),
          (192, 64, True), (64, 64, True), (96, 32, True), (32, 32, True),
          (48, 16, True), (16, 16, True), (16, 3, False)]

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def init_params(seed=0, scale=1.0, layers=LAYERS):
    """He-style normal initialisation (std sqrt(2 / (27 cin))), zero bias;
    the last layer is scaled down by 0.1 so the initial field is small."""
    rng = np.random.default_rng(seed)
    params = []
    for li, (ci, co, relu) in enumerate(layers):
        std = np.sqrt(2.0 / (27 * ci)) * scale * (1.0 if relu else 0.1)
        params.append((rng.standard_normal((27, ci, co)) * std, np.zeros(co)))
    return params


def _shift(x, dz, dy, dx):
    """out[p] = x[p + d] with zeros outside."""
    out = np.zeros_like(x)
    Z, Y, X = x.shape[:3]
    zs, ze = max(0, -dz), Z - max(0, dz)
    ys, ye = max(0, -dy), Y - max(0, dy)
    xs, xe = max(0, -dx), X - max(0, dx)
    out[zs:ze, ys:ye, xs:xe] = x[zs + dz:ze + dz, ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv(x, w, b):
    """y[p, o] = b[o] + sum_t sum_i x[p + d_t, i] w[t, i, o]  (zero padding)."""
    y = np.broadcast_to(b, x.shape[:3] + (w.shape[2],)).astype(np.float64).copy()
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += _shift(x, dz, dy, dx) @ w[t]
    return y


def conv_backward(x, w, dy):
    """Gradients of conv with respect to x, w and b."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dz, dy_, dx_) in enumerate(TAPS):
        xs = _shift(x, dz, dy_, dx_)
        dw[t] = xs.reshape(-1, x.shape[3]).T @ dy.reshape(-1, dy.shape[3])
        dx += _shift(dy @ w[t].T, -dz, -dy_, -dx_)
    db = dy.reshape(-1, dy.shape[3]).sum(0)
    return dx, dw, db


def pool(x):
    Z, Y, X, C = x.shape
    return x.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).mean((1, 3, 5))


def pool_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_backward(dy):
    Z, Y, X, C = dy.shape
    return dy.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).sum((1, 3, 5))


def _keep(a):
    return a


def forward(params, x, rnd=None):
    """Returns the output and the list of cached activations.

    rnd (optional) is applied to every activation the network stores between
    layers (each convolution output but the last, each pooling output), to
    model a reduced-precision storage format; the arithmetic itself stays in
    FP64.  Default: no rounding."""
    r = rnd or _keep
    acts = {}

    def c(i, a):
        y = conv(a, *params[i])
        if not LAYERS[i][2]:
            return y                       # the head output is kept as computed
        return r(np.maximum(y, 0.0))

    acts["x"] = x
    acts["e1a"] = c(0, x)
    acts["e1"] = c(1, acts["e1a"])
    acts["p1"] = r(pool(acts["e1"]))
    acts["e2a"] = c(2, acts["p1"])
    acts["e2"] = c(3, acts["e2a"])
    acts["p2"] = r(pool(acts["e2"]))
    acts["e3a"] = c(4, acts["p2"])
    acts["e3"] = c(5, acts["e3a"])
    acts["p3"] = r(pool(acts["e3"]))
    acts["e4a"] = c(6, acts["p3"])
    acts["e4"] = c(7, acts["e4a"])
    acts["c3"] = np.concatenate([up(acts["e4"]), acts["e3"]], axis=3)
    acts["f3a"] = c(8, acts["c3"])
    acts["f3"] = c(9, acts["f3a"])
    acts["c2"] = np.concatenate([up(acts["f3"]), acts["e2"]], axis=3)
    acts["f2a"] = c(10, acts["c2"])
    acts["f2"] = c(11, acts["f2a"])
    acts["c1"] = np.concatenate([up(acts["f2"]), acts["e1"]], axis=3)
    acts["f1a"] = c(12, acts["c1"])
    acts["f1"] = c(13, acts["f1a"])
    acts["out"] = c(14, acts["f1"])
    return acts["out"], acts


# (layer, input activation, output activation)
_GRAPH = [(0, "x", "e1a"), (1, "e1a", "e1"), (2, "p1", "e2a"), (3, "e2a", "e2"),
          (4, "p2", "e3a"), (5, "e3a", "e3"), (6, "p3", "e4a"), (7, "e4a", "e4"),
          (8, "c3", "f3a"), (9, "f3a", "f3"), (10, "c2", "f2a"), (11, "f2a", "f2"),
          (12, "c1", "f1a"), (13, "f1a", "f1"), (14, "f1", "out")]


def backward(params, acts, dout, rnd=None):
    """Gradients of every parameter given d(loss)/d(out).

    rnd (optional) is applied to every activation gradient as it is stored
    (each input gradient of a convolution, each upsampling gradient, each sum
    of a skip gradient and a pooling gradient); parameter gradients are not
    rounded.  Default: no rounding."""
    r = rnd or _keep
    grads = [None] * len(LAYERS)
    g = {"out": dout}

    def add(name, v):
        g[name] = r(g[name] + v) if name in g else r(v)

    def layer_back(i):
        _, src, dst = _GRAPH[i]
        d = g.pop(dst)
        if LAYERS[i][2]:
            d = d * (acts[dst] > 0.0)          # ReLU
        dx, dw, db = conv_backward(acts[src], params[i][0], d)
        grads[i] = (dw, db)
        add(src, dx)

    def split(cname, upname, skip, cu):
        d = g.pop(cname)
        add(upname, up_backward(d[..., :cu]))
        add(skip, d[..., cu:])

    for i in (14, 13, 12):
        layer_back(i)
    split("c1", "f2", "e1", 32)
    for i in (11, 10):
        layer_back(i)
    split("c2", "f3", "e2", 64)
    for i in (9, 8):
        layer_back(i)
    split("c3", "e4", "e3", 128)
    for i in (7, 6):
        layer_back(i)
    add("e3", pool_backward(g.pop("p3")))
    for i in (5, 4):
        layer_back(i)
    add("e2", pool_backward(g.pop("p2")))
    for i in (3, 2):
        layer_back(i)
    add("e1", pool_backward(g.pop("p1")))
    for i in (1, 0):
        layer_back(i)
    return grads, g.get("x")


def mse(out, target):
    """Mean squared error over every element and its gradient."""
    diff = out - target
    return float((diff ** 2).mean()), 2.0 * diff / diff.size
