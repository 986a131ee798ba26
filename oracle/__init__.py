"""FP64 CPU oracle of the factored Levenberg-Marquardt registration step.

TEST INFRASTRUCTURE ONLY.  This package wraps ``oracle.c`` (plain C, double
precision, written from arXiv 2603.19371) for the test-suite, the smoke check
and the CPU-baseline leg of the benchmark.  The product path never imports it,
and it imports nothing from the product package.

Arrays are numpy float64, C-contiguous; volumes are [z][y][x] and fields are
[3][z][y][x] with component 0/1/2 the displacement along x/y/z in voxels.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("window", C.c_int), ("grad_sigma", C.c_double),
                ("cc_eps", C.c_double), ("step_eps", C.c_double),
                ("compositive", C.c_int), ("lambda_inc", C.c_double),
                ("lambda_dec", C.c_double), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("tau", C.c_double),
                ("max_retries", C.c_int), ("tile", C.c_int), ("similarity", C.c_int),
                ("mi_bins", C.c_int)]


class _Adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


class _State(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("loss", C.c_double),
                ("loss_prev", C.c_double), ("cand_loss", C.c_double),
                ("n_hist", C.c_int), ("retries", C.c_int),
                ("accepted", C.c_int), ("stalled", C.c_int)]


_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_LIB_PATH)
        i, d, l = C.c_int, C.c_double, C.c_long
        sig = {
            "orc_set_threads": (None, [i]),
            "orc_get_threads": (i, []),
            "orc_sample": (d, [_D, i, i, i, d, d, d, _D]),
            "orc_warp": (None, [_D, _D, i, i, i, _D, _D]),
            "orc_box_sum": (None, [_D, i, i, i, i, _D]),
            "orc_window_stats": (None, [_D, _D, i, i, i, i, i, i, i, _D]),
            "orc_lncc": (d, [_D, _D, i, i, i, i, d, _D]),
            "orc_dsumcc_dmw": (None, [_D, _D, i, i, i, i, d, _D]),
            "orc_loss_grad": (d, [_D, _D, _D, i, i, i, i, d, _D]),
            "orc_grad_at": (None, [_D, _D, _D, i, i, i, i, d, i, i, i, _D]),
            "orc_gauss": (None, [_D, i, i, i, i, d, _D]),
            "orc_cc_at": (d, [_D, _D, _D, i, i, i, i, d, i, i, i]),
            "orc_gauss_at": (None, [_D, i, i, i, i, d, i, i, i, _D]),
            "orc_gauss_radius": (i, [d]),
            "orc_closed_form": (None, [_D, i, i, i, d, d, _D]),
            "orc_explicit_solve": (None, [_D, d, d, _D]),
            "orc_integrate": (None, [_D, _D, i, i, i, d, i, _D]),
            "orc_tile_hessian": (None, [_D, i, i, i, i, _D]),
            "orc_mse_loss_grad": (d, [_D, _D, _D, i, i, i, _D]),
            "orc_demons_step": (None, [_D, _D, _D, i, i, i, d, _D]),
            "orc_mi_loss_grad": (d, [_D, _D, _D, i, i, i, i, _D, _D]),
            "orc_bspline3": (d, [d]),
            "orc_dbspline3": (d, [d]),
            "orc_tile_step": (None, [_D, i, i, i, i, d, d, _D]),
            "orc_adam_direction": (None, [_D, _D, _D, l, l, C.POINTER(_Adam), _D]),
            "orc_adam_iter": (None, [C.POINTER(_Params), C.POINTER(_Adam), _D, _D, _D,
                                     _D, _D, _D, i, i, i, l, C.POINTER(_State)]),
            "orc_decide": (i, [C.POINTER(_Params), C.POINTER(_State), d, i]),
            "orc_begin": (None, [C.POINTER(_Params), _D, _D, _D, i, i, i, d,
                                 C.POINTER(_State), _D]),
            "orc_attempt": (i, [C.POINTER(_Params), _D, _D, _D, _D, i, i, i,
                                C.POINTER(_State), i]),
            "orc_avgpool": (None, [_D, i, i, i, i, _D]),
            "orc_upsample_field": (None, [_D, i, i, i, _D, i, i, i]),
            "orc_folded_count": (l, [_D, i, i, i, _D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


@dataclass
class Params:
    """Hyper-parameters; defaults are the synthetic-phantom setting
    (lambda x2 on a bad step, x0.5 on a good one, rejection at tau = 0)."""
    window: int = 5
    grad_sigma: float = 1.0
    cc_eps: float = 1e-5
    step_eps: float = 1.0
    compositive: int = 1
    lambda_inc: float = 2.0
    lambda_dec: float = 0.5
    lambda_min: float = 1e-12
    lambda_max: float = 1e6
    tau: float = 0.0
    max_retries: int = 10
    tile: int = 1
    similarity: int = 0       # 0 LNCC, 1 squared error, 2 Demons step, 3 MI
    mi_bins: int = 32

    def c(self) -> _Params:
        return _Params(self.window, self.grad_sigma, self.cc_eps, self.step_eps,
                       self.compositive, self.lambda_inc, self.lambda_dec,
                       self.lambda_min, self.lambda_max, self.tau,
                       self.max_retries, self.tile, self.similarity, self.mi_bins)


@dataclass
class AdamParams:
    """The Adam comparator's hyper-parameters (beta1, beta2 as in Sec. 3)."""
    lr: float = 0.1
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self) -> _Adam:
        return _Adam(self.lr, self.beta1, self.beta2, self.eps)


@dataclass
class State:
    lambda_: float = 1.0
    loss: float = 0.0
    loss_prev: float = 0.0
    cand_loss: float = 0.0
    n_hist: int = 0
    retries: int = 0
    accepted: int = 0
    stalled: int = 0

    def c(self) -> _State:
        return _State(self.lambda_, self.loss, self.loss_prev, self.cand_loss,
                      self.n_hist, self.retries, self.accepted, self.stalled)

    @staticmethod
    def from_c(s: _State) -> "State":
        return State(s.lambda_, s.loss, s.loss_prev, s.cand_loss, s.n_hist,
                     s.retries, s.accepted, s.stalled)


# ---------------------------------------------------------------- O1 warp
def sample(V, p, with_grad=False):
    V = _f64(V)
    nz, ny, nx = V.shape
    d = np.zeros(3)
    v = lib().orc_sample(_p(V), nz, ny, nx, float(p[0]), float(p[1]),
                         float(p[2]), _p(d))
    return (v, d) if with_grad else v


def warp(M, u, with_grad=False):
    M, u = _f64(M), _f64(u)
    nz, ny, nx = M.shape
    Mw = np.empty_like(M)
    dMw = np.empty((3,) + M.shape) if with_grad else None
    lib().orc_warp(_p(M), _p(u), nz, ny, nx, _p(Mw),
                   _p(dMw) if with_grad else None)
    return (Mw, dMw) if with_grad else Mw


# ---------------------------------------------------------------- O2/O3 LNCC
def box_sum(a, w):
    a = _f64(a)
    out = np.empty_like(a)
    lib().orc_box_sum(_p(a), *a.shape, int(w), _p(out))
    return out


def window_stats(F, Mw, w, x, y, z):
    F, Mw = _f64(F), _f64(Mw)
    st = np.zeros(5)
    lib().orc_window_stats(_p(F), _p(Mw), *F.shape, int(w), x, y, z, _p(st))
    return st


def lncc(F, Mw, w, eps, with_map=False):
    F, Mw = _f64(F), _f64(Mw)
    cc = np.empty_like(F) if with_map else None
    m = lib().orc_lncc(_p(F), _p(Mw), *F.shape, int(w), float(eps),
                       _p(cc) if with_map else None)
    return (m, cc) if with_map else m


def dsumcc_dmw(F, Mw, w, eps):
    F, Mw = _f64(F), _f64(Mw)
    out = np.empty_like(F)
    lib().orc_dsumcc_dmw(_p(F), _p(Mw), *F.shape, int(w), float(eps), _p(out))
    return out


def loss_grad(F, M, u, w, eps, with_grad=True):
    """Returns (L, g_raw) with L = -mean cc and g_raw = N dL/du."""
    F, M, u = _f64(F), _f64(M), _f64(u)
    g = np.empty((3,) + F.shape) if with_grad else None
    L = lib().orc_loss_grad(_p(F), _p(M), _p(u), *F.shape, int(w), float(eps),
                            _p(g) if with_grad else None)
    return (L, g) if with_grad else L


def mse_loss_grad(F, M, u, with_grad=True):
    """Returns (L, g_raw) with L = mean (F - M o (Id+u))^2 and g_raw = N dr/du,
    r = sqrt(L)."""
    F, M, u = _f64(F), _f64(M), _f64(u)
    g = np.empty((3,) + F.shape) if with_grad else None
    L = lib().orc_mse_loss_grad(_p(F), _p(M), _p(u), *F.shape, _p(g) if with_grad else None)
    return (L, g) if with_grad else L


def mi_loss_grad(F, M, u, bins=32, with_grad=True, with_hist=False):
    """Returns (L, g_raw[, hist]) with L = -MI (bits) of F and M o (Id + u)
    and g_raw = N dr/du, r = log2(bins) - MI."""
    F, M, u = _f64(F), _f64(M), _f64(u)
    g = np.empty((3,) + F.shape) if with_grad else None
    h = np.empty((bins, bins)) if with_hist else None
    L = lib().orc_mi_loss_grad(_p(F), _p(M), _p(u), *F.shape, int(bins),
                               _p(g) if with_grad else None, _p(h) if with_hist else None)
    out = (L, g) if with_grad else (L,)
    return out + ((h,) if with_hist else ()) if (with_hist or with_grad) else L


def bspline3(t):
    return lib().orc_bspline3(float(t))


def dbspline3(t):
    return lib().orc_dbspline3(float(t))


def demons_step(F, M, u, lam):
    F, M, u = _f64(F), _f64(M), _f64(u)
    du = np.empty((3,) + F.shape)
    lib().orc_demons_step(_p(F), _p(M), _p(u), *F.shape, float(lam), _p(du))
    return du


def grad_at(F, M, u, w, eps, x, y, z):
    F, M, u = _f64(F), _f64(M), _f64(u)
    g = np.zeros(3)
    lib().orc_grad_at(_p(F), _p(M), _p(u), *F.shape, int(w), float(eps),
                      int(x), int(y), int(z), _p(g))
    return g


def cc_at(F, M, u, w, eps, x, y, z):
    F, M, u = _f64(F), _f64(M), _f64(u)
    return lib().orc_cc_at(_p(F), _p(M), _p(u), *F.shape, int(w), float(eps),
                           int(x), int(y), int(z))


# ---------------------------------------------------------------- O4..O6
def gauss_radius(sigma):
    return int(lib().orc_gauss_radius(float(sigma)))


def gauss(g, sigma):
    g = _f64(g)
    nc = 1 if g.ndim == 3 else g.shape[0]
    shp = g.shape[-3:]
    out = np.empty_like(g)
    lib().orc_gauss(_p(g), nc, *shp, float(sigma), _p(out))
    return out


def gauss_at(g, sigma, x, y, z):
    g = _f64(g)
    nc = 1 if g.ndim == 3 else g.shape[0]
    out = np.zeros(nc)
    lib().orc_gauss_at(_p(g), nc, *g.shape[-3:], float(sigma), int(x), int(y),
                       int(z), _p(out))
    return out


def closed_form(gs, r, lam):
    gs = _f64(gs)
    out = np.empty_like(gs)
    lib().orc_closed_form(_p(gs), *gs.shape[1:], float(r), float(lam), _p(out))
    return out


def explicit_solve(g, r, lam):
    g = _f64(g)
    d = np.zeros(3)
    lib().orc_explicit_solve(_p(g), float(r), float(lam), _p(d))
    return d


def tile_hessian(gs, k):
    """Pooled Hessian of tile side k (eq. tilen): [tz][ty][tx][6] with entries
    (xx, yy, zz, xy, xz, yz), the mean of gs gs^T over each tile."""
    gs = _f64(gs)
    nz, ny, nx = gs.shape[1:]
    t = tuple((n + k - 1) // k for n in (nz, ny, nx))
    H = np.empty(t + (6,))
    lib().orc_tile_hessian(_p(gs), nz, ny, nx, int(k), _p(H))
    return H


def tile_step(gs, k, r, lam):
    gs = _f64(gs)
    out = np.empty_like(gs)
    lib().orc_tile_step(_p(gs), *gs.shape[1:], int(k), float(r), float(lam), _p(out))
    return out


def adam_direction(gs, m, v, t, ap: AdamParams):
    """One bias-corrected Adam direction at step t; m and v (float64,
    C-contiguous) are updated in place."""
    gs = _f64(gs)
    assert m.dtype == np.float64 and v.dtype == np.float64
    du = np.empty_like(gs)
    a = ap.c()
    lib().orc_adam_direction(_p(gs), _p(m), _p(v), gs.size, int(t), C.byref(a), _p(du))
    return du


def integrate(u, v, eps=1.0, compositive=1):
    u, v = _f64(u), _f64(v)
    out = np.empty_like(u)
    lib().orc_integrate(_p(u), _p(v), *u.shape[1:], float(eps),
                        int(compositive), _p(out))
    return out


# ---------------------------------------------------------------- O7 decision
def decide(params: Params, state: State, cand_loss: float, force: int = -1):
    cp, cs = params.c(), state.c()
    acc = lib().orc_decide(C.byref(cp), C.byref(cs), float(cand_loss), int(force))
    return bool(acc), State.from_c(cs)


# ---------------------------------------------------------------- one pair
@dataclass
class Pair:
    """An LM registration of one image pair, advanced attempt by attempt."""
    F: np.ndarray
    M: np.ndarray
    params: Params
    u: np.ndarray = None
    gs: np.ndarray = None
    state: State = field(default_factory=State)

    def begin(self, u0=None, lambda0=1.0):
        self.F, self.M = _f64(self.F), _f64(self.M)
        self.u = _f64(np.zeros((3,) + self.F.shape) if u0 is None else u0).copy()
        self.gs = np.empty_like(self.u)
        cp, cs = self.params.c(), _State()
        lib().orc_begin(C.byref(cp), _p(self.F), _p(self.M), _p(self.u),
                        *self.F.shape, float(lambda0), C.byref(cs), _p(self.gs))
        self.state = State.from_c(cs)
        return self

    def attempt(self, force: int = -1) -> bool:
        cp, cs = self.params.c(), self.state.c()
        acc = lib().orc_attempt(C.byref(cp), _p(self.F), _p(self.M), _p(self.u),
                                _p(self.gs), *self.F.shape, C.byref(cs),
                                int(force))
        self.state = State.from_c(cs)
        return bool(acc)


@dataclass
class AdamPair:
    """The Adam comparator on one image pair: same loss, gradient, smoothing
    and integration as the LM pair; the step comes from Adam's moments of
    the smoothed gradient and is always kept."""
    F: np.ndarray
    M: np.ndarray
    params: Params
    adam: AdamParams = field(default_factory=AdamParams)
    u: np.ndarray = None
    gs: np.ndarray = None
    m: np.ndarray = None
    v: np.ndarray = None
    t: int = 0
    state: State = field(default_factory=State)

    def begin(self, u0=None):
        pr = Pair(self.F, self.M, self.params).begin(u0, lambda0=1.0)
        self.F, self.M, self.u, self.gs, self.state = pr.F, pr.M, pr.u, pr.gs, pr.state
        self.m = np.zeros_like(self.u)
        self.v = np.zeros_like(self.u)
        self.t = 0
        return self

    def iterate(self):
        self.t += 1
        cp, ca, cs = self.params.c(), self.adam.c(), self.state.c()
        lib().orc_adam_iter(C.byref(cp), C.byref(ca), _p(self.F), _p(self.M), _p(self.u),
                            _p(self.gs), _p(self.m), _p(self.v), *self.F.shape, self.t,
                            C.byref(cs))
        self.state = State.from_c(cs)
        return self.state.loss


# ---------------------------------------------------------------- O8, O9
def avgpool(a, f):
    a = _f64(a)
    nz, ny, nx = a.shape
    out = np.empty((nz // f, ny // f, nx // f))
    lib().orc_avgpool(_p(a), nz, ny, nx, int(f), _p(out))
    return out


def upsample_field(uc, fine_shape):
    uc = _f64(uc)
    uf = np.empty((3,) + tuple(fine_shape))
    lib().orc_upsample_field(_p(uc), *uc.shape[1:], _p(uf), *fine_shape)
    return uf


def folded_count(u, with_det=False):
    u = _f64(u)
    det = np.empty(u.shape[1:]) if with_det else None
    n = lib().orc_folded_count(_p(u), *u.shape[1:], _p(det) if with_det else None)
    return (int(n), det) if with_det else int(n)


def register(F, M, params: Params, levels, lambda0=1.0, forces=None):
    """Coarse-to-fine registration (Sec. 2.1).  ``levels`` is a list of
    (pool_factor, attempts) from coarse to fine; consecutive factors differ by
    two.  Each level restarts lambda and the loss history (a reading: losses
    at different resolutions are not comparable).  Returns the final field and
    the per-attempt decisions of every level."""
    F, M = _f64(F), _f64(M)
    u = None
    decisions = []
    prev_shape = None
    for li, (f, iters) in enumerate(levels):
        Fl = F if f == 1 else avgpool(F, f)
        Ml = M if f == 1 else avgpool(M, f)
        if u is None:
            u0 = np.zeros((3,) + Fl.shape)
        else:
            assert tuple(s * 2 for s in prev_shape) == Fl.shape
            u0 = upsample_field(u, Fl.shape)
        pr = Pair(Fl, Ml, params).begin(u0, lambda0)
        dl = []
        for t in range(iters):
            fc = -1 if forces is None else forces[li][t]
            dl.append(pr.attempt(fc))
        decisions.append(dl)
        u = pr.u
        prev_shape = Fl.shape
    return u, decisions
