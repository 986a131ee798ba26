"""ctypes binding of liblmreg (include/lmreg.h).

Argument marshalling only: every step of the registration runs in the HIP
kernels of liblmreg.so.  torch provides device memory and streams.  Before a
call reaches the library, the binding checks on the host that every tensor is
a contiguous CUDA tensor of the dtype and shape the call expects, so that no
kernel is launched on a buffer smaller than its grid assumes.

There is no fallback: if liblmreg.so is missing or fails to load, importing
this module raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmreg.so")

LMR_F32, LMR_BF16 = 0, 1
LMR_ACC_F64, LMR_ACC_F32C = 0, 1
_STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory",
           3: "HIP runtime error", 4: "call out of order", 5: "pair is frozen",
           6: "batched launch not co-resident"}


class LmrError(RuntimeError):
    pass


# lmr_stencil_form
LMR_EBUSY = 6
LMR_STENCIL_AUTO, LMR_STENCIL_MARCH, LMR_STENCIL_CUBE = 0, 1, 2


class Params(C.Structure):
    """Mirror of lmr_params."""
    _fields_ = [("window", C.c_int), ("grad_sigma", C.c_double),
                ("cc_eps", C.c_double), ("step_eps", C.c_double),
                ("compositive", C.c_int), ("accum", C.c_int),
                ("lambda_inc", C.c_double), ("lambda_dec", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double),
                ("tau", C.c_double), ("max_retries", C.c_int),
                ("tile", C.c_int), ("optimizer", C.c_int), ("adam_lr", C.c_double),
                ("adam_beta1", C.c_double), ("adam_beta2", C.c_double),
                ("adam_eps", C.c_double), ("similarity", C.c_int), ("mi_bins", C.c_int),
                ("stencil", C.c_int)]

    @staticmethod
    def make(**kw) -> "Params":
        p = Params()
        lib().lmr_default_params(C.byref(p))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        return p

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PairState(C.Structure):
    """Mirror of lmr_pair_state."""
    _fields_ = [("lambda_", C.c_double), ("loss", C.c_double),
                ("loss_prev", C.c_double), ("cand_loss", C.c_double),
                ("n_hist", C.c_int32), ("retries", C.c_int32),
                ("accepted", C.c_int32), ("stalled", C.c_int32),
                ("attempts", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelTime(C.Structure):
    """Mirror of lmr_kernel_time."""
    _fields_ = [("count", C.c_int64), ("total_ms", C.c_double),
                ("min_ms", C.c_double), ("max_ms", C.c_double)]


KERNELS = ("update", "lncc_fwd", "decide", "lncc_bwd", "smooth")

_lib = None
_V, _I, _D, _LL = C.c_void_p, C.c_int, C.c_double, C.c_longlong


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LmrError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2603_19371_amd.build`")
        L = C.CDLL(LIB_PATH)
        sig = {
            "lmr_strerror": (C.c_char_p, [_I]),
            "lmr_last_error": (C.c_char_p, []),
            "lmr_default_params": (None, [C.POINTER(Params)]),
            "lmr_create": (_I, [C.POINTER(_V), _I, _I, _I, _I, C.POINTER(Params), _V]),
            "lmr_destroy": (None, [_V]),
            "lmr_begin": (_I, [_V, _V, _V, _V, _D]),
            "lmr_step": (_I, [_V, _V, _V, _I]),
            "lmr_step_forced": (_I, [_V, _V, _V, C.POINTER(_I), _I]),
            "lmr_get_field": (_I, [_V, _V]),
            "lmr_workspace_bytes": (_I, [_V, C.POINTER(C.c_size_t)]),
            "lmr_get_grad": (_I, [_V, _V]),
            "lmr_get_state": (_I, [_V, C.POINTER(PairState)]),
            "lmr_loss_grad": (_I, [_V, _V, _V, _V, C.POINTER(_D), _V, _V, _V]),
            "lmr_update": (_I, [_V, _V, _V, _D, _D, _V]),
            "lmr_warp": (_I, [_V, _I, _V, _I, _I, _I, _V, _V, _V]),
            "lmr_decide_probe": (_I, [_V, C.POINTER(PairState), _D, _I,
                                      C.POINTER(PairState)]),
            "lmr_smooth": (_I, [_V, _V, _V]),
            "lmr_set_state": (_I, [_V, C.POINTER(PairState)]),
            "lmr_folded_count": (_I, [_V, _V, C.POINTER(_LL), _V]),
            "lmr_kernel_name": (C.c_char_p, [_I]),
            "lmr_profile_start": (_I, [_V, _I, _I]),
            "lmr_profile_stop": (_I, [_V, C.POINTER(KernelTime)]),
            "lmr_avgpool": (_I, [_V, _I, _I, _I, _I, _I, _V, _V]),
            "lmr_upsample_field": (_I, [_V, _I, _I, _I, _V, _V]),
            "lmr_pyramid_create": (_I, [C.POINTER(_V), _I, _I, _I, _I,
                                        C.POINTER(Params), _I, C.POINTER(_I), _V]),
            "lmr_pyramid_run": (_I, [_V, _V, _V, C.POINTER(_I), _D, C.POINTER(_I),
                                     _V]),
            "lmr_pyramid_level": (_V, [_V, _I]),
            "lmr_pyramid_destroy": (None, [_V]),
            "lmr_pyramid_use_graphs": (_I, [_V, _I]),
            "lmr_batch_create": (_I, [C.POINTER(_V), _I, C.POINTER(_I), _I,
                                      C.POINTER(Params)]),
            "lmr_batch_begin": (_I, [_V, C.POINTER(_V), C.POINTER(_V),
                                     C.POINTER(_D)]),
            "lmr_batch_step": (_I, [_V, _I, _I]),
            "lmr_batch_sync": (_I, [_V]),
            "lmr_force_decision": (_I, [_V, _I]),
            "lmr_batch_test_residency": (_I, [_V, _I]),
            "lmr_batch_pair": (_V, [_V, _I]),
            "lmr_batch_set_config": (_I, [_V, _I, _I, _I]),
            "lmr_batch_get_config": (_I, [_V, C.POINTER(_I)]),
            "lmr_batch_tune": (_I, [_V, C.POINTER(_V), C.POINTER(_V), C.c_char_p,
                                    _I, C.POINTER(_D)]),
            "lmr_batch_destroy": (None, [_V]),
            "lmr_unet_param_count": (C.c_int64, []),
            "lmr_unet_layer_info": (_I, [_I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I),
                                         C.POINTER(C.c_int64)]),
            "lmr_unet_create": (_I, [C.POINTER(_V), _I, _I, _I, _V]),
            "lmr_unet_destroy": (None, [_V]),
            "lmr_unet_set_params": (_I, [_V, _V]),
            "lmr_unet_get_params": (_I, [_V, _V]),
            "lmr_unet_get_grads": (_I, [_V, _V]),
            "lmr_unet_forward": (_I, [_V, _V, _V, _I, _I, _V]),
            "lmr_unet_backward": (_I, [_V, _V, _D, _I, _V]),
            "lmr_unet_adam": (_I, [_V, _D, _D, _D, _D, _D]),
            "lmr_unet_layer_probe": (_I, [_V, _I, _V, _I, _V, _I, _V, _I, _V, _I, _V,
                                          _V]),
            "lmr_loss_grad_noalloc": (_I, [_V, _V, _I, _V, _I, _I, _I, C.POINTER(Params),
                                           _V, _V, _V, _V, _V]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names this binding requires the library to export."""
    lib()
    return ["lmr_strerror", "lmr_last_error", "lmr_default_params", "lmr_create",
            "lmr_destroy", "lmr_begin", "lmr_step", "lmr_step_forced",
            "lmr_get_field", "lmr_get_grad", "lmr_get_state", "lmr_loss_grad",
            "lmr_workspace_bytes",
            "lmr_update", "lmr_warp", "lmr_decide_probe", "lmr_smooth",
            "lmr_set_state", "lmr_kernel_name", "lmr_profile_start",
            "lmr_profile_stop", "lmr_avgpool", "lmr_upsample_field",
            "lmr_pyramid_create", "lmr_pyramid_run", "lmr_pyramid_level",
            "lmr_pyramid_destroy", "lmr_pyramid_use_graphs", "lmr_folded_count", "lmr_batch_create",
            "lmr_force_decision", "lmr_batch_begin", "lmr_batch_step", "lmr_batch_sync",
            "lmr_batch_test_residency", "lmr_batch_pair",
            "lmr_batch_set_config", "lmr_batch_get_config", "lmr_batch_tune",
            "lmr_batch_destroy", "lmr_unet_param_count", "lmr_unet_layer_info",
            "lmr_unet_create", "lmr_unet_destroy", "lmr_unet_set_params",
            "lmr_unet_get_params", "lmr_unet_get_grads", "lmr_unet_forward",
            "lmr_unet_backward", "lmr_unet_adam", "lmr_unet_layer_probe",
            "lmr_loss_grad_noalloc"]


def _check(status: int, what: str):
    if status != 0:
        detail = lib().lmr_last_error().decode()
        raise LmrError(f"{what}: {_STATUS.get(status, status)}"
                       + (f" ({detail})" if detail else ""))


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _img_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return LMR_F32
    if t.dtype == torch.bfloat16:
        return LMR_BF16
    raise LmrError(f"image dtype must be float32 or bfloat16, got {t.dtype}")


def _dev(t: torch.Tensor, shape, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise LmrError(f"{name} must be a CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise LmrError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise LmrError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise LmrError(f"{name} must be contiguous")
    return t.data_ptr()


class Context:
    """One registration pair on one stream (lmr_ctx)."""

    def __init__(self, shape, img_dtype=torch.float32, params: Params | None = None,
                 stream=None, **kw):
        self.shape = tuple(int(s) for s in shape)
        self.img_dtype = img_dtype
        self.params = params if params is not None else Params.make(**kw)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = _V()
        self._destroy = lib().lmr_destroy
        code = LMR_BF16 if img_dtype == torch.bfloat16 else LMR_F32
        _check(lib().lmr_create(C.byref(self._h), *self.shape, code,
                                C.byref(self.params), _stream_handle(self.stream)),
               "lmr_create")

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None  # (module globals may be gone at interpreter exit)

    __del__ = close

    def _imgs(self, F, M):
        return (_dev(F, self.shape, self.img_dtype, "fixed"),
                _dev(M, self.shape, self.img_dtype, "moving"))

    def _field(self, u, name="field"):
        return _dev(u, (3,) + self.shape, torch.float32, name)

    def begin(self, F, M, field=None, lambda0=1.0):
        f, m = self._imgs(F, M)
        u = self._field(field) if field is not None else None
        _check(lib().lmr_begin(self._h, f, m, u, float(lambda0)), "lmr_begin")
        return self

    def step(self, F, M, n=1):
        f, m = self._imgs(F, M)
        _check(lib().lmr_step(self._h, f, m, int(n)), "lmr_step")

    def step_forced(self, F, M, decisions):
        f, m = self._imgs(F, M)
        arr = (C.c_int * len(decisions))(*[int(d) for d in decisions])
        _check(lib().lmr_step_forced(self._h, f, m, arr, len(decisions)),
               "lmr_step_forced")

    def force_decision(self, decision: int):
        """Decision of every later step() attempt: 1, 0, or -1 (automatic)."""
        _check(lib().lmr_force_decision(self._h, int(decision)), "lmr_force_decision")

    def field(self, out=None):
        out = out if out is not None else torch.empty((3,) + self.shape,
                                                      device="cuda")
        _check(lib().lmr_get_field(self._h, self._field(out, "out")), "lmr_get_field")
        return out

    def workspace_bytes(self) -> int:
        n = C.c_size_t()
        _check(lib().lmr_workspace_bytes(self._h, C.byref(n)), "lmr_workspace_bytes")
        return n.value

    def grad(self, out=None):
        out = out if out is not None else torch.empty((3,) + self.shape,
                                                      device="cuda")
        _check(lib().lmr_get_grad(self._h, self._field(out, "out")), "lmr_get_grad")
        return out

    def state(self) -> dict:
        s = PairState()
        _check(lib().lmr_get_state(self._h, C.byref(s)), "lmr_get_state")
        return s.as_dict()

    def profile_start(self, max_attempts=1000, stride=1):
        _check(lib().lmr_profile_start(self._h, int(max_attempts), int(stride)),
               "lmr_profile_start")

    def profile_stop(self) -> dict:
        return _profile_stop(self._h)

    def folded_count(self, u=None, with_det=False):
        """Voxels with det(I + grad u) <= 0 (u None: the accepted field)."""
        up = self._field(u, "u") if u is not None else None
        det = torch.empty(self.shape, device="cuda") if with_det else None
        n = C.c_longlong()
        _check(lib().lmr_folded_count(self._h, up, C.byref(n),
                                      det.data_ptr() if with_det else None),
               "lmr_folded_count")
        return (n.value, det) if with_det else n.value

    def set_state(self, state: dict):
        s = PairState(**{k: state.get(k, 0) for k, _ in PairState._fields_})
        _check(lib().lmr_set_state(self._h, C.byref(s)), "lmr_set_state")

    def loss_grad(self, F, M, u, raw=True, smooth=True, cc=False):
        f, m = self._imgs(F, M)
        up = self._field(u, "u")
        gr = torch.empty((3,) + self.shape, device="cuda") if raw else None
        gs = torch.empty((3,) + self.shape, device="cuda") if smooth else None
        cm = torch.empty(self.shape, device="cuda") if cc else None
        L = C.c_double()
        _check(lib().lmr_loss_grad(self._h, f, m, up, C.byref(L),
                                   gr.data_ptr() if raw else None,
                                   gs.data_ptr() if smooth else None,
                                   cm.data_ptr() if cc else None), "lmr_loss_grad")
        return L.value, gr, gs, cm

    def smooth(self, g, out=None):
        out = out if out is not None else torch.empty((3,) + self.shape,
                                                      device="cuda")
        if out.data_ptr() == g.data_ptr():
            raise LmrError("smooth: g and out must be distinct")
        _check(lib().lmr_smooth(self._h, self._field(g, "g"),
                                self._field(out, "out")), "lmr_smooth")
        return out

    def decide_probe(self, state: dict, cand_loss: float, force: int = -1) -> dict:
        sin = PairState(**{k: state.get(k, 0) for k, _ in PairState._fields_})
        sout = PairState()
        _check(lib().lmr_decide_probe(self._h, C.byref(sin), float(cand_loss),
                                      int(force), C.byref(sout)), "lmr_decide_probe")
        return sout.as_dict()

    def update(self, u, g_smooth, r, lam, out=None):
        out = out if out is not None else torch.empty((3,) + self.shape,
                                                      device="cuda")
        _check(lib().lmr_update(self._h, self._field(u, "u"),
                                self._field(g_smooth, "g_smooth"), float(r),
                                float(lam), self._field(out, "out")), "lmr_update")
        return out


def loss_grad_noalloc(F, M, u, params: Params | None = None, raw=True, smooth=True,
                      cc=False, out=None, stream=None, **kw):
    """lmr_loss_grad_noalloc: loss and gradients of u without a context and
    without allocating in the library.  Returns (loss, g_raw, g_smooth, cc)
    as device tensors (loss: float64 [1]); `out` may supply them (a dict with
    keys loss, g_raw, g_smooth, cc) so that the call allocates nothing at
    all.  Enqueues only."""
    shape = tuple(F.shape)
    p = params if params is not None else Params.make(**kw)
    f = _dev(F, shape, F.dtype, "fixed")
    m = _dev(M, shape, F.dtype, "moving")
    up = _dev(u, (3,) + shape, torch.float32, "u")
    out = dict(out or {})
    if "loss" not in out:
        out["loss"] = torch.empty(1, dtype=torch.float64, device="cuda")
    for key, want, sh in (("g_raw", raw, (3,) + shape), ("g_smooth", smooth, (3,) + shape),
                          ("cc", cc, shape)):
        if want and key not in out:
            out[key] = torch.empty(sh, device="cuda")
        if not want:
            out[key] = None
    ptr = {k: (_dev(v, tuple(v.shape), v.dtype, k) if v is not None else None)
           for k, v in out.items()}
    _check(lib().lmr_loss_grad_noalloc(f, m, _img_code(F), up, *shape, C.byref(p),
                                       ptr["loss"], ptr["g_raw"], ptr["g_smooth"], ptr["cc"],
                                       _stream_handle(stream)), "lmr_loss_grad_noalloc")
    return out["loss"], out["g_raw"], out["g_smooth"], out["cc"]


def warp(M: torch.Tensor, u: torch.Tensor, with_grad=False, stream=None):
    shape = tuple(M.shape)
    if len(shape) != 3:
        raise LmrError("moving must be [nz][ny][nx]")
    m = _dev(M, shape, M.dtype, "moving")
    up = _dev(u, (3,) + shape, torch.float32, "u")
    Mw = torch.empty(shape, device=M.device)
    dMw = torch.empty((3,) + shape, device=M.device) if with_grad else None
    _check(lib().lmr_warp(m, _img_code(M), up, *shape, Mw.data_ptr(),
                          dMw.data_ptr() if with_grad else None,
                          _stream_handle(stream)), "lmr_warp")
    return (Mw, dMw) if with_grad else Mw


def _profile_stop(h) -> dict:
    arr = (KernelTime * len(KERNELS))()
    _check(lib().lmr_profile_stop(h, arr), "lmr_profile_stop")
    out = {}
    for k, name in enumerate(KERNELS):
        t = arr[k]
        out[name] = dict(count=int(t.count), total_ms=t.total_ms, min_ms=t.min_ms,
                         max_ms=t.max_ms,
                         avg_ms=(t.total_ms / t.count) if t.count else float("nan"))
    return out


class LevelView:
    """Borrowed view of one pyramid level's context."""

    def __init__(self, handle, shape, img_dtype=torch.float32):
        self._h = handle
        self.shape = shape
        self.img_dtype = img_dtype

    def _imgs(self, F, M):
        return (_dev(F, self.shape, self.img_dtype, "fixed"),
                _dev(M, self.shape, self.img_dtype, "moving"))

    def begin(self, F, M, field=None, lambda0=1.0):
        f, m = self._imgs(F, M)
        u = _dev(field, (3,) + self.shape, torch.float32, "field") if field is not None \
            else None
        _check(lib().lmr_begin(self._h, f, m, u, float(lambda0)), "lmr_begin")

    def step(self, F, M, n=1):
        """Attempts on this level (images of this level's size)."""
        f, m = self._imgs(F, M)
        _check(lib().lmr_step(self._h, f, m, int(n)), "lmr_step")

    def field(self, sync=True):
        """Copy of the accepted field.  sync=True synchronises the context's
        stream (which need not be torch's current one); sync=False only
        enqueues the copy on it."""
        out = torch.empty((3,) + self.shape, device="cuda")
        _check(lib().lmr_get_field(self._h, out.data_ptr()), "lmr_get_field")
        if sync:
            _check(lib().lmr_get_state(self._h, C.byref(PairState())), "lmr_get_state")
        return out

    def grad(self, sync=True):
        """Copy of the smoothed gradient of the accepted field (as field())."""
        out = torch.empty((3,) + self.shape, device="cuda")
        _check(lib().lmr_get_grad(self._h, out.data_ptr()), "lmr_get_grad")
        if sync:
            _check(lib().lmr_get_state(self._h, C.byref(PairState())), "lmr_get_state")
        return out

    def folded_count(self, u=None):
        up = _dev(u, (3,) + self.shape, torch.float32, "u") if u is not None else None
        n = C.c_longlong()
        _check(lib().lmr_folded_count(self._h, up, C.byref(n), None), "lmr_folded_count")
        return n.value

    def state(self) -> dict:
        s = PairState()
        _check(lib().lmr_get_state(self._h, C.byref(s)), "lmr_get_state")
        return s.as_dict()

    def profile_start(self, max_attempts=1000, stride=1):
        _check(lib().lmr_profile_start(self._h, int(max_attempts), int(stride)),
               "lmr_profile_start")

    def profile_stop(self) -> dict:
        return _profile_stop(self._h)


class Pyramid:
    """Coarse-to-fine registration (lmr_pyramid)."""

    def __init__(self, shape, factors=(4, 2, 1), img_dtype=torch.float32,
                 params: Params | None = None, stream=None, **kw):
        self.shape = tuple(int(s) for s in shape)
        self.factors = tuple(int(f) for f in factors)
        self.img_dtype = img_dtype
        self.params = params if params is not None else Params.make(**kw)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = _V()
        self._destroy = lib().lmr_pyramid_destroy
        fa = (C.c_int * len(self.factors))(*self.factors)
        code = LMR_BF16 if img_dtype == torch.bfloat16 else LMR_F32
        _check(lib().lmr_pyramid_create(C.byref(self._h), *self.shape, code,
                                        C.byref(self.params), len(self.factors), fa,
                                        _stream_handle(self.stream)),
               "lmr_pyramid_create")

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None  # (module globals may be gone at interpreter exit)

    __del__ = close

    def use_graphs(self, enable: bool):
        _check(lib().lmr_pyramid_use_graphs(self._h, int(bool(enable))),
               "lmr_pyramid_use_graphs")

    def level(self, l) -> LevelView:
        h = lib().lmr_pyramid_level(self._h, int(l))
        if not h:
            raise LmrError(f"no level {l}")
        f = self.factors[l]
        return LevelView(C.c_void_p(h), tuple(s // f for s in self.shape),
                         self.img_dtype if f == 1 else torch.float32)

    def run(self, F, M, iters, lambda0=1.0, decisions=None, out=None):
        f = _dev(F, self.shape, self.img_dtype, "fixed")
        m = _dev(M, self.shape, self.img_dtype, "moving")
        if len(iters) != len(self.factors):
            raise LmrError("one iteration count per level is required")
        it = (C.c_int * len(iters))(*[int(i) for i in iters])
        dp = None
        if decisions is not None:
            if len(decisions) != sum(iters):
                raise LmrError("decisions must hold sum(iters) entries")
            dp = (C.c_int * len(decisions))(*[int(d) for d in decisions])
        out = out if out is not None else torch.empty((3,) + self.shape, device="cuda")
        _check(lib().lmr_pyramid_run(self._h, f, m, it, float(lambda0), dp,
                                     _dev(out, (3,) + self.shape, torch.float32,
                                          "out")), "lmr_pyramid_run")
        return out


class Batch:
    """Uneven-size pairs advanced together by one persistent launch per
    iteration (lmr_batch).  The batch owns its stream; every call that reads
    results synchronises it."""

    def __init__(self, shapes, img_dtype=torch.float32, params: Params | None = None,
                 **kw):
        self.shapes = [tuple(int(s) for s in sh) for sh in shapes]
        self.img_dtype = img_dtype
        self.params = params if params is not None else Params.make(**kw)
        self._h = _V()
        self._destroy = lib().lmr_batch_destroy
        flat = (C.c_int * (3 * len(self.shapes)))(*[s for sh in self.shapes for s in sh])
        code = LMR_BF16 if img_dtype == torch.bfloat16 else LMR_F32
        _check(lib().lmr_batch_create(C.byref(self._h), len(self.shapes), flat, code,
                                      C.byref(self.params)), "lmr_batch_create")
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None  # (module globals may be gone at interpreter exit)

    __del__ = close

    def _ptrs(self, Fs, Ms):
        if len(Fs) != len(self.shapes) or len(Ms) != len(self.shapes):
            raise LmrError("one fixed and one moving image per pair")
        fp = (C.c_void_p * len(Fs))(*[_dev(F, sh, self.img_dtype, "fixed")
                                      for F, sh in zip(Fs, self.shapes)])
        mp = (C.c_void_p * len(Ms))(*[_dev(M, sh, self.img_dtype, "moving")
                                      for M, sh in zip(Ms, self.shapes)])
        return fp, mp

    def begin(self, Fs, Ms, lambda0=None):
        fp, mp = self._ptrs(Fs, Ms)
        lp = None if lambda0 is None else (C.c_double * len(Fs))(*lambda0)
        _check(lib().lmr_batch_begin(self._h, fp, mp, lp), "lmr_batch_begin")
        self._keep = (list(Fs), list(Ms))   # the device table points at them

    def step(self, n=1, graph=True):
        _check(lib().lmr_batch_step(self._h, int(n), int(bool(graph))), "lmr_batch_step")

    def sync(self):
        _check(lib().lmr_batch_sync(self._h), "lmr_batch_sync")

    def sync_status(self) -> int:
        """lmr_batch_sync's status (0, or LMR_EBUSY / LMR_EHIP) without raising."""
        return int(lib().lmr_batch_sync(self._h))

    def test_residency(self, late_block: int):
        _check(lib().lmr_batch_test_residency(self._h, int(late_block)),
               "lmr_batch_test_residency")

    def tune(self, Fs, Ms, cache_path=None, iters=3):
        fp, mp = self._ptrs(Fs, Ms)
        ms = C.c_double()
        _check(lib().lmr_batch_tune(self._h, fp, mp,
                                    cache_path.encode() if cache_path else None,
                                    int(iters), C.byref(ms)), "lmr_batch_tune")
        return ms.value

    def config(self):
        cfg = (C.c_int * 3)()
        _check(lib().lmr_batch_get_config(self._h, cfg), "lmr_batch_get_config")
        return dict(target_tiles=cfg[0], min_cz=cfg[1], blocks_per_cu=cfg[2])

    def set_config(self, target_tiles, min_cz, blocks_per_cu=0):
        _check(lib().lmr_batch_set_config(self._h, int(target_tiles), int(min_cz),
                                          int(blocks_per_cu)), "lmr_batch_set_config")

    def pair(self, i) -> "PairView":
        h = lib().lmr_batch_pair(self._h, int(i))
        if not h:
            raise LmrError(f"no pair {i}")
        return PairView(C.c_void_p(h), self.shapes[i], self.img_dtype)


class PairView(LevelView):
    """Borrowed view of one pair of a batch."""


def avgpool(img: torch.Tensor, f: int, stream=None) -> torch.Tensor:
    shape = tuple(img.shape)
    if len(shape) != 3 or any(s % f for s in shape):
        raise LmrError("avgpool: [nz][ny][nx] divisible by f required")
    p = _dev(img, shape, img.dtype, "img")
    out = torch.empty(tuple(s // f for s in shape), device=img.device)
    _check(lib().lmr_avgpool(p, _img_code(img), *shape, int(f), out.data_ptr(),
                             _stream_handle(stream)), "lmr_avgpool")
    return out


def upsample_field(uc: torch.Tensor, stream=None) -> torch.Tensor:
    if uc.dim() != 4 or uc.shape[0] != 3:
        raise LmrError("upsample_field: [3][nz][ny][nx] required")
    shape = tuple(uc.shape[1:])
    p = _dev(uc, (3,) + shape, torch.float32, "uc")
    out = torch.empty((3,) + tuple(2 * s for s in shape), device=uc.device)
    _check(lib().lmr_upsample_field(p, *shape, out.data_ptr(), _stream_handle(stream)),
           "lmr_upsample_field")
    return out


def unet_layers():
    """(cin, cout, relu, offset) of every U-Net layer (lmreg_unet.h)."""
    out = []
    for l in range(15):
        ci, co, re, off = C.c_int(), C.c_int(), C.c_int(), C.c_int64()
        _check(lib().lmr_unet_layer_info(l, C.byref(ci), C.byref(co), C.byref(re),
                                         C.byref(off)), "lmr_unet_layer_info")
        out.append((ci.value, co.value, bool(re.value), off.value))
    return out


def unet_param_count() -> int:
    return int(lib().lmr_unet_param_count())


class UNet:
    """The learned initializer's network (lmr_unet) at a fixed resolution."""

    def __init__(self, shape, stream=None):
        self.shape = tuple(int(s) for s in shape)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.n_params = unet_param_count()
        self._h = _V()
        self._destroy = lib().lmr_unet_destroy
        _check(lib().lmr_unet_create(C.byref(self._h), *self.shape,
                                     _stream_handle(self.stream)), "lmr_unet_create")

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None  # (module globals may be gone at interpreter exit)

    __del__ = close

    def set_params(self, flat: torch.Tensor):
        _check(lib().lmr_unet_set_params(
            self._h, _dev(flat, (self.n_params,), torch.float32, "params")),
            "lmr_unet_set_params")

    def params(self) -> torch.Tensor:
        out = torch.empty(self.n_params, device="cuda")
        _check(lib().lmr_unet_get_params(self._h, out.data_ptr()), "lmr_unet_get_params")
        return out

    def grads(self) -> torch.Tensor:
        out = torch.empty(self.n_params, device="cuda")
        _check(lib().lmr_unet_get_grads(self._h, out.data_ptr()), "lmr_unet_get_grads")
        return out

    def forward(self, F, M, pool=False, out=None):
        """Predicted field [3][nz][ny][nx] (FP32) from images of the network's
        size, or of twice its size with pool=True."""
        ish = tuple(2 * s for s in self.shape) if pool else self.shape
        f = _dev(F, ish, F.dtype, "fixed")
        m = _dev(M, ish, F.dtype, "moving")
        if out is None:
            out = torch.empty((3,) + self.shape, device="cuda")
        _check(lib().lmr_unet_forward(self._h, f, m, _img_code(F), int(bool(pool)),
                                      _dev(out, (3,) + self.shape, torch.float32, "out")),
               "lmr_unet_forward")
        return out

    def backward(self, target, target_scale=1.0, accumulate=False, loss=None):
        """MSE backward against target_scale * target; `loss` (a float64 CUDA
        tensor of one element) receives the MSE without synchronising."""
        lp = _dev(loss, (1,), torch.float64, "loss") if loss is not None else None
        _check(lib().lmr_unet_backward(
            self._h, _dev(target, (3,) + self.shape, torch.float32, "target"),
            float(target_scale), int(bool(accumulate)), lp), "lmr_unet_backward")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        _check(lib().lmr_unet_adam(self._h, float(lr), float(beta1), float(beta2),
                                   float(eps), float(grad_scale)), "lmr_unet_adam")

    def layer_probe(self, layer, x, dz=None):
        """One layer alone (lmr_unet_layer_probe).  x: int16 CUDA tensor of
        BF16 bits [N_l][ldx]; dz (optional) likewise [N_l][ldz].  Returns
        (y FP32 [N_l][cout], dx BF16 bits [N_l][cin] or None, dW [27][cin][cout]
        or None, db [cout] or None)."""
        ci, co, _, _ = unet_layers()[layer]
        n = x.shape[0]
        for t, name in ((x, "x"),) + (((dz, "dz"),) if dz is not None else ()):
            if not (t.is_cuda and t.dtype == torch.int16 and t.dim() == 2 and
                    t.is_contiguous() and t.shape[0] == n):
                raise LmrError(f"{name} must be a contiguous int16 CUDA tensor [N][ld]")
        y = torch.empty((n, co), device="cuda")
        dx = dW = db = None
        if dz is not None:
            dx = torch.empty((n, ci), dtype=torch.int16, device="cuda")
            dW = torch.empty((27, ci, co), device="cuda")
            db = torch.empty(co, device="cuda")
        _check(lib().lmr_unet_layer_probe(
            self._h, int(layer), x.data_ptr(), x.shape[1], y.data_ptr(), co,
            dz.data_ptr() if dz is not None else None, dz.shape[1] if dz is not None else 0,
            dx.data_ptr() if dx is not None else None, ci,
            dW.data_ptr() if dW is not None else None,
            db.data_ptr() if db is not None else None), "lmr_unet_layer_probe")
        return y, dx, dW, db
