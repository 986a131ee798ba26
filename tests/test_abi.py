"""The C-ABI library loads and exports every function include/*.h declares.

Runs without a GPU: no call here launches a kernel.  Argument checks that the
library performs before touching the device are exercised too.
"""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(lmr_\w+)\s*\(", txt, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    d = _declared()
    for must in ("lmr_create", "lmr_begin", "lmr_step", "lmr_get_state",
                 "lmr_destroy", "lmr_loss_grad", "lmr_warp"):
        assert must in d


def test_library_exports_every_declared_symbol():
    from paper_2603_19371_amd import _lib
    L = _lib.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.exported_symbols()) <= set(_declared())


def test_default_params_and_errors_without_device():
    from paper_2603_19371_amd import _lib
    L = _lib.lib()
    p = _lib.Params.make()
    assert p.window == 5 and p.grad_sigma == 1.0 and p.cc_eps == 1e-5
    assert p.lambda_inc == 2.0 and p.lambda_dec == 0.5 and p.tau == 0.0
    h = C.c_void_p()
    for bad in (dict(window=4), dict(window=11), dict(lambda_inc=1.0),
                dict(lambda_dec=1.0), dict(grad_sigma=-1.0), dict(step_eps=0.0),
                dict(lambda_min=0.0), dict(max_retries=0), dict(accum=7),
                dict(tile=0), dict(tile=17), dict(optimizer=2), dict(optimizer=1, tile=2),
                dict(optimizer=1, adam_lr=0.0), dict(optimizer=1, adam_beta2=1.0)):
        pb = _lib.Params.make(**bad)
        assert L.lmr_create(C.byref(h), 8, 8, 8, 0, C.byref(pb), None) == 1, bad
    assert L.lmr_create(C.byref(h), 0, 8, 8, 0, C.byref(p), None) == 1
    assert L.lmr_create(C.byref(h), 8, 8, 8, 5, C.byref(p), None) == 1
    assert L.lmr_create(C.byref(h), 1024, 1024, 1024, 0, C.byref(p), None) == 1
    assert L.lmr_strerror(0) == b"ok"
    assert L.lmr_step(None, None, None, 1) == 1


def test_binding_rejects_bad_tensors_before_the_library():
    torch = pytest.importorskip("torch")
    from paper_2603_19371_amd import _lib
    with pytest.raises(_lib.LmrError):
        _lib._dev(torch.zeros(4, 4, 4), (4, 4, 4), torch.float32, "x")  # CPU tensor
