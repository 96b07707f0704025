"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/*.h declares, and rejects bad arguments before any
device work."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_2607_16897_amd as dpt
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(dpt_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = dpt.load()
    declared = _declared()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(lib, name), f"{name} declared but not exported"
    assert declared <= set(dpt.SIGNATURES), "binding lacks a declared entry point"


def test_bad_arguments_are_rejected():
    lib = dpt.load()
    cam = dpt.make_camera(synth.CAM_640)
    prm = dpt.make_params()
    h = ctypes.c_void_p()
    assert lib.dpt_create(None, ctypes.byref(prm), 100, None, ctypes.byref(h)) == dpt.DPT_E_ARG
    assert b"NULL" in lib.dpt_last_error()
    bad = dpt.make_params(levels=9)
    assert lib.dpt_create(ctypes.byref(cam), ctypes.byref(bad), 100, None, ctypes.byref(h)) == dpt.DPT_E_ARG
    bad = dpt.make_params(max_iters=0)
    assert lib.dpt_create(ctypes.byref(cam), ctypes.byref(bad), 100, None, ctypes.byref(h)) == dpt.DPT_E_ARG
    bad = dpt.make_params(pattern=((40, 0),))
    assert lib.dpt_create(ctypes.byref(cam), ctypes.byref(bad), 100, None, ctypes.byref(h)) == dpt.DPT_E_ARG
    assert lib.dpt_create(ctypes.byref(cam), ctypes.byref(prm), 0, None, ctypes.byref(h)) == dpt.DPT_E_ARG
    assert lib.dpt_create(ctypes.byref(cam), ctypes.byref(prm), 1 << 20, None, ctypes.byref(h)) == dpt.DPT_E_ARG
    tiny = dpt.Camera(8, 8, 10.0, 10.0, 4.0, 4.0)
    assert lib.dpt_create(ctypes.byref(tiny), ctypes.byref(prm), 10, None, ctypes.byref(h)) == dpt.DPT_E_ARG
    assert lib.dpt_create(ctypes.byref(cam), ctypes.byref(prm), 10, None, None) == dpt.DPT_E_ARG
    # NULL contexts
    r = dpt.Result()
    T = (ctypes.c_double * 16)(*np.eye(4).reshape(-1))
    assert lib.dpt_track_frame(None, T, ctypes.byref(r)) == dpt.DPT_E_ARG
    assert lib.dpt_build_pyramid(None, 0, None, 640, 0) == dpt.DPT_E_ARG
    lib.dpt_destroy(None)
