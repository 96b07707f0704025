"""API errors on a live context (the error path, forced from the host): calls
out of order, out-of-range arguments and invalid flag combinations return a
negative status with a message and leave the context usable; a frame of an
unrelated scene tracks to a high robust error rather than failing the call."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_state_and_argument_errors_leave_the_context_usable(gpu_lib):
    dpt = gpu_lib
    lib = dpt.load()
    cam = synth.CAM_640
    trk = dpt.Tracker(cam, dpt.make_params(levels=3), max_points=500)
    r = dpt.Result()
    T = (ctypes.c_double * 16)(*np.eye(4).reshape(-1))
    assert lib.dpt_track_frame(trk._h, T, ctypes.byref(r)) == dpt.DPT_E_STATE  # no pyramids, no reference
    assert b"reference" in lib.dpt_last_error() or b"pyramid" in lib.dpt_last_error()
    d = synth.pair(1, cam)
    img = np.ascontiguousarray(d["ref"])
    p = img.ctypes.data
    assert lib.dpt_build_pyramid(trk._h, 2, p, cam.width, 0) == dpt.DPT_E_ARG  # no such slot
    assert lib.dpt_build_pyramid(trk._h, 0, p, cam.width - 1, 0) == dpt.DPT_E_ARG  # pitch < width
    assert lib.dpt_build_pyramid(trk._h, 0, p, cam.width, 5) == dpt.DPT_E_ARG  # unknown memory kind
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    out = np.empty((10, 10), np.uint8)
    assert lib.dpt_get_pyramid(trk._h, 0, 3, out.ctypes.data) == dpt.DPT_E_ARG  # level beyond the pyramid
    P = synth.backproject(cam, d["depth"], oracle.select_points(d["ref"], 500, 8), d["T_rw"])
    Tm = (ctypes.c_double * 16)(*d["T_rw"].reshape(-1))
    big = np.zeros((501, 3), np.float32)
    assert lib.dpt_set_reference_points(trk._h, big.ctypes.data, 501, Tm, 0) == dpt.DPT_E_ARG  # above capacity
    nan = np.eye(4)
    nan[0, 3] = np.nan
    assert lib.dpt_set_reference_points(trk._h, P.ctypes.data, 500,
                                        (ctypes.c_double * 16)(*nan.reshape(-1)), 0) == dpt.DPT_E_ARG
    assert lib.dpt_get_fixed_hessian(trk._h, 0, np.empty(36).ctypes.data, ctypes.byref(ctypes.c_int32())) \
        == dpt.DPT_E_STATE  # not a fixed-H context
    assert lib.dpt_get_pyramid_f32(trk._h, 0, 0, np.empty(cam.width * cam.height, np.float32).ctypes.data) \
        == dpt.DPT_E_STATE  # no float pyramid in this context
    # still usable: the same context tracks normally
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    g = trk.track(np.eye(4))
    o = oracle.Reference(cam, oracle.make_params(levels=3), d["ref"], P, d["T_rw"]).track(d["cur"], np.eye(4))
    rot, tr = oracle.pose_error(g["T_cw"], o["T_cw"])
    assert g["status"] == 0 and rot < 1e-4 and tr < 1e-4


@pytest.mark.parametrize("kw", [dict(precision=1, fixed_h=True), dict(precision=1, gauss=True),
                                dict(precision=1, pattern=synth.square_pattern(3)), dict(flags=4)])
def test_invalid_parameter_combinations(gpu_lib, kw):
    dpt = gpu_lib
    with pytest.raises(dpt.DptError) as e:
        dpt.Tracker(synth.CAM_640, dpt.make_params(levels=3, **kw), max_points=10)
    assert e.value.code == dpt.DPT_E_ARG


def test_unrelated_scene_gives_a_high_error(gpu_lib):
    dpt = gpu_lib
    cam = synth.CAM_640
    d, other = synth.pair(2, cam), synth.pair(90, cam)
    P = synth.backproject(cam, d["depth"], oracle.select_points(d["ref"], 500, 8), d["T_rw"])
    trk = dpt.Tracker(cam, dpt.make_params(levels=3), max_points=500)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    good = trk.track(np.eye(4))
    trk.build_pyramid(dpt.SLOT_CUR, other["cur"])
    bad = trk.track(np.eye(4))
    assert good["status"] == 0
    assert bad["final_cost"] > 10 * good["final_cost"]
