"""Edge cases at the limits of the interface, against the oracle: the largest
pattern (K = 128), the deepest pyramid (8 levels) on a 2047x1535 frame, a
16000-point map with 7x7 patches on the Gaussian pyramid, and empty maps on
the generic-pattern paths."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL, COST_TOL = 1e-4, 1e-4, 1e-3
LAUNCHES = [(1, 256), (2, 256)]


def _oparams(p, gauss=False):
    pat = np.array(p.pattern[:2 * p.n_pattern]).reshape(-1, 2)
    return oracle.make_params(levels=p.levels, max_iters=p.max_iters, huber_k=p.huber_k, step_eps=p.step_eps,
                              min_points=p.min_points, pattern=pat, z_min=p.z_min, gauss=gauss)


def _run(dpt, cam, n, seed, launch, gauss=False, **kw):
    d = synth.pair(seed, cam)
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    prm = dpt.make_params(gauss=gauss, **kw)
    trk = dpt.Tracker(cam, prm, max_points=n)
    trk.set_launch_config(*launch)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    g = trk.track(np.eye(4))
    o = oracle.Reference(cam, _oparams(prm, gauss), d["ref"], P, d["T_rw"]).track(d["cur"], np.eye(4))
    rot, tr = oracle.pose_error(g["T_cw"], o["T_cw"])
    rel = abs(g["final_cost"] - o["final_cost"]) / max(o["final_cost"], 1e-12)
    print(f"{cam.width}x{cam.height} n={n} {launch}: rot {rot:.2e} tr {tr:.2e} cost {rel:.2e} "
          f"status {g['status']}/{o['status']} iters {g['iterations']}/{o['iterations']}")
    assert g["status"] == o["status"]
    assert g["status"] in (0, 1)
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL
    return g


def _pattern128():
    sq = synth.square_pattern(11)  # 121 offsets
    extra = np.array([(-7, 0), (7, 0), (0, -7), (0, 7), (-6, -6), (6, 6), (6, -6)], np.int32)
    return np.vstack([sq, extra])


@pytest.mark.parametrize("launch", LAUNCHES)
def test_largest_pattern(gpu_lib, launch):
    pat = _pattern128()
    assert len(pat) == 128
    _run(gpu_lib, synth.CAM_640, 300, 12, launch, levels=3, pattern=pat)


def test_eight_levels_large_frame(gpu_lib):
    cam = synth.Camera(2047, 1535, 900.0, 900.0, 1023.0, 767.0)
    _run(gpu_lib, cam, 3000, 14, (2, 256), levels=8)


def test_generic_16k_points_gauss_7x7(gpu_lib):
    _run(gpu_lib, synth.CAM_1280, 16000, 15, (2, 256), gauss=True, levels=4, pattern=synth.square_pattern(7))


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("gauss", [False, True])
def test_empty_map_generic(gpu_lib, launch, gauss):
    dpt = gpu_lib
    d = synth.pair(3)
    trk = dpt.Tracker(synth.CAM_640, dpt.make_params(levels=3, gauss=gauss, pattern=synth.square_pattern(5)),
                      max_points=64)
    trk.set_launch_config(*launch)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(np.zeros((0, 3), np.float32), d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    r = trk.track(np.eye(4))
    assert r["status"] == dpt.TRACK_TOO_FEW_POINTS and r["iterations"] == 0
