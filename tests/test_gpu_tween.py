"""GPU tween-window schedule (dpt_tween_*) against the oracle's schedule
(Sec. III, Sec. IV-D) on a seeded sequence with exposure flicker and dropped
frames: the same decision on every frame, the same anchors, direct poses
within the tracker's parity bar, and the same share of direct frames."""
import numpy as np
import pytest

import oracle
import synth
from oracle import tween

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL = 1e-4, 1e-4


def _run_gpu(dpt, trk, frames, pol):
    recs = []
    for k, (img, depth, T) in enumerate(frames):
        if k == 0:
            trk.tween_anchor(img, depth.astype(np.float32), T)
            recs.append(dict(decision=None, pose=T, track=None))
            continue
        r = trk.tween_frame(img)
        if r["decision"] == dpt.TWEEN_DIRECT:
            r["pose"] = r["track"]["T_cw"]
        else:
            trk.tween_anchor(img, depth.astype(np.float32), T)
            r["pose"] = T
        recs.append(r)
    return recs


@pytest.mark.parametrize("launch", [(0, 256), (1, 256)])  # auto (cooperative), one workgroup
def test_tween_schedule_matches_oracle(gpu_lib, launch):
    dpt = gpu_lib
    cam = synth.CAM_752
    frames = [(im, d.astype(np.float32), T) for _, im, d, T, _ in
              synth.tween_frames(n_frames=90, jump=(40, 160), p_jump=0.05)]  # both sides read FP32 depths
    pol = dict(max_cost=20.0, max_baseline=0.035, max_direct=12, n_points=2000, margin=8)  # margins: cost > 12, baseline > 4e-3
    prm = dpt.make_params(levels=4)
    trk = dpt.Tracker(cam, prm, max_points=2000)
    trk.set_launch_config(*launch)
    trk.tween_set_policy(pol["max_cost"], pol["max_direct"], pol["n_points"], max_baseline=pol["max_baseline"],
                         margin=pol["margin"])
    g = _run_gpu(dpt, trk, frames, pol)
    o = tween.run(frames, pol, tween.oracle_reference(cam, oracle.make_params(levels=4), pol))
    gd = [r["decision"] for r in g]
    od = [r["decision"] for r in o]
    print("gpu   ", gd)
    print("oracle", od)
    assert gd == od
    assert len(set(od[1:])) >= 3  # the run exercises several rules
    for k, (a, b) in enumerate(zip(g, o)):
        if b["track"] is None:
            continue
        assert a["track"]["status"] == b["track"]["status"]
        if b["track"]["status"] in (oracle.OK, oracle.MAX_ITERS) and b["track"]["final_cost"] < pol["max_cost"]:
            rot, tr = oracle.pose_error(a["track"]["T_cw"], b["track"]["T_cw"])
            assert rot < ROT_TOL and tr < TR_TOL, (k, rot, tr)
            assert abs(a["track"]["final_cost"] - b["track"]["final_cost"]) <= 1e-3 * b["track"]["final_cost"]
            assert abs(a["baseline"] - b["baseline"]) < 1e-4
    gts = [f[2] for f in frames]
    sg, so = tween.summary(g, gts), tween.summary(o, gts)
    print("gpu", sg, "\noracle", so)
    assert sg["counts"] == so["counts"]
    assert abs(sg["ate_rmse_m"] - so["ate_rmse_m"]) < 1e-4


def test_tween_state_errors_and_max_frames(gpu_lib):
    dpt = gpu_lib
    cam = synth.CAM_640
    frames = [(im, d, T) for _, im, d, T, _ in synth.tween_frames(n_frames=4, cam=cam, p_jump=0.0, p_flicker=0.0)]
    trk = dpt.Tracker(cam, dpt.make_params(levels=3), max_points=300)
    with pytest.raises(dpt.DptError):  # no policy
        trk.tween_anchor(frames[0][0], frames[0][1].astype(np.float32), frames[0][2])
    with pytest.raises(dpt.DptError):  # n_points above the context's capacity
        trk.tween_set_policy(20.0, 2, 301)
    trk.tween_set_policy(20.0, 1, 300)
    with pytest.raises(dpt.DptError):  # no reference yet
        trk.tween_frame(frames[1][0])
    trk.tween_anchor(frames[0][0], frames[0][1].astype(np.float32), frames[0][2])
    r1 = trk.tween_frame(frames[1][0])
    assert r1["decision"] == dpt.TWEEN_DIRECT and r1["direct_since_ref"] == 1 and r1["tracked"]
    r2 = trk.tween_frame(frames[2][0])
    assert r2["decision"] == dpt.TWEEN_MAX_FRAMES and not r2["tracked"]
    with pytest.raises(dpt.DptError):  # the indirect side must anchor first
        trk.tween_frame(frames[3][0])
    trk.tween_anchor(frames[2][0], frames[2][1].astype(np.float32), frames[2][2])
    r3 = trk.tween_frame(frames[3][0])
    assert r3["decision"] == dpt.TWEEN_DIRECT and r3["direct_since_ref"] == 1
    rot, tr = oracle.pose_error(r3["track"]["T_cw"], frames[3][2])
    assert rot < 2e-3 and tr < 5e-3


def test_tween_schedule_with_reference_stream(gpu_lib):
    """The schedule's re-anchoring runs its reference updates on a second
    stream when the context has one: every decision and pose bitwise as on one
    stream."""
    dpt = gpu_lib
    cam = synth.CAM_752
    frames = [(im, d.astype(np.float32), T) for _, im, d, T, _ in
              synth.tween_frames(n_frames=60, jump=(40, 160), p_jump=0.05)]
    pol = dict(max_cost=20.0, max_baseline=0.035, max_direct=12, n_points=2000, margin=8)
    runs = []
    rs = dpt.Stream()
    for second in (False, True):
        trk = dpt.Tracker(cam, dpt.make_params(levels=4), max_points=2000)
        if second:
            trk.set_reference_stream(rs)
        trk.tween_set_policy(pol["max_cost"], pol["max_direct"], pol["n_points"], max_baseline=pol["max_baseline"],
                             margin=pol["margin"])
        runs.append(_run_gpu(dpt, trk, frames, pol))
        trk.close()
    rs.close()
    a, b = runs
    assert [r["decision"] for r in a] == [r["decision"] for r in b]
    for ra, rb in zip(a, b):
        np.testing.assert_array_equal(np.asarray(ra["pose"]), np.asarray(rb["pose"]))
