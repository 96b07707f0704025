"""Asynchronous tracks (dpt_track_enqueue / dpt_synchronize) and the pose
history with the constant-velocity start computed on the GPU: the same results
as the synchronous path started from the host's prediction, and the oracle's."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL = 1e-4, 1e-4
# Same-start comparisons: the GPU's prediction inverts poses as rigid motions,
# the host's with a general inverse; the estimates come from FP32 rotations
# (orthonormal to ~1e-7), so the two starts differ at that level, and a
# Gauss-Newton run that stops at max |delta| < 1e-5 may end that far apart.
SAME_TOL = 2e-5
WINDOW = 10


def _oparams(p):
    pat = np.array(p.pattern[:2 * p.n_pattern]).reshape(-1, 2)
    return oracle.make_params(levels=p.levels, max_iters=p.max_iters, huber_k=p.huber_k, step_eps=p.step_eps,
                              min_points=p.min_points, pattern=pat, z_min=p.z_min)


def _cv(T2, T1):
    return T1 @ np.linalg.inv(T2) @ T1


def _windows(n_win, seed=2607, cam=synth.CAM_752):
    traj, scene = synth.Trajectory(seed), synth.Scene(seed)
    out = []
    for w in range(n_win):
        k0 = WINDOW * w + 30
        imgs, gts, depth = [], [], None
        for j in range(WINDOW):
            T = traj.T_cw(k0 + j)
            img, dep = scene.render(cam, T, synth.pixel_noise(seed, k0 + j, cam, 2.0), want_depth=(j == 0))
            depth = dep.astype(np.float32) if j == 0 else depth
            imgs.append(img)
            gts.append(T)
        out.append(dict(imgs=imgs, gts=gts, depth=depth, T_prev=traj.T_cw(k0 - 1)))
    return out


def _sync_window(dpt, trk, win, n):
    trk.build_pyramid(dpt.SLOT_REF, win["imgs"][0])
    trk.set_reference_from_depth(n, win["depth"], win["gts"][0])
    prev2, prev1, res = win["T_prev"], win["gts"][0], []
    for j in range(1, WINDOW):
        trk.build_pyramid(dpt.SLOT_CUR, win["imgs"][j])
        r = trk.track(_cv(prev2, prev1))
        prev2, prev1 = prev1, r["T_cw"]
        res.append(r)
    return res


def _enqueue_window(dpt, trk, win, n, dev=None):
    imgs = dev if dev is not None else win["imgs"]
    trk.build_pyramid(dpt.SLOT_REF, imgs[0])
    trk.set_reference_from_depth(n, win["depth"], win["gts"][0])
    trk.set_pose_history(win["T_prev"], win["gts"][0])
    for j in range(1, WINDOW):
        trk.build_pyramid(dpt.SLOT_CUR, imgs[j])
        trk.track_enqueue(None)


def test_constant_velocity_enqueue_matches_host_prediction(gpu_lib):
    import torch

    dpt = gpu_lib
    cam, n = synth.CAM_752, 2000
    wins = _windows(2)
    prm = dpt.make_params(levels=4)
    sync_trk = dpt.Tracker(cam, prm, max_points=n)
    want = [r for w in wins for r in _sync_window(dpt, sync_trk, w, n)]
    trk = dpt.Tracker(cam, prm, max_points=n)
    for w in wins:  # both windows in flight at once: reference updates ordered on the stream
        _enqueue_window(dpt, trk, w, n, dev=[torch.from_numpy(im).cuda() for im in w["imgs"]])
    got = trk.synchronize()
    assert len(got) == len(want) == 2 * (WINDOW - 1)
    # Two chains of predictions cannot be compared frame by frame: a start
    # difference along a weakly constrained direction survives a track (its
    # Gauss-Newton steps fall below the 1e-5 threshold) and the constant-velocity
    # extrapolation amplifies it (about 2.4x per frame here, from 3e-8 m).  So
    # both chains are held to the tracking accuracy, and every frame is compared
    # with the oracle started from exactly the same prediction below.
    gts = [w["gts"][j] for w in wins for j in range(1, WINDOW)]
    for g, s, gt in zip(got, want, gts):
        assert g["status"] == s["status"] == 0
        for r in (g, s):
            rot, tr = oracle.pose_error(r["T_cw"], gt)
            assert rot < 2e-3 and tr < 5e-3, (rot, tr)
    # and the oracle, started from the same predictions
    refs = []
    for w in wins:
        idx = oracle.select_points(w["imgs"][0], n, 8)
        refs.append(oracle.Reference(cam, _oparams(prm), w["imgs"][0],
                                     synth.backproject(cam, w["depth"].astype(np.float64), idx, w["gts"][0]),
                                     w["gts"][0]))
    k = 0
    for wi, w in enumerate(wins):
        prev2, prev1 = w["T_prev"], w["gts"][0]
        for j in range(1, WINDOW):
            o = refs[wi].track(w["imgs"][j], _cv(prev2, prev1))
            rot, tr = oracle.pose_error(got[k]["T_cw"], o["T_cw"])
            assert rot < ROT_TOL and tr < TR_TOL
            prev2, prev1 = prev1, got[k]["T_cw"]
            k += 1


def test_given_enqueue_equals_track_frame_and_ring_limit(gpu_lib):
    dpt = gpu_lib
    d = synth.pair(4)
    cam, n = synth.CAM_640, 500
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    prm = dpt.make_params(levels=3)
    trk = dpt.Tracker(cam, prm, max_points=n)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    starts = [synth.random_perturbation(np.random.default_rng([4, i]), 0.5, 0.01) for i in range(dpt.MAX_IN_FLIGHT)]
    want = [trk.track(T) for T in starts[:5]]
    for T in starts:
        trk.track_enqueue(T)
    with pytest.raises(dpt.DptError):  # one track more than the ring holds
        trk.track_enqueue(starts[0])
    got = trk.synchronize()
    assert len(got) == dpt.MAX_IN_FLIGHT
    for g, s in zip(got, want):
        np.testing.assert_array_equal(g["T_cw"], s["T_cw"])
        assert g["iterations"] == s["iterations"] and g["final_cost"] == s["final_cost"]
    assert trk.synchronize() == []


def test_history_follows_synchronous_tracks(gpu_lib):
    """Every track appends its estimate; the next constant-velocity start is
    P1 P0^-1 P1 from the last two."""
    dpt = gpu_lib
    cam, n = synth.CAM_752, 2000
    win = _windows(1)[0]
    prm = dpt.make_params(levels=4)
    trk = dpt.Tracker(cam, prm, max_points=n)
    trk.build_pyramid(dpt.SLOT_REF, win["imgs"][0])
    trk.set_reference_from_depth(n, win["depth"], win["gts"][0])
    trk.build_pyramid(dpt.SLOT_CUR, win["imgs"][1])
    a = trk.track(win["gts"][1])
    trk.build_pyramid(dpt.SLOT_CUR, win["imgs"][2])
    b = trk.track(win["gts"][2])
    trk.build_pyramid(dpt.SLOT_CUR, win["imgs"][3])
    trk.track_enqueue(None)
    got = trk.synchronize()[0]
    want = trk.track(_cv(a["T_cw"], b["T_cw"]))
    rot, tr = oracle.pose_error(got["T_cw"], want["T_cw"])
    assert rot < SAME_TOL and tr < SAME_TOL


def test_batch_enqueue_matches_plain_enqueue(gpu_lib):
    import torch

    dpt = gpu_lib
    cam, n = synth.CAM_752, 1500
    wins = [_windows(1, seed=50 + s)[0] for s in range(3)]
    prm = dpt.make_params(levels=4)
    bt = dpt.BatchTracker([cam] * 3, prm, [n] * 3)
    dev = [[torch.from_numpy(im).cuda() for im in w["imgs"]] for w in wins]
    bt.build_pyramids(dpt.SLOT_REF, [d[0] for d in dev])
    for s, w in enumerate(wins):
        bt.set_reference_from_depth(s, n, torch.from_numpy(w["depth"]).cuda(), w["gts"][0])
        bt.set_pose_history(s, w["T_prev"], w["gts"][0])
    for j in range(1, WINDOW):
        bt.build_pyramids(dpt.SLOT_CUR, [d[j] for d in dev])
        bt.track_enqueue(None)
    got = bt.synchronize()
    assert len(got) == WINDOW - 1
    for s, w in enumerate(wins):
        trk = dpt.Tracker(cam, prm, max_points=n)
        _enqueue_window(dpt, trk, w, n, dev=dev[s])
        plain = trk.synchronize()
        for j in range(WINDOW - 1):
            rot, tr = oracle.pose_error(got[j][s]["T_cw"], plain[j]["T_cw"])
            assert rot < 1e-6 and tr < 1e-6  # same starts (both on the GPU): same iterates
            assert oracle.pose_error(plain[j]["T_cw"], w["gts"][j + 1])[0] < 2e-3


def test_workgroup_path_and_profile_counts(gpu_lib):
    dpt = gpu_lib
    d = synth.pair(2)
    cam, n = synth.CAM_640, 500
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    prm = dpt.make_params(levels=3)
    trk = dpt.Tracker(cam, prm, max_points=n)
    trk.set_launch_config(dpt.LAUNCH_WORKGROUP, 256)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    with pytest.raises(dpt.DptError):
        trk.track_enqueue(None)  # the constant-velocity start needs the cooperative track
    trk.track_enqueue(np.eye(4))  # runs synchronously on this path
    assert len(trk.synchronize()) == 1
    trk.set_launch_config(dpt.LAUNCH_COOP, 256)
    trk.set_profiling(True)
    for _ in range(3):
        trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
        trk.track_enqueue(np.eye(4))
    trk.synchronize()
    p = trk.profile()
    assert p["n_track"] == 3 and p["n_pyramid"] == 3
    assert p["track_ms"] > 0 and p["pyramid_ms"] > 0
    trk.set_profiling(True, every=4)  # launches 0, 4, 8 of the next 10 are timed
    for _ in range(10):
        trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
        trk.track_enqueue(np.eye(4))
    trk.synchronize()
    p = trk.profile()
    assert p["n_track"] == 3 and p["n_pyramid"] == 3
    assert p["track_ms"] > 0
    with pytest.raises(dpt.DptError):
        trk.set_profiling(True, every=-1)


def test_batch_reference_update_all_equals_per_stream(gpu_lib):
    """The one-launch-sequence reference update and history of every stream give
    the same caches and tracks as the per-stream calls."""
    import torch

    dpt = gpu_lib
    cams = [synth.CAM_752, synth.CAM_640, synth.CAM_752]
    n_pts = [1800, 700, 2000]
    wins = [_windows(1, seed=70 + s, cam=cams[s])[0] for s in range(3)]
    prm = dpt.make_params(levels=3)
    dev = [[torch.from_numpy(im).cuda() for im in w["imgs"]] for w in wins]
    depth = [torch.from_numpy(w["depth"]).cuda() for w in wins]
    res = []
    for mode in ("all", "each"):
        bt = dpt.BatchTracker(cams, prm, [2000] * 3)
        bt.build_pyramids(dpt.SLOT_REF, [d[0] for d in dev])
        if mode == "all":
            bt.set_reference_from_depth_all(n_pts, depth, np.stack([w["gts"][0] for w in wins]))
            bt.set_pose_history_all(np.stack([w["T_prev"] for w in wins]), np.stack([w["gts"][0] for w in wins]))
        else:
            for s, w in enumerate(wins):
                bt.set_reference_from_depth(s, n_pts[s], depth[s], w["gts"][0])
                bt.set_pose_history(s, w["T_prev"], w["gts"][0])
        for j in range(1, WINDOW):
            bt.build_pyramids(dpt.SLOT_CUR, [d[j] for d in dev])
            bt.track_enqueue(None)
        res.append(bt.synchronize())
    for j in range(WINDOW - 1):
        for s in range(3):
            np.testing.assert_array_equal(res[0][j][s]["T_cw"], res[1][j][s]["T_cw"])
            assert res[0][j][s]["n_valid_points"] == res[1][j][s]["n_valid_points"]
            assert oracle.pose_error(res[0][j][s]["T_cw"], wins[s]["gts"][j + 1])[0] < 2e-3
