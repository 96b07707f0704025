"""GPU reference update from a depth map (dpt_set_reference_from_depth): point
selection, FP64 back-projection and the IC precompute all on the device,
against the oracle's selection, the host FP64 back-projection (the same
formula, written independently in synth.backproject) and the oracle's cache
and track on the same inputs."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL, COST_TOL = 1e-4, 1e-4, 1e-3


def _oparams(p):
    pat = np.array(p.pattern[:2 * p.n_pattern]).reshape(-1, 2)
    return oracle.make_params(levels=p.levels, max_iters=p.max_iters, huber_k=p.huber_k, step_eps=p.step_eps,
                              min_points=p.min_points, pattern=pat, z_min=p.z_min)


def _keyframe(cam, k_ref=40, k_cur=45, seed=2607):
    traj, scene = synth.Trajectory(seed), synth.Scene(seed)
    T_rw, T_cur = traj.T_cw(k_ref), traj.T_cw(k_cur)
    img, depth = scene.render(cam, T_rw, synth.pixel_noise(seed, k_ref, cam, 2.0), want_depth=True)
    cur, _ = scene.render(cam, T_cur, synth.pixel_noise(seed, k_cur, cam, 2.0), want_depth=False)
    return img, depth.astype(np.float32), cur, T_rw, T_cur, traj.T_cw(k_cur - 1)


@pytest.mark.parametrize("on_device", [True, False])
def test_depth_reference_matches_host_points(gpu_lib, on_device):
    import torch

    dpt = gpu_lib
    cam, n, levels = synth.CAM_752, 2000, 4
    img, depth, cur, T_rw, T_cur, T_prev = _keyframe(cam)
    prm = dpt.make_params(levels=levels)
    trk = dpt.Tracker(cam, prm, max_points=n)
    trk.build_pyramid(dpt.SLOT_REF, img)
    trk.set_reference_from_depth(n, torch.from_numpy(depth).cuda() if on_device else depth, T_rw)
    # oracle side: the same FP32 depths, back-projected in FP64 on the host
    idx = oracle.select_points(img, n, 8)
    P = synth.backproject(cam, depth.astype(np.float64), idx, T_rw)
    ref = oracle.Reference(cam, _oparams(prm), img, P, T_rw)
    for l in range(levels):
        g, o = trk.reference_cache(l), ref.cache(l)
        np.testing.assert_allclose(g["x0"], o["x0"], rtol=2e-6, atol=2e-6)
        assert (g["valid"] == o["refvalid"]).mean() > 0.995
        both = g["valid"] & o["refvalid"]
        np.testing.assert_allclose(g["I0"][both], o["I0"][both], atol=2e-3)
    trk.build_pyramid(dpt.SLOT_CUR, cur)
    r, w = trk.track(T_prev), ref.track(cur, T_prev)
    rot, tr = oracle.pose_error(r["T_cw"], w["T_cw"])
    assert rot < ROT_TOL and tr < TR_TOL
    assert abs(r["final_cost"] - w["final_cost"]) <= COST_TOL * w["final_cost"]
    assert oracle.pose_error(r["T_cw"], T_cur)[0] < 2e-3  # and it tracked the true motion


def test_depth_reference_invalid_depths_and_short_selection(gpu_lib):
    """Pixels with zero, negative or non-finite depth become never-valid points;
    asking for more points than there are candidates pads the map with invalid
    points after the selected ones."""
    dpt = gpu_lib
    cam = synth.Camera(96, 64, 80.0, 80.0, 48.0, 32.0)
    img, depth = synth.Scene(11).render(cam, np.eye(4), want_depth=True)
    depth = depth.astype(np.float32)
    m = 8
    C = (cam.width - 2 * m) * (cam.height - 2 * m)
    n = C + 40  # every candidate, then 40 padding entries
    idx = oracle.select_points(img, n, m)
    assert len(idx) == C
    bad = idx[::7]  # every 7th selected pixel loses its depth
    flat = depth.reshape(-1).copy()
    flat[bad[0::3]] = 0.0
    flat[bad[1::3]] = -1.0
    flat[bad[2::3]] = np.nan
    depth_bad = flat.reshape(depth.shape)
    prm = dpt.make_params(levels=1, pattern=((0, 0),), min_points=1)
    trk = dpt.Tracker(cam, prm, max_points=n)
    trk.build_pyramid(dpt.SLOT_REF, img)
    trk.set_reference_from_depth(n, depth_bad, np.eye(4), margin=m)
    g = trk.reference_cache(0)
    assert len(g["valid"]) == n
    good = np.ones(n, bool)
    good[np.arange(0, C, 7)] = False
    good[C:] = False
    assert not g["valid"][~good].any()
    # the points with depth: the same as the host back-projection
    P = synth.backproject(cam, depth.astype(np.float64), idx, np.eye(4))
    np.testing.assert_allclose(g["x0"][:C][good[:C]], P[good[:C]], rtol=2e-6, atol=2e-6)
    ref = oracle.Reference(cam, _oparams(prm), img, P[good[:C]], np.eye(4))
    np.testing.assert_array_equal(g["valid"][:C][good[:C]], ref.cache(0)["refvalid"])


def test_batch_depth_reference_equals_plain(gpu_lib):
    import torch

    dpt = gpu_lib
    cam, n = synth.CAM_752, 1500
    frames = [_keyframe(cam, k_ref=10 * s + 20, k_cur=10 * s + 23) for s in range(3)]
    prm = dpt.make_params(levels=4)
    bt = dpt.BatchTracker([cam] * 3, prm, [n] * 3)
    bt.build_pyramids(dpt.SLOT_REF, [torch.from_numpy(f[0]).cuda() for f in frames])
    for s, f in enumerate(frames):
        bt.set_reference_from_depth(s, n, torch.from_numpy(f[1]).cuda(), f[3])
    bt.build_pyramids(dpt.SLOT_CUR, [torch.from_numpy(f[2]).cuda() for f in frames])
    res = bt.track(np.stack([f[5] for f in frames]))
    for s, f in enumerate(frames):
        t = dpt.Tracker(cam, prm, max_points=n)
        t.build_pyramid(dpt.SLOT_REF, f[0])
        t.set_reference_from_depth(n, f[1], f[3])
        t.build_pyramid(dpt.SLOT_CUR, f[2])
        r = t.track(f[5])
        rot, tr = oracle.pose_error(res[s]["T_cw"], r["T_cw"])
        assert rot < 1e-5 and tr < 1e-5
        assert res[s]["iterations"] == r["iterations"]
