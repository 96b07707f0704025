"""Batched streams (many independent cameras in one launch sequence) against the
single-stream tracker and the FP64 oracle, per stream."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL, COST_TOL = 1e-4, 1e-4, 1e-3


def _streams(n_streams, n_frames=2):
    out = []
    for s in range(n_streams):
        d = synth.stream_frames(s, n_frames=n_frames)
        d["n_points"] = min(d["n_points"], 3000)  # keep the oracle side quick
        idx = oracle.select_points(d["ref"], d["n_points"], 8)
        d["P"] = synth.backproject(d["cam"], d["depth"], idx, np.eye(4))
        d["idx"] = idx
        out.append(d)
    return out


@pytest.fixture(scope="module")
def streams():
    return _streams(6)


def _cmp(g, o):
    rot, tr = oracle.pose_error(g["T_cw"], o["T_cw"])
    rel = abs(g["final_cost"] - o["final_cost"]) / max(o["final_cost"], 1e-12)
    return rot, tr, rel


@pytest.mark.parametrize("launch", [(2, 256), (2, 64), (1, 256), (3, 128)])
@pytest.mark.parametrize("on_device", [True, False])
def test_batch_matches_oracle_and_plain(gpu_lib, streams, launch, on_device):
    import torch

    dpt = gpu_lib
    prm = dpt.make_params(levels=3)
    cams = [d["cam"] for d in streams]
    bt = dpt.BatchTracker(cams, prm, [d["n_points"] for d in streams])
    bt.set_launch_config(*launch)
    conv = (lambda x: torch.from_numpy(x).cuda()) if on_device else (lambda x: x)
    bt.build_pyramids(dpt.SLOT_REF, [conv(d["ref"]) for d in streams])
    for s, d in enumerate(streams):
        np.testing.assert_array_equal(bt.select_points(s, d["n_points"], 8), d["idx"])
        bt.set_reference_points(s, d["P"], np.eye(4))
    refs = [oracle.Reference(d["cam"], oracle.make_params(levels=3), d["ref"], d["P"], np.eye(4)) for d in streams]
    for f in range(2):
        bt.build_pyramids(dpt.SLOT_CUR, [conv(d["frames"][f]) for d in streams])
        res = bt.track(np.stack([np.eye(4)] * len(streams)))
        for s, d in enumerate(streams):
            o = refs[s].track(d["frames"][f], np.eye(4))
            rot, tr, rel = _cmp(res[s], o)
            assert res[s]["status"] == o["status"], (s, f)
            assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL, (s, f, rot, tr, rel)
    # plain single-stream context on one stream gives the same pose to rounding
    d = streams[0]
    trk = dpt.Tracker(d["cam"], prm, max_points=d["n_points"])
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(d["P"], np.eye(4))
    trk.build_pyramid(dpt.SLOT_CUR, d["frames"][1])
    g = trk.track(np.eye(4))
    rot, tr, rel = _cmp(res[0], g)
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


def test_batch_deterministic_and_reusable(gpu_lib, streams):
    dpt = gpu_lib
    prm = dpt.make_params(levels=3)
    bt = dpt.BatchTracker([d["cam"] for d in streams], prm, [d["n_points"] for d in streams])
    bt.build_pyramids(dpt.SLOT_REF, [d["ref"] for d in streams])
    for s, d in enumerate(streams):
        bt.set_reference_points(s, d["P"], np.eye(4))
    bt.build_pyramids(dpt.SLOT_CUR, [d["frames"][0] for d in streams])
    a = bt.track(np.stack([np.eye(4)] * len(streams)))
    b = bt.track(np.stack([np.eye(4)] * len(streams)))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x["T_cw"], y["T_cw"])
    # shrink one map: the launch groups are rebuilt
    bt.set_reference_points(2, streams[2]["P"][:100], np.eye(4))
    c = bt.track(np.stack([np.eye(4)] * len(streams)))
    assert c[2]["n_valid_points"] <= 100 and c[0]["iterations"] == a[0]["iterations"]
    # empty map on one stream: that stream reports too few points, the others are unaffected
    bt.set_reference_points(3, np.zeros((0, 3), np.float32), np.eye(4))
    e = bt.track(np.stack([np.eye(4)] * len(streams)))
    assert e[3]["status"] == dpt.TRACK_TOO_FEW_POINTS
    np.testing.assert_array_equal(e[0]["T_cw"], a[0]["T_cw"])


@pytest.mark.parametrize("precision", [0, 1])
def test_full_capacity_batch_equals_plain(gpu_lib, precision):
    """64 streams of 2000 points (8 chunks of 256 each, 512 workgroups: every
    co-resident slot of the device in one cooperative launch when the XCD
    packing balances) give, stream by stream, the poses of 64 plain contexts,
    frame by frame and as window tracks."""
    import torch

    dpt = gpu_lib
    cam, n, S = synth.CAM_752, 2000, 64
    traj, scene = [synth.Trajectory(7000 + s) for s in range(4)], [synth.Scene(7000 + s) for s in range(4)]
    seqs = []
    for s in range(4):
        img0, depth = scene[s].render(cam, traj[s].T_cw(30), synth.pixel_noise(s, 30, cam, 2.0), want_depth=True)
        frames = np.stack([scene[s].render(cam, traj[s].T_cw(30 + j), synth.pixel_noise(s, 30 + j, cam, 2.0),
                                           want_depth=False)[0] for j in (1, 2, 3)])
        seqs.append((img0, depth.astype(np.float32), frames, traj[s].T_cw(29), traj[s].T_cw(30)))
    prm = dpt.make_params(levels=4, precision=precision)
    bt = dpt.BatchTracker([cam] * S, prm, [n] * S)
    bt.set_launch_config(dpt.LAUNCH_COOP, 256)
    T_rw = np.stack([seqs[s % 4][4] for s in range(S)])
    T_prev = np.stack([seqs[s % 4][3] for s in range(S)])

    def refresh():
        bt.build_pyramids(dpt.SLOT_REF, [torch.from_numpy(seqs[s % 4][0]).cuda() for s in range(S)])
        bt.set_reference_from_depth_all([n] * S, [torch.from_numpy(seqs[s % 4][1]).cuda() for s in range(S)], T_rw)
        bt.set_pose_history_all(T_prev, T_rw)

    refresh()
    for j in range(3):
        bt.build_pyramids(dpt.SLOT_CUR, [torch.from_numpy(seqs[s % 4][2][j]).cuda() for s in range(S)])
        bt.track_enqueue(None)
    per_frame = bt.synchronize()
    refresh()
    bt.track_window_enqueue([torch.from_numpy(seqs[s % 4][2]).cuda() for s in range(S)])
    window = bt.synchronize()
    for j in range(3):
        for s in range(S):
            np.testing.assert_array_equal(per_frame[j][s]["T_cw"], window[j][s]["T_cw"])
    for q in range(4):  # streams q, q + 4, ... saw the same frames: one plain context per sequence
        t = dpt.Tracker(cam, prm, max_points=n)
        t.build_pyramid(dpt.SLOT_REF, seqs[q][0])
        t.set_reference_from_depth(n, seqs[q][1], seqs[q][4])
        t.set_pose_history(seqs[q][3], seqs[q][4])
        for j in range(3):
            t.build_pyramid(dpt.SLOT_CUR, seqs[q][2][j])
            t.track_enqueue(None)
        plain = t.synchronize()
        for j in range(3):
            assert plain[j]["status"] in (0, 1)
            for s in range(q, S, 4):
                np.testing.assert_array_equal(per_frame[j][s]["T_cw"], plain[j]["T_cw"])
                assert per_frame[j][s]["iterations"] == plain[j]["iterations"]
