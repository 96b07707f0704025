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


@pytest.mark.parametrize("launch", [(2, 256), (2, 64), (1, 256)])
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
