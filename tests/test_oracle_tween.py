"""Pins of the oracle's tween-window schedule (Sec. III, Sec. IV-D): the
decision rule on scripted outcomes, the window bookkeeping with a scripted
tracker, the constant-velocity start against a closed form, and two special
cases of a real run that reduce to fixed schedules."""
import numpy as np
import pytest

import oracle
import synth
from oracle import tween

POL = dict(max_cost=20.0, max_baseline=0.05, max_direct=3, n_points=300, margin=8)


def test_decide_rule_and_precedence():
    d = tween.decide
    assert d(oracle.OK, 5.0, 0.01, POL) == tween.DIRECT
    assert d(oracle.MAX_ITERS, 5.0, 0.01, POL) == tween.DIRECT        # the cap still returns a pose
    assert d(oracle.OK, 20.0, 0.01, POL) == tween.DIRECT              # at the threshold: accepted
    assert d(oracle.OK, 20.0001, 0.01, POL) == tween.COST
    assert d(oracle.OK, float("nan"), 0.01, POL) == tween.COST
    assert d(oracle.TOO_FEW_POINTS, 1.0, 0.0, POL) == tween.FAILED     # failure first
    assert d(oracle.NOT_PD, 1e9, 1e9, POL) == tween.FAILED
    assert d(oracle.OK, 1e9, 1e9, POL) == tween.COST                  # then the error
    assert d(oracle.OK, 5.0, 0.0501, POL) == tween.BASELINE           # then the baseline
    assert d(oracle.OK, 5.0, 1e9, dict(POL, max_baseline=0.0)) == tween.DIRECT  # disabled


def _pose(k, xi=np.array([0.002, -0.001, 0.003, 0.01, 0.0, -0.004])):
    return oracle.se3_exp(k * xi)


class _ScriptedRef:
    """Stands in for a reference: returns a scripted outcome per call and
    records the starts it was given."""

    def __init__(self, T, script, log):
        self.T_rw, self.script, self.log = T, script, log

    def track(self, img, start):
        self.log.append(start)
        status, cost, T = self.script.pop(0)
        return dict(status=status, final_cost=cost, T_cw=T)


def test_window_bookkeeping_with_scripted_tracker():
    """Anchors restart the count; MAX_FRAMES needs no track; every start is the
    constant-velocity prediction of the last two accepted or anchored poses,
    which on a constant-twist trajectory T_k = exp(k xi) is exactly T_k."""
    n = 10
    gts = [_pose(k) for k in range(n)]
    # frames 1-3 direct (their true poses), 4 max frames, 5 cost, 6-7 direct, 8 failed, 9 direct
    script = [(oracle.OK, 1.0, gts[1]), (oracle.OK, 1.0, gts[2]), (oracle.OK, 1.0, gts[3]),
              (oracle.OK, 99.0, gts[5]), (oracle.OK, 1.0, gts[6]), (oracle.OK, 1.0, gts[7]),
              (oracle.NOT_PD, 1.0, gts[8]), (oracle.OK, 1.0, gts[9])]
    starts, anchors = [], []

    def make(img, depth, T):
        anchors.append(T)
        return _ScriptedRef(T, script, starts)

    recs = tween.run([(None, None, g) for g in gts], dict(POL, max_baseline=0.0), make)
    assert [r["decision"] for r in recs] == [None, 0, 0, 0, tween.MAX_FRAMES, tween.COST, 0, 0, tween.FAILED, 0]
    assert len(anchors) == 4  # frames 0, 4, 5, 8
    tracked = [1, 2, 3, 5, 6, 7, 8, 9]
    for k, s in zip(tracked, starts):
        if k == 1:  # the first anchor seeds both history entries: the start is the anchor itself
            np.testing.assert_allclose(s, gts[0], atol=1e-12)
        else:
            np.testing.assert_allclose(s, gts[k], atol=1e-12)
    for k, r in enumerate(recs):
        np.testing.assert_allclose(r["pose"], gts[k], atol=1e-12)


def _frames(n, cam=synth.CAM_640, **kw):
    return [(im, d, T) for _, im, d, T, _ in synth.tween_frames(n_frames=n, cam=cam, **kw)]


def test_unlimited_error_gives_the_fixed_window():
    """With no error or baseline limit, the schedule is the fixed keyframe
    window: one anchor, then max_direct direct frames, repeated."""
    fr = _frames(14, p_jump=0.0, p_flicker=0.0)
    pol = dict(max_cost=float("inf"), max_baseline=0.0, max_direct=4, n_points=300, margin=8)
    recs = tween.run(fr, pol, tween.oracle_reference(synth.CAM_640, oracle.make_params(levels=3), pol))
    dec = [r["decision"] for r in recs]
    assert dec == [None, 0, 0, 0, 0, 4, 0, 0, 0, 0, 4, 0, 0, 0]
    s = tween.summary(recs, [f[2] for f in fr])
    assert s["counts"][0] == 11 and abs(s["direct_pct"] - 100 * 11 / 13) < 1e-9
    assert s["ate_max_m"] < 1e-2  # direct drift within a window stays at the mm level


def test_no_direct_frames_is_exact():
    fr = _frames(5, p_jump=0.0, p_flicker=0.0)
    pol = dict(max_cost=20.0, max_baseline=0.0, max_direct=0, n_points=300, margin=8)
    recs = tween.run(fr, pol, tween.oracle_reference(synth.CAM_640, oracle.make_params(levels=3), pol))
    assert [r["decision"] for r in recs[1:]] == [tween.MAX_FRAMES] * 4
    s = tween.summary(recs, [f[2] for f in fr])
    assert s["direct_pct"] == 0.0 and s["ate_rmse_m"] == 0.0


def test_flicker_is_rejected_by_the_error():
    """A frame with an exposure gain the photometric model cannot absorb
    exceeds the error threshold; it becomes the reference, so the next (normal)
    frame exceeds it too, and the one after tracks against a normal reference."""
    fr = _frames(8, p_jump=0.0, p_flicker=0.0)
    img, d, T = fr[5]
    fr[5] = (np.clip(np.rint(img * 1.3), 0, 255).astype(np.uint8), d, T)
    pol = dict(max_cost=20.0, max_baseline=0.0, max_direct=20, n_points=300, margin=8)
    recs = tween.run(fr, pol, tween.oracle_reference(synth.CAM_640, oracle.make_params(levels=3), pol))
    assert [r["decision"] for r in recs[1:]] == [0, 0, 0, 0, tween.COST, tween.COST, 0]
    assert recs[5]["track"]["final_cost"] > 5 * 20.0


def test_cv_start_is_rigid_and_exact():
    T0, T1 = _pose(3), _pose(4)
    S = tween.cv_start(T0, T1)
    np.testing.assert_allclose(S, _pose(5), atol=1e-12)
    np.testing.assert_allclose(S[:3, :3] @ S[:3, :3].T, np.eye(3), atol=1e-14)


def test_backproject_inverts_projection():
    cam = synth.CAM_640
    rng = np.random.default_rng(4)
    depth = rng.uniform(1.0, 4.0, (cam.height, cam.width))
    T = _pose(7)
    idx = rng.integers(0, cam.width * cam.height, 50)
    P = tween.backproject(cam, depth, idx, T).astype(np.float64)
    Pc = P @ T[:3, :3].T + T[:3, 3]
    y, x = np.divmod(idx, cam.width)
    np.testing.assert_allclose(cam.fx * Pc[:, 0] / Pc[:, 2] + cam.cx, x, atol=1e-3)
    np.testing.assert_allclose(cam.fy * Pc[:, 1] / Pc[:, 2] + cam.cy, y, atol=1e-3)
    np.testing.assert_allclose(Pc[:, 2], depth.reshape(-1)[idx], rtol=1e-6)
