"""Tween-window schedule on the FP64 oracle tracker (test infrastructure).

Only the test suite and the benchmark's CPU-baseline leg use this module.  It
restates the schedule of the paper's Sec. III (a direct window of tween frames
per reference, a baseline criterion) and Sec. IV-D (a direct frame is accepted
when the tracker returns a valid pose and the robust photometric error stays
below the switching threshold; the indirect pipeline takes over when tracking
fails, the error exceeds the threshold, or the window reached its maximum
number of direct frames, and the frame it handles refreshes the reference).

Readings (the paper gives no values and no further detail):
  - one threshold on the mean Huber cost serves as both the switching and the
    failure threshold;
  - a pose counts as valid unless the track reports too few points or a
    singular system (reaching the iteration cap still returns a pose);
  - the baseline is the distance between camera centres of the direct estimate
    and the reference; max_baseline <= 0 disables it;
  - the indirect pipeline (ORB-SLAM2 in the paper) is stood in for by the
    frame's true pose and its depth, from which the new reference's map points
    are taken;
  - the direct start is the constant-velocity prediction T1 T0^-1 T1 from the
    last two accepted or anchored poses.
"""
from __future__ import annotations

import numpy as np

from . import OK, MAX_ITERS, Reference, make_camera, select_points

DIRECT, FAILED, COST, BASELINE, MAX_FRAMES = 0, 1, 2, 3, 4


def camera_centre(T) -> np.ndarray:
    T = np.asarray(T, np.float64)
    return -T[:3, :3].T @ T[:3, 3]


def decide(status: int, final_cost: float, baseline: float, policy: dict) -> int:
    """Decision for a frame that was tracked directly (Sec. IV-D)."""
    if status not in (OK, MAX_ITERS):
        return FAILED
    if not final_cost <= policy["max_cost"]:
        return COST
    if policy.get("max_baseline", 0.0) > 0.0 and baseline > policy["max_baseline"]:
        return BASELINE
    return DIRECT


def nearest_rotation(T) -> np.ndarray:
    """T with its rotation replaced by the nearest rotation matrix (SVD polar factor)."""
    T = np.array(T, np.float64)
    U, _, Vt = np.linalg.svd(T[:3, :3])
    T[:3, :3] = U @ Vt
    return T


def rigid_inverse(T) -> np.ndarray:
    T = np.asarray(T, np.float64)
    out = np.eye(4)
    out[:3, :3] = T[:3, :3].T
    out[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return out


def cv_start(T_older, T_newer) -> np.ndarray:
    return nearest_rotation(T_newer @ rigid_inverse(T_older) @ T_newer)


def backproject(cam, depth, idx, T_rw) -> np.ndarray:
    """World points of level-0 pixels idx (y W + x) at their depths: P = R^T (z K^-1 [x y 1]^T - t),
    FP64, rounded to FP32 (the map points a reference consumes)."""
    c = make_camera(cam)
    idx = np.asarray(idx, np.int64)
    y, x = np.divmod(idx, c.width)
    z = np.asarray(depth, np.float64).reshape(-1)[idx]
    Pc = np.stack([(x - c.cx) / c.fx * z, (y - c.cy) / c.fy * z, z], axis=1)
    R, t = np.asarray(T_rw)[:3, :3], np.asarray(T_rw)[:3, 3]
    return ((Pc - t) @ R).astype(np.float32)


def oracle_reference(cam, params, policy):
    """Reference factory for run(): the oracle tracker on the anchor frame's map."""
    def make(img, depth, T):
        idx = select_points(img, policy["n_points"], policy.get("margin", 8))
        return Reference(cam, params, img, backproject(cam, depth, idx, T), T)
    return make


def run(frames, policy: dict, make_reference):
    """frames: iterable of (image, depth, true T_cw).  The first frame anchors.
    Returns one record per frame: decision (None for an anchor-only first frame),
    pose (the accepted direct pose, else the true pose), the direct attempt's
    result (or None) and the start it used."""
    out = []
    ref = None
    hist = None  # the last two accepted or anchored poses, older first
    n_direct = 0
    for img, depth, T_gt in frames:
        T_gt = np.asarray(T_gt, np.float64)
        if ref is None:
            ref = make_reference(img, depth, T_gt)
            hist = (T_gt, T_gt)
            out.append(dict(decision=None, pose=T_gt, track=None, start=None, n_direct=0))
            continue
        rec = dict(track=None, start=None)
        if n_direct >= policy["max_direct"]:
            decision = MAX_FRAMES
        else:
            start = cv_start(*hist)
            r = ref.track(img, start)
            base = float(np.linalg.norm(camera_centre(r["T_cw"]) - camera_centre(ref.T_rw)))
            decision = decide(r["status"], r["final_cost"], base, policy)
            rec.update(track=r, start=start, baseline=base)
        if decision == DIRECT:
            n_direct += 1
            hist = (hist[1], np.asarray(rec["track"]["T_cw"], np.float64))
            rec.update(decision=decision, pose=hist[1], n_direct=n_direct)
        else:
            ref = make_reference(img, depth, T_gt)
            hist = (hist[1], T_gt)
            rec.update(decision=decision, pose=T_gt, n_direct=n_direct)
            n_direct = 0
        out.append(rec)
    return out


def summary(records, gts) -> dict:
    """Share of frames the direct tracker handled (the paper's Table III measure)
    and the RMSE / max of camera-centre errors against the true poses (an ATE
    analogue without alignment: both live in the same world frame)."""
    dec = [r["decision"] for r in records[1:]]
    err = [float(np.linalg.norm(camera_centre(r["pose"]) - camera_centre(g))) for r, g in zip(records, gts)]
    counts = {k: int(sum(d == k for d in dec)) for k in (DIRECT, FAILED, COST, BASELINE, MAX_FRAMES)}
    return dict(frames=len(dec), direct_pct=100.0 * counts[DIRECT] / max(len(dec), 1), counts=counts,
                ate_rmse_m=float(np.sqrt(np.mean(np.square(err)))), ate_max_m=float(np.max(err)))
