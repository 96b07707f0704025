#!/usr/bin/env python3
"""Benchmark of the MI355X direct photometric tracker; prints one JSON line.

Headline (`value`): tracked frames/s of the plain FP32 tracker on one stream of
the 752x480 sequence: seeded 3-plane scene (fx = fy = 458, cx = 367, cy = 248),
smooth 200 Hz trajectory, Gaussian pixel noise sigma = 2, 4 pyramid levels,
2000 map points with the 8-pixel pattern, Huber k = 9, <= 10 iterations per
level.  A step is one keyframe window: the reference frame's pyramid, point
selection, back-projection of the selected pixels from the keyframe's depth map
and IC precompute (all on the device), then 9 frames each with its pyramid and
coarse-to-fine track started from the constant-velocity prediction.  Frames and
keyframe depth maps are resident in device memory before the timed region;
reference refreshes are amortised into the rate.  Residual samples/s counts every residual evaluated,
the final cost pass included.

Further legs in the same line: batched streams (64 sequences of the headline
shape; the mixed-resolution 64-stream batch against the same tracks through
plain contexts), the mixed-precision variant (headline workload and a
1280x720 / 16k-point stress case), the fixed-H mode (the paper's constant-H
track on the headline workload), the paper's per-point shape (Gaussian FP32
pyramid, 6 levels, 7x7 patches), the tween-window schedule (share of direct
frames, camera-centre error), the learned initialiser against the
constant-velocity prior, and the FP64 oracle on the host (cpu_baseline), which
also tracks the first timed window of each leg from the same starts to give
the per-frame pose differences between the GPU path and the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tracked frames/s (752x480, 2k pts) and residual samples/s, batched vs plain"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per residual sample of the track pass (K = 8): template
# intensity and gradient (3 x 4 B in FP32, 3 x 2 B in FP16), the point's x0
# shared by its 8 samples (12 B / 8) and four uint8 bilinear taps
BYTES_PER_SAMPLE_F32 = 12.0 + 12.0 / 8 + 4.0
BYTES_PER_SAMPLE_MIXED = 6.0 + 12.0 / 8 + 4.0
PMC_FILE = os.path.join(ROOT, "profiles", "track_kernels_pmc.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2607_16897_amd", "csrc", f)
                  for f in ("dpt_coop.hip", "dpt_device.h", "dpt_internal.h")]

CAM = None  # synth.CAM_752, set in main
LAUNCH_NAME = {0: "auto", 2: "coop", 3: "pairs"}  # launch mode -> the --launch name
LEVELS, N_POINTS, WINDOW = 4, 2000, 10


def track_kernel_name(launch: str, chunk: int, window: bool, mixed: bool = False, fixed: bool = False) -> str:
    """The cooperative 8-pixel track kernel a launch configuration runs (as rocprofv3 names it)."""
    pairs = launch == "pairs"
    threads = 2 * chunk if pairs else chunk
    name = (f"coop_track_kernel<{threads}, {'true' if mixed else 'false'}, {'true' if fixed else 'false'}, false, "
            f"unsigned char, {'true' if window else 'false'}")
    return name + (", 2>" if pairs else ", 1>")


def kernel_source_hash() -> str:
    """Hash of the sources the cooperative track kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def pose_error(Ta, Tb):
    """(rotation angle in rad, translation in m) of Ta Tb^-1."""
    R = Ta[:3, :3] @ Tb[:3, :3].T
    t = Ta[:3, 3] - R @ Tb[:3, 3]
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    return float(np.arctan2(s, c)), float(np.linalg.norm(t))


def err_summary(errs):
    e = np.asarray(errs, np.float64).reshape(-1, 2)
    return {"rot_rad_max": float(e[:, 0].max()), "rot_rad_p99": float(np.percentile(e[:, 0], 99)),
            "rot_rad_median": float(np.median(e[:, 0])), "trans_m_max": float(e[:, 1].max()),
            "trans_m_p99": float(np.percentile(e[:, 1], 99)), "trans_m_median": float(np.median(e[:, 1]))}


def make_windows(n_windows: int, seed: int = 2607, cam=None):
    """Render n_windows keyframe windows of the sequence (10 frames each)."""
    import synth

    cam = cam or CAM
    traj = synth.Trajectory(seed)
    scene = synth.Scene(seed)
    wins = []
    for w in range(n_windows):
        k0 = WINDOW * w
        imgs, gts, depth = [], [], None
        for j in range(WINDOW):
            k = k0 + j
            T = traj.T_cw(k)
            img, dep = scene.render(cam, T, synth.pixel_noise(seed, k, cam, 2.0), want_depth=(j == 0))
            if j == 0:
                depth = dep
            imgs.append(img)
            gts.append(T)
        wins.append(dict(k0=k0, imgs=imgs, gts=gts, depth=depth.astype(np.float32), T_prev=traj.T_cw(k0 - 1)))
    return wins


def to_device(wins):
    """Frames and keyframe depth of every window as device tensors: the frames of
    a window in one [10, H, W] tensor (keyframe first), handed out as views."""
    import torch

    out = []
    for w in wins:
        stack = torch.from_numpy(np.stack(w["imgs"])).cuda()
        out.append(([stack[j] for j in range(len(w["imgs"]))], torch.from_numpy(w["depth"]).cuda(), stack))
    return out


def cv_init(prev2, prev1):
    """Constant-velocity prediction T_k = T_{k-1} T_{k-2}^-1 T_{k-1}."""
    return prev1 @ np.linalg.inv(prev2) @ prev1


def new_stats():
    return {k: [] for k in ("samples", "iters", "status", "T", "init", "gt")}


LOOKAHEAD = 8  # windows kept enqueued ahead: the oldest one's results are collected while the rest run
# Launches between two timed ones in the timed region: each HIP event record is a
# queue marker that holds the next kernel for several microseconds, so timing
# every launch would slow the stream by ~20 us per frame.
PROFILE_EVERY = 8
PROFILE_EVERY_WINDOW = 4  # window tracks: one launch per 9 frames


def enqueue_window(dpt, trk, win, dev, n_points, window=True):
    """One keyframe window, enqueued without waiting: the reference refresh
    (pyramid, selection, back-projection from the keyframe's depth and IC
    precompute, all on the device), the pose history (the frame before the
    keyframe and the keyframe, true poses), then the 9 tween frames, each
    tracked from the constant-velocity prediction of the two poses before it
    (computed on the GPU): window=True in one window track (one pyramid launch
    for the 9 frames, one track launch), else frame by frame (a pyramid and a
    track launch per frame).  Both give bitwise the same poses.
    dev = (device frames, device depth, the window's [10, H, W] frame stack)."""
    dev_imgs, dev_depth, stack = dev
    trk.build_pyramid(dpt.SLOT_REF, dev_imgs[0])
    trk.set_reference_from_depth(n_points, dev_depth, win["gts"][0])
    trk.set_pose_history(win["T_prev"], win["gts"][0])
    if window:
        trk.track_window_enqueue(stack[1:])
        return
    for j in range(1, WINDOW):
        trk.build_pyramid(dpt.SLOT_CUR, dev_imgs[j])
        trk.track_enqueue(None)


def collect(results, wins_done, stats):
    """Per-frame statistics of synchronised windows; the start of each frame is
    re-derived on the host (the same constant-velocity formula)."""
    k = 0
    for win in wins_done:
        prev2, prev1 = win["T_prev"], win["gts"][0]
        for j in range(1, WINDOW):
            r = results[k]
            k += 1
            T = np.array(r["T_cw"], np.float64).reshape(4, 4)
            stats["init"].append(cv_init(prev2, prev1))
            prev2, prev1 = prev1, T
            stats["samples"].append(int(r["samples"]))
            stats["iters"].append(int(r["iterations"]))
            stats["status"].append(int(r["status"]))
            stats["T"].append(T)
            stats["gt"].append(win["gts"][j])


REF_STREAM = True  # reference updates on a second stream (the --single-stream flag turns it off)
_REF_STREAM_OBJ = []


def reference_stream(dpt):
    """The one stream every leg's reference updates run on.  A process that
    used more streams than the GPU has hardware queues (4 here) ran all later
    kernels slower (the batched track 0.19 -> 0.28 ms after eight streams had
    each been used once), so the legs share one instead of taking a new one."""
    if not _REF_STREAM_OBJ:
        _REF_STREAM_OBJ.append(dpt.Stream())
    return _REF_STREAM_OBJ[0]


def timed_plain(dpt, synth, wins, dev, steps, warmup, prm, launch, chunk, n_points=N_POINTS, cam=None, window=True):
    """warmup + steps keyframe windows through one context, enqueued
    asynchronously (window tracks, or frame by frame); the first timed window is
    wins[warmup % len(wins)].  With REF_STREAM each keyframe's reference update
    runs on a second stream beside the previous window's tracks.  Returns
    (elapsed s, stats, profile totals of the timed region)."""
    import torch

    cam = cam or CAM
    trk = dpt.Tracker(cam, prm, max_points=n_points)
    trk.set_launch_config(launch, chunk)
    if REF_STREAM:
        trk.set_reference_stream(reference_stream(dpt))
    n = len(wins)
    every = PROFILE_EVERY if not window else PROFILE_EVERY_WINDOW
    for w in range(warmup):
        enqueue_window(dpt, trk, wins[w % n], dev[w % n], n_points, window)
    trk.synchronize()
    trk.set_profiling(True, every=every)
    stats = new_stats()
    done, results = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        w = (warmup + s) % n
        enqueue_window(dpt, trk, wins[w], dev[w], n_points, window)
        done.append(wins[w])
        if s >= LOOKAHEAD:  # the GPU keeps LOOKAHEAD windows while the host takes the oldest one's results
            results.append(trk.collect(WINDOW - 1, arrays=True))
    results.append(trk.synchronize(arrays=True))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = trk.profile()
    prof["frames_per_launch"] = WINDOW - 1 if window else 1
    trk.set_profiling(False)
    trk.close()
    collect(np.concatenate(results), done, stats)
    return el, stats, prof


def frame_track_ms(prof):
    """Track kernel time per frame: the average launch over the frames one launch tracks."""
    return prof["track_ms"] / prof["n_track"] / prof.get("frames_per_launch", 1)


# ---------------------------------------------------------------- batched legs
def batched_inputs(n_streams: int, n_win: int):
    """n_streams independent sequences of the headline shape, stream s on its own
    scene and trajectory (seed 2607 + s), n_win keyframe windows each, resident on
    the device.  Returns (wins, frames, wframes, depths, T_rw, T_prev, render s)."""
    import torch

    t_r = time.perf_counter()
    wins = [make_windows(n_win, seed=2607 + s) for s in range(n_streams)]
    render_s = time.perf_counter() - t_r
    # [frame index, stream, H, W] per window: a frame index's images are one
    # [streams, H, W] block, and a stream's frames sit at a constant stride;
    # one [streams, H, W] float32 depth tensor of the keyframes per window
    stacks = [torch.from_numpy(np.stack([np.stack([wins[s][w]["imgs"][j] for s in range(n_streams)])
                                         for j in range(WINDOW)])).cuda() for w in range(n_win)]
    frames = [[stacks[w][j] for j in range(WINDOW)] for w in range(n_win)]
    depths = [torch.from_numpy(np.stack([wins[s][w]["depth"] for s in range(n_streams)])).cuda()
              for w in range(n_win)]
    torch.cuda.synchronize()
    T_rw = [np.stack([wins[s][w]["gts"][0] for s in range(n_streams)]) for w in range(n_win)]
    T_prev = [np.stack([wins[s][w]["T_prev"] for s in range(n_streams)]) for w in range(n_win)]
    wframes = [[stacks[w][1:, s] for s in range(n_streams)] for w in range(n_win)]
    return wins, frames, wframes, depths, T_rw, T_prev, render_s


def bench_batched_sequences(dpt, synth, n_streams: int, steps: int, warmup: int, n_win: int = 2):
    """The sequences of batched_inputs tracked together: a step is one keyframe
    window of every stream.  Returns the FP32 result, and the same frames through
    the mixed-precision variant under "mixed_precision"."""
    wins, frames, wframes, depths, T_rw, T_prev, render_s = batched_inputs(n_streams, n_win)
    args = (dpt, wins, frames, wframes, depths, T_rw, T_prev, n_streams, steps, warmup, n_win)
    out = _batched_run(*args, dpt.PREC_FP32, True)
    out["frame_by_frame"] = _batched_run(*args, dpt.PREC_FP32, False, out["launch"])
    out["mixed_precision"] = _batched_run(*args, dpt.PREC_MIXED, True)
    out["mixed_precision"]["frame_by_frame"] = _batched_run(*args, dpt.PREC_MIXED, False,
                                                            out["mixed_precision"]["launch"])
    for o in (out, out["mixed_precision"]):  # the same tuned launch: bitwise the same poses
        o["poses_bitwise_equal_frame_by_frame"] = bool(np.array_equal(o.pop("poses"), o["frame_by_frame"].pop("poses")))
    out["setup_render_s"] = round(render_s, 2)
    return out


def _batched_run(dpt, wins, frames, wframes, depths, T_rw, T_prev, n_streams, steps, warmup, n_win, precision,
                 window, tuned=None):
    """One batched leg: window=True tracks each keyframe window's 9 frames of
    every stream in one window track, else frame by frame (one batched pyramid
    and track launch per frame).  tuned: the launch an earlier leg's autotuner
    chose (its "launch" entry), else tune here."""
    import torch

    from paper_2607_16897_amd import autotune

    mixed = precision == dpt.PREC_MIXED
    prm = dpt.make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5, precision=precision)
    bt = dpt.BatchTracker([CAM] * n_streams, prm, [N_POINTS] * n_streams)
    if REF_STREAM:  # each keyframe's reference updates overlap the previous window's tracks
        bt.set_reference_stream(reference_stream(dpt))
    stats = {"samples": [], "iters": [], "status": []}

    def enqueue(w, window=window):
        bt.build_pyramids(dpt.SLOT_REF, frames[w][0])
        bt.set_reference_from_depth_all(N_POINTS, depths[w], T_rw[w])
        bt.set_pose_history_all(T_prev[w], T_rw[w])
        if window:
            bt.track_window_enqueue(wframes[w])
            return
        for j in range(1, WINDOW):
            bt.build_pyramids(dpt.SLOT_CUR, frames[w][j])
            bt.track_enqueue(None)

    if tuned is None:  # tune on the last frame of the first window, started from the true poses
        enqueue(0, False)
        bt.synchronize()
        key = autotune.shape_key([CAM] * n_streams, [N_POINTS] * n_streams, LEVELS, 8)
        mode, chunk, timings = autotune.tune(bt, np.stack([wins[s][0]["gts"][WINDOW - 1] for s in range(n_streams)]),
                                             key, cache=None, candidates=autotune.COOP_CANDIDATES)
    else:
        mode, chunk, timings = tuned["mode"], tuned["chunk"], tuned["autotune_ms"]
        bt.set_launch_config(mode, chunk)
    for w in range(warmup):
        enqueue(w % n_win)
    bt.synchronize()
    bt.set_profiling(True, every=PROFILE_EVERY)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(steps):
        enqueue((warmup + st) % n_win)
        if st >= LOOKAHEAD:  # as in timed_plain
            results.append(bt.collect(WINDOW - 1, arrays=True))
    results.append(bt.synchronize(arrays=True))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = bt.profile()
    bt.set_profiling(False)
    bt.close()
    res = np.concatenate(results)  # (launches, streams)
    gts = np.stack([np.stack([wins[s][(warmup + st) % n_win]["gts"][j] for s in range(n_streams)])
                    for st in range(steps) for j in range(1, WINDOW)])
    errs = [pose_error(np.asarray(T).reshape(4, 4), G) for T, G in
            zip(res["T_cw"].reshape(-1, 16), gts.reshape(-1, 4, 4))]
    stats["samples"] = list(res["samples"].sum(axis=1))
    stats["iters"] = list(res["iterations"].reshape(-1))
    stats["status"] = list(res["status"].reshape(-1))
    tracked = n_streams * (WINDOW - 1) * steps
    fpl = WINDOW - 1 if window else 1
    track_ms = prof["track_ms"] / prof["n_track"]
    samp_launch = float(np.mean(stats["samples"])) * fpl
    achieved = samp_launch * (BYTES_PER_SAMPLE_MIXED if mixed else BYTES_PER_SAMPLE_F32) / (track_ms * 1e-3) / 1e9
    return {"workload": f"{n_streams} independent 752x480 sequences, 2000 points each, 4 levels, sigma=2, "
                        f"keyframe every 10 frames, {'mixed precision' if mixed else 'FP32'}, tracked together, "
                        f"{'one window track per keyframe window' if window else 'frame by frame'}",
            "value": round(tracked / el, 1), "unit": "frames/s", "samples_per_s": round(sum(stats["samples"]) / el, 1),
            "ms_per_step": round(el * 1e3 / steps, 4), "steps": steps,
            "track_launch_ms": round(track_ms, 5), "frames_per_launch_per_stream": fpl,
            "track_only_frames_per_s": round(n_streams * fpl / (track_ms * 1e-3), 1),
            "poses": res["T_cw"].copy(),
            "launch": {"mode": mode, "chunk": chunk, "autotune_ms": timings},
            "iterations_per_frame": round(float(np.mean(stats["iters"])), 3),
            "status_counts": {str(k): int(v) for k, v in zip(*np.unique(stats["status"], return_counts=True))},
            "pose_error_vs_gt": err_summary(errs),
            "roofline": {"kernel": track_kernel_name(LAUNCH_NAME.get(mode, "coop"), chunk, window, mixed),
                         "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 5), "samples_per_launch": round(samp_launch, 1),
                         "traffic": (traffic_from_profile("batched_mixed" if mixed else "batched_fp32",
                                                          {"mode": mode, "chunk": chunk}) if window else None)}}


def bench_batched_mixed(dpt, synth, n_streams: int, n_frames: int, reps: int, keep=None):
    """Mixed batch: stream s draws its resolution from {640x480, 752x480,
    1280x720} and its map size log-uniformly in [300, 8000]; one reference and
    n_frames perturbed views (<= 1 deg, <= 2 cm) each, identity start.  Batched
    against the same tracks through one plain context per stream, run one
    after another; both enqueued without host waits."""
    import torch

    from paper_2607_16897_amd import autotune

    from concurrent.futures import ThreadPoolExecutor

    t_r = time.perf_counter()
    with ThreadPoolExecutor(max(1, host_cpu()["share"])) as ex:  # the renderer's C calls release the GIL
        streams = list(ex.map(lambda s: synth.stream_frames(s, n_frames=n_frames), range(n_streams)))
    render_s = time.perf_counter() - t_r
    if keep is not None:  # the host baseline tracks the same streams
        keep.extend(streams)
    prm = dpt.make_params(levels=3, max_iters=10, huber_k=9.0, step_eps=1e-5)
    cams = [d["cam"] for d in streams]
    npts = [d["n_points"] for d in streams]
    dev_ref = [torch.from_numpy(d["ref"]).cuda() for d in streams]
    dev_frames = [[torch.from_numpy(f).cuda() for f in d["frames"]] for d in streams]
    bt = dpt.BatchTracker(cams, prm, npts)
    bt.build_pyramids(dpt.SLOT_REF, dev_ref)
    pts = []
    for s, d in enumerate(streams):
        idx = bt.select_points(s, d["n_points"], 8)
        pts.append(synth.backproject(d["cam"], d["depth"], idx, np.eye(4)))
        bt.set_reference_points(s, pts[-1], np.eye(4))
    I = np.stack([np.eye(4)] * n_streams)
    bt.build_pyramids(dpt.SLOT_CUR, [f[0] for f in dev_frames])
    key = autotune.shape_key(cams, npts, 3, 8)
    mode, chunk, timings = autotune.tune(bt, I, key, cache=None)
    # the chosen configuration's launch groups are built by its first track:
    # outside the timed region
    bt.track(I)
    # every frame is an independent pair tracked from the identity: all are
    # enqueued (each frame's pyramid build is ordered after the previous
    # frame's track), the results come back at the end
    bt.set_profiling(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        for f in range(n_frames):
            bt.build_pyramids(dpt.SLOT_CUR, [fr[f] for fr in dev_frames])
            bt.track_enqueue(I)
    res_all = bt.synchronize()
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    prof = bt.profile()
    bt.set_profiling(False)
    bt.close()
    samples = sum(x["samples"] for res in res_all for x in res)
    batched_T = [[x["T_cw"] for x in res] for res in res_all[:n_frames]]
    plain = []
    for s, d in enumerate(streams):
        t = dpt.Tracker(d["cam"], prm, max_points=d["n_points"])
        t.build_pyramid(dpt.SLOT_REF, dev_ref[s])
        t.set_reference_points(pts[s], np.eye(4))
        plain.append(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):  # the same frames through 64 plain contexts, enqueued alike
        for f in range(n_frames):
            for s in range(n_streams):
                plain[s].build_pyramid(dpt.SLOT_CUR, dev_frames[s][f])
                plain[s].track_enqueue(np.eye(4))
    plain_res = [t.synchronize() for t in plain]
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    plain_T = [[plain_res[s][f]["T_cw"] for s in range(n_streams)] for f in range(n_frames)]
    for t in plain:
        t.close()
    diff = max(max(pose_error(a, b)) for fa, fb in zip(batched_T, plain_T) for a, b in zip(fa, fb))
    tracked = n_streams * n_frames * reps
    track_ms = prof["track_ms"] / prof["n_track"]
    return {"workload": f"{n_streams} streams, resolutions U{{640x480, 752x480, 1280x720}}, map sizes log-uniform "
                        f"300-8000 (total {sum(npts)} points), 3 levels, {n_frames} perturbed frames per stream",
            "batched_frames_per_s": round(tracked / t_b, 1), "plain_frames_per_s": round(tracked / t_p, 1),
            "speedup": round(t_p / t_b, 2), "batched_samples_per_s": round(samples / t_b, 1),
            "track_launch_ms": round(track_ms, 5),
            "track_only_frames_per_s": round(n_streams / (track_ms * 1e-3), 1),
            "max_pose_diff_batched_vs_plain": diff, "launch": {"mode": mode, "chunk": chunk, "autotune_ms": timings},
            "setup_render_s": round(render_s, 2)}


# ---------------------------------------------------------------- precision legs
def bench_mixed_precision(dpt, synth, wins, dev, steps, launch, chunk):
    """The headline workload through the mixed-precision variant (FP16 template
    cache, Kahan-compensated FP32 sums, FP64 solve, exponential and pose)."""
    prm = dpt.make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5, precision=dpt.PREC_MIXED)
    el, st, prof = timed_plain(dpt, synth, wins, dev, steps, 1, prm, launch, chunk)
    track_ms = frame_track_ms(prof)
    achieved = float(np.mean(st["samples"])) * BYTES_PER_SAMPLE_MIXED / (track_ms * 1e-3) / 1e9
    out = {"workload": "the headline workload, mixed precision", "frames_per_s": round(steps * (WINDOW - 1) / el, 2),
           "track_ms_per_frame": round(track_ms, 5), "iterations_per_frame": round(float(np.mean(st["iters"])), 3),
           "pose_error_vs_gt": err_summary([pose_error(T, G) for T, G in zip(st["T"], st["gt"])]),
           "roofline": {"kernel": track_kernel_name(LAUNCH_NAME[launch], chunk, True, mixed=True), "bound": "hbm",
                        "unit": "GB/s", "peak": HBM_PEAK_GBS, "achieved": round(achieved, 3),
                        "frac": round(achieved / HBM_PEAK_GBS, 6),
                        "traffic": traffic_from_profile("mixed", {"mode": launch, "chunk": chunk})}}
    return out, st


def bench_fixed_h(dpt, synth, wins, dev, steps, launch, chunk):
    """The headline workload through the paper's own inverse-compositional track:
    per level a constant H reduced once per reference, only b and the cost
    reduced per iteration, no robust weights."""
    prm = dpt.make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5, fixed_h=True)
    el, st, prof = timed_plain(dpt, synth, wins, dev, steps, 1, prm, launch, chunk)
    track_ms = frame_track_ms(prof)
    iters = float(np.mean(st["iters"]))
    achieved = float(np.mean(st["samples"])) * BYTES_PER_SAMPLE_F32 / (track_ms * 1e-3) / 1e9
    out = {"workload": "the headline workload, fixed-H mode (constant H per level, b only, no weights)",
           "frames_per_s": round(steps * (WINDOW - 1) / el, 2), "track_ms_per_frame": round(track_ms, 5),
           "iterations_per_frame": round(iters, 3),
           "track_us_per_iteration": round(track_ms * 1e3 / (iters + 1), 3),
           "status_counts": {str(k): int(v) for k, v in zip(*np.unique(st["status"], return_counts=True))},
           "pose_error_vs_gt": err_summary([pose_error(T, G) for T, G in zip(st["T"], st["gt"])]),
           "roofline": {"kernel": track_kernel_name(LAUNCH_NAME[launch], chunk, True, fixed=True), "bound": "hbm",
                        "unit": "GB/s",
                        "peak": HBM_PEAK_GBS, "achieved": round(achieved, 3),
                        "frac": round(achieved / HBM_PEAK_GBS, 6),
                        "traffic": traffic_from_profile("fixed", {"mode": launch, "chunk": chunk})}}
    return out, st


def bench_paper_shape(dpt, synth, wins, dev, steps):
    """The paper's per-point shape on the headline sequence: the floating-point
    Gaussian pyramid, 6 levels, 7x7 patches (49 samples per point), 2000 points;
    cooperative generic-pattern track (four lanes per point), windows enqueued
    like the headline's but frame by frame (window tracks read box pyramids)."""
    prm = dpt.make_params(levels=6, max_iters=10, huber_k=9.0, step_eps=1e-5, gauss=True,
                          pattern=synth.square_pattern(7))
    el, st, prof = timed_plain(dpt, synth, wins, dev, steps, 1, prm, dpt.LAUNCH_AUTO, 256, window=False)
    track_ms = frame_track_ms(prof)
    samp = float(np.mean(st["samples"]))
    # per sample: 12 B of template and gradient, x0 shared by 49 samples, four FP32 taps
    bps = 12.0 + 12.0 / 49 + 16.0
    achieved = samp * bps / (track_ms * 1e-3) / 1e9
    out = {"workload": "the headline sequence at the paper's shape: FP32 Gaussian pyramid, 6 levels, 7x7 patches, "
                       "2000 points",
           "frames_per_s": round(steps * (WINDOW - 1) / el, 2), "track_ms_per_frame": round(track_ms, 5),
           "iterations_per_frame": round(float(np.mean(st["iters"])), 3),
           "samples_per_frame": round(samp, 1),
           "status_counts": {str(k): int(v) for k, v in zip(*np.unique(st["status"], return_counts=True))},
           "pose_error_vs_gt": err_summary([pose_error(T, G) for T, G in zip(st["T"], st["gt"])]),
           "roofline": {"kernel": "coop_track_kernel<256, false, false, true, float, false, 1>", "bound": "hbm",
                        "unit": "GB/s", "peak": HBM_PEAK_GBS, "bytes_per_sample": round(bps, 3),
                        "achieved": round(achieved, 3), "frac": round(achieved / HBM_PEAK_GBS, 6),
                        "traffic": traffic_from_profile("paper", {"mode": dpt.LAUNCH_AUTO, "chunk": 256})}}
    return out, st


TWEEN_POLICY = dict(max_cost=20.0, max_baseline=0.035, max_direct=12, n_points=N_POINTS, margin=8)


def bench_tween(dpt, synth, n_frames: int):
    """The tween-window schedule (Sec. III, Sec. IV-D) over a 752x480 sequence
    with exposure flicker and dropped frames; the true pose and depth stand in
    for the indirect pipeline whenever the schedule hands a frame back.  Frames
    and depths are resident in device memory; the rate covers direct tracks and
    re-anchoring (pyramid, selection, back-projection, precompute)."""
    import torch

    frames = [(im, d.astype(np.float32), T) for _, im, d, T, _ in
              synth.tween_frames(n_frames=n_frames, jump=(40, 160), p_jump=0.05)]
    dev = [(torch.from_numpy(im).cuda(), torch.from_numpy(d).cuda()) for im, d, _ in frames]
    p = TWEEN_POLICY

    def run():
        # a fresh context: its first anchor seeds both history entries, as in the oracle's schedule
        trk = dpt.Tracker(CAM, dpt.make_params(levels=LEVELS), max_points=N_POINTS)
        trk.tween_set_policy(p["max_cost"], p["max_direct"], p["n_points"], max_baseline=p["max_baseline"],
                             margin=p["margin"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = []
        trk.tween_anchor(dev[0][0], dev[0][1], frames[0][2])
        recs.append(dict(decision=None, pose=frames[0][2]))
        for k in range(1, len(frames)):
            r = trk.tween_frame(dev[k][0])
            if r["decision"] == dpt.TWEEN_DIRECT:
                recs.append(dict(decision=0, pose=r["track"]["T_cw"]))
            else:
                trk.tween_anchor(dev[k][0], dev[k][1], frames[k][2])
                recs.append(dict(decision=r["decision"], pose=frames[k][2]))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        trk.close()
        return recs, el

    run()  # warm-up
    recs, el = run()
    dec = [r["decision"] for r in recs[1:]]
    counts = {name: int(sum(d == v for d in dec)) for name, v in
              (("direct", 0), ("failed", 1), ("cost", 2), ("baseline", 3), ("max_frames", 4))}
    err = [pose_error(r["pose"], T)[1] for r, (_, _, T) in zip(recs, frames)]
    centre = lambda T: -T[:3, :3].T @ T[:3, 3]
    cerr = [float(np.linalg.norm(centre(np.asarray(r["pose"])) - centre(T))) for r, (_, _, T) in zip(recs, frames)]
    out = {"workload": f"{n_frames}-frame 752x480 sequence with exposure flicker (p=0.05, gain 1.15-1.35) and "
                       "dropped frames (p=0.05, jumps of 40-160 samples), 2000 points, 4 levels",
           "policy": p, "frames_per_s": round((len(frames) - 1) / el, 2),
           "direct_pct": round(100.0 * counts["direct"] / len(dec), 2), "decisions": counts,
           "centre_error_rmse_m": round(float(np.sqrt(np.mean(np.square(cerr)))), 7),
           "centre_error_max_m": round(float(np.max(cerr)), 7), "pose_translation_error_max_m": round(max(err), 7)}
    return out, frames, dec


def bench_stress(dpt, synth):
    """1280x720, 16000 points, 4 levels: one keyframe window of the sequence,
    tracked in FP32 and in mixed precision."""
    import torch

    cam = synth.CAM_1280
    wins = make_windows(1, cam=cam)
    dev = to_device(wins)
    out, raw = {}, {}
    for name, prec in (("fp32", dpt.PREC_FP32), ("mixed", dpt.PREC_MIXED)):
        prm = dpt.make_params(levels=4, max_iters=10, huber_k=9.0, step_eps=1e-5, precision=prec)
        el, st, prof = timed_plain(dpt, synth, wins, dev, 2, 1, prm, dpt.LAUNCH_COOP, 256, n_points=16000, cam=cam)
        out[name] = {"frames_per_s": round(2 * (WINDOW - 1) / el, 1),
                     "track_ms_per_frame": round(frame_track_ms(prof), 5),
                     "iterations_per_frame": round(float(np.mean(st["iters"])), 3),
                     "pose_error_vs_gt": err_summary([pose_error(T, G) for T, G in zip(st["T"], st["gt"])])}
        raw[name] = st
    return wins, out, raw


# ---------------------------------------------------------------- learned initialiser leg
# convolution FLOPs per pair of the initialiser's forward pass: 2 Ho Wo CO 9 CI per layer
CNN_LAYERS = ((2, 16, 30, 47), (16, 32, 15, 24), (32, 64, 8, 12), (64, 64, 4, 6))  # CI, CO, Ho, Wo
CNN_FWD_FLOP = [2 * ho * wo * co * 9 * ci for ci, co, ho, wo in CNN_LAYERS]
BF16_PEAK_TFLOPS = 2500.0


def bench_cnn_train(dpt, batch: int = 256, steps: int = 50):
    """Training steps of the initialiser on device-resident random pairs (the
    step of the 200k-pair training run: forward, loss, backward, Adam, and the
    loss read back).  Algorithmic FLOPs per step: the forward convolutions, the
    weight gradients (the same products) and the data gradients of layers 2-4."""
    import torch

    from paper_2607_16897_amd import initialiser as ini

    g = torch.Generator(device="cpu").manual_seed(5)
    pairs = torch.randint(0, 256, (batch, 2, 60, 94), dtype=torch.uint8, generator=g).cuda()
    tg = (torch.randn((batch, 6), generator=g) * 0.5).cuda()
    net = dpt.Cnn(max_batch=batch)
    net.set_params(ini.init_params(3))
    for _ in range(3):
        net.train_step(pairs, tg, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(pairs, tg, 1e-4)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    net.close()
    flop = batch * (3 * sum(CNN_FWD_FLOP) - CNN_FWD_FLOP[0])
    tf = flop / (ms * 1e-3) / 1e12
    return {"batch": batch, "steps": steps, "ms_per_step": round(ms, 4), "flop_per_step": flop,
            "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": BF16_PEAK_TFLOPS, "achieved": round(tf, 3),
                         "frac": round(tf / BF16_PEAK_TFLOPS, 6),
                         "note": "a 9.4 MFLOP-per-pair network: ~20 launches of 5-33 us of small-tile MFMA work, "
                                 "latency- and launch-bound; the step includes the loss read back to the host"}}


def bench_learned_init(dpt, n_streams: int, n_frames: int):
    from paper_2607_16897_amd import initialiser as ini

    wdir = os.path.join(ROOT, "paper_2607_16897_amd", "weights")
    net = dpt.Cnn(max_batch=n_streams)
    net.set_params(ini.load_checkpoint(os.path.join(wdir, "initialiser")))
    res = ini.evaluate(net, n_streams, n_frames, seed=99001)
    net.close()
    meta = json.load(open(os.path.join(wdir, "initialiser.json")))
    res["workload"] = (f"{n_streams} streams x {n_frames} frames at 752x480 on held-out scenes; the current pose "
                       "drifts up to 5 deg / 10 cm from the reference with per-frame jerks; batched tracking from "
                       "the BF16 CNN's proposal (computed and exponentiated on the GPU) vs the constant-velocity "
                       "prediction (on the GPU), every frame enqueued without a host wait")
    res["train_step"] = bench_cnn_train(dpt)
    res["training"] = {k: meta[k] for k in ("pairs", "epochs_run", "train_seconds", "val_loss", "dataset_seconds")}
    return res


# ---------------------------------------------------------------- CPU baseline (the oracle)
def host_cpu() -> dict:
    """The host the oracle runs on: CPU model, logical CPUs of the machine
    (nproc) and of this process's affinity mask, and the share of them the
    multi-threaded baseline uses: OMP_NUM_THREADS where the environment sets the
    process's CPU share that way, else every CPU of the affinity mask."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    share = affinity
    try:
        share = max(1, min(affinity, int(os.environ.get("OMP_NUM_THREADS", affinity))))
    except ValueError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": affinity, "share": share,
            "share_from": "OMP_NUM_THREADS" if "OMP_NUM_THREADS" in os.environ else "affinity"}


def cpu_baseline(wins, seconds: float, comparisons, tween_run=None, c3_streams=None):
    """The FP64 oracle on one host thread, on the headline windows until
    `seconds` elapse.  `comparisons` maps a leg name to (frames [(window, j)],
    starts, GPU poses, camera, windows, points, levels): the oracle tracks each
    of those frames from the same start for the pose differences.  With
    c3_streams (the mixed-resolution batch's streams), also that batch on every
    host core of the share, one stream per thread."""
    import oracle
    import synth

    prm = oracle.make_params(levels=LEVELS)
    t0 = time.perf_counter()
    n = 0
    while True:
        win = wins[n % len(wins)]
        idx = oracle.select_points(win["imgs"][0], N_POINTS, 8)
        ref = oracle.Reference(CAM, prm, win["imgs"][0], synth.backproject(CAM, win["depth"], idx, win["gts"][0]),
                               win["gts"][0])
        prev2, prev1 = win["T_prev"], win["gts"][0]
        for j in range(1, WINDOW):
            r = ref.track(win["imgs"][j], cv_init(prev2, prev1))
            prev2, prev1 = prev1, r["T_cw"]
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    out = {"value": round((WINDOW - 1) * n / el, 2), "unit": "frames/s", "cores": 1, "kind": "oracle",
           "sample": f"{n} keyframe windows ({(WINDOW - 1) * n} tracked frames) of the headline sequence in "
                     f"{el:.1f} s, FP64 C oracle (gcc -O2) on one host thread"}
    # the same windows on the host cores this GPU's process is given (one window per thread at a time;
    # the oracle's C calls release the interpreter lock), about a third as long
    from concurrent.futures import ThreadPoolExecutor

    host = host_cpu()
    threads = host["share"]

    def one_window(w):
        win = wins[w % len(wins)]
        idx = oracle.select_points(win["imgs"][0], N_POINTS, 8)
        ref = oracle.Reference(CAM, prm, win["imgs"][0], synth.backproject(CAM, win["depth"], idx, win["gts"][0]),
                               win["gts"][0])
        prev2, prev1 = win["T_prev"], win["gts"][0]
        for j in range(1, WINDOW):
            r = ref.track(win["imgs"][j], cv_init(prev2, prev1))
            prev2, prev1 = prev1, r["T_cw"]
        return WINDOW - 1

    t0 = time.perf_counter()
    done, w = 0, 0
    with ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < seconds / 3:
            done += sum(ex.map(one_window, range(w, w + threads)))
            w += threads
    el_all = time.perf_counter() - t0
    out["all_cores"] = {"value": round(done / el_all, 2), "unit": "frames/s", "cores": threads,
                        "sample": f"{done // (WINDOW - 1)} keyframe windows in {el_all:.1f} s, {threads} threads"}
    if c3_streams:
        p3 = oracle.make_params(levels=3)

        def one_stream(k):  # the stream's reference, then its frames from the identity, until the budget ends
            d = c3_streams[k % len(c3_streams)]
            idx = oracle.select_points(d["ref"], d["n_points"], 8)
            ref = oracle.Reference(d["cam"], p3, d["ref"], synth.backproject(d["cam"], d["depth"], idx, np.eye(4)),
                                   np.eye(4))
            n = 0
            for f in d["frames"]:
                if time.perf_counter() - t0 >= seconds / 3:
                    break
                ref.track(f, np.eye(4))
                n += 1
            return n

        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            done3 = sum(ex.map(one_stream, range(threads)))
        el3 = time.perf_counter() - t0
        out["c3_batch_all_cores"] = {
            "value": round(done3 / el3, 2), "unit": "frames/s", "cores": threads,
            "per_core": round(done3 / el3 / threads, 3),
            "sample": f"{done3} frames of the first {threads} mixed-resolution streams (one stream per thread, each "
                      f"its reference and then its frames from the identity) in {el3:.1f} s"}
    out["host"] = host
    diffs = {}
    for name, (frames, starts, poses, cam, wset, npts, levels, *extra) in comparisons.items():
        p = oracle.make_params(levels=levels, **(extra[0] if extra else {}))
        refs, errs = {}, []
        for (w, j), T0, Tg in zip(frames, starts, poses):
            if w not in refs:
                win = wset[w]
                idx = oracle.select_points(win["imgs"][0], npts, 8)
                refs[w] = oracle.Reference(cam, p, win["imgs"][0],
                                           synth.backproject(cam, win["depth"], idx, win["gts"][0]), win["gts"][0])
            errs.append(pose_error(Tg, refs[w].track(wset[w]["imgs"][j], T0)["T_cw"]))
        diffs[name] = dict(frames=len(errs), **err_summary(errs))
    if tween_run is not None:  # the oracle's schedule on the same frames: decisions must agree
        from oracle import tween

        frames, gpu_dec = tween_run
        recs = tween.run(frames, TWEEN_POLICY, tween.oracle_reference(CAM, oracle.make_params(levels=LEVELS),
                                                                      TWEEN_POLICY))
        s = tween.summary(recs, [f[2] for f in frames])
        odec = [r["decision"] for r in recs[1:]]
        diffs["tween_schedule"] = dict(frames=len(odec), same_decisions=int(sum(a == b for a, b in zip(odec, gpu_dec))),
                                       oracle_direct_pct=round(s["direct_pct"], 2),
                                       oracle_centre_error_rmse_m=round(s["ate_rmse_m"], 7))
    return out, diffs


def traffic_from_profile(leg, launch=None):
    """HBM bytes per track launch of a leg from the committed rocprofv3 PMC summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is none for the
    leg, the kernel sources changed since the counters were taken, or the leg now
    runs another launch configuration than the profiled one."""
    if not os.path.exists(PMC_FILE):
        return None
    e = json.load(open(PMC_FILE)).get("legs", {}).get(leg)
    if not e or e.get("kernel_source_sha") != kernel_source_hash():
        return None
    if launch is not None and e.get("launch") != launch:
        return None
    return e.get("bytes_per_launch")


# legs a --pmc-leg run can isolate: their track launches and nothing else of the bench
PMC_LEGS = ("headline", "headline_frame", "mixed", "fixed", "paper", "batched_fp32", "batched_mixed")


def pmc_leg(args, leg, meta_path):
    """Runs only `leg`'s track launches (warmup + steps keyframe windows, the
    launch configuration the bench measures the leg with), for rocprofv3 --pmc
    runs, and writes how many track launches it made to meta_path."""
    import torch

    import paper_2607_16897_amd as dpt
    import synth

    global CAM
    CAM = synth.CAM_752
    dpt.load()
    torch.cuda.set_device(0)
    launch = {"auto": dpt.LAUNCH_AUTO, "coop": dpt.LAUNCH_COOP, "pairs": dpt.LAUNCH_COOP_PAIRS}[args.launch]
    n_win = args.steps + args.warmup
    if leg.startswith("batched"):
        mode, chunk = args.batch_launch
        wins, frames, wframes, depths, T_rw, T_prev, _ = batched_inputs(args.batch_streams, 2)
        prec = dpt.PREC_MIXED if leg == "batched_mixed" else dpt.PREC_FP32
        _batched_run(dpt, wins, frames, wframes, depths, T_rw, T_prev, args.batch_streams, args.steps, args.warmup,
                     2, prec, True, {"mode": mode, "chunk": chunk, "autotune_ms": None})
        launches = n_win
    else:
        wins = make_windows(min(n_win, 24))
        dev = to_device(wins)
        kw = dict(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5)
        window, mode, chunk = leg != "headline_frame", launch, args.chunk
        if leg == "mixed":
            kw["precision"] = dpt.PREC_MIXED
        elif leg == "fixed":
            kw["fixed_h"] = True
        elif leg == "paper":
            kw.update(levels=6, gauss=True, pattern=synth.square_pattern(7))
            window, mode, chunk = False, dpt.LAUNCH_AUTO, 256
        timed_plain(dpt, synth, wins, dev, args.steps, args.warmup, dpt.make_params(**kw), mode, chunk,
                    window=window)
        launches = n_win * (1 if window else WINDOW - 1)
    torch.cuda.synchronize()
    with open(meta_path, "w") as f:
        json.dump({"leg": leg, "launches": launches, "launch": {"mode": mode, "chunk": chunk},
                   "steps": args.steps, "warmup": args.warmup}, f)
    print(f"# pmc leg {leg}: {launches} track launches", file=sys.stderr, flush=True)


def pmc_summary(leg, meta_path, copy_fetch_dir, copy_write_dir, *dirs):
    """Per track launch of `leg`: every counter that the rocprofv3 --pmc runs in
    `dirs` took on the track kernels (summed over the launch's dispatches: a batch
    track is one dispatch per launch group), with FETCH_SIZE and WRITE_SIZE (KiB)
    turned into HBM bytes by the factor the same counter reads for the plain copy
    of --calibrate-copy (bytes moved / counter bytes).  Adds the leg to the
    summary the roofline's `traffic` field reads and prints it."""
    import csv
    import glob

    meta = json.load(open(meta_path))
    if meta["leg"] != leg:
        raise SystemExit(f"{meta_path} describes leg {meta['leg']}, not {leg}")

    def rows(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        return list(csv.DictReader(open(f)))

    def copy_factor(d, counter):
        v = [float(r["Counter_Value"]) for r in rows(d) if r["Counter_Name"] == counter and "copyBuffer" in
             r["Kernel_Name"]]
        return COPY_MIB * (1 << 20) / (float(np.median(v)) * 1024.0)

    launches = meta["launches"]
    per_launch, kernels = {}, {}
    for d in dirs:
        for r in rows(d):
            if "track" not in r["Kernel_Name"]:
                continue
            c = r["Counter_Name"]
            per_launch[c] = per_launch.get(c, 0.0) + float(r["Counter_Value"]) / launches
            k = kernels.setdefault(r["Kernel_Name"], {})
            k.setdefault(c, set()).add((r["Dispatch_Id"], r["Grid_Size"]))
    disp = {name: {"dispatches": max(len(v) for v in k.values()),
                   "grid_sizes": sorted({int(g) for v in k.values() for _, g in v})} for name, k in kernels.items()}
    out = {"leg": leg, "launch": meta["launch"], "launches": launches, "kernels": disp,
           "counters_per_launch": {c: round(v, 3) for c, v in sorted(per_launch.items())},
           "kernel_source_sha": kernel_source_hash()}
    if "FETCH_SIZE" in per_launch and "WRITE_SIZE" in per_launch:
        ff, wf = copy_factor(copy_fetch_dir, "FETCH_SIZE"), copy_factor(copy_write_dir, "WRITE_SIZE")
        out["copy_scale"] = {"fetch": ff, "write": wf}
        out["fetch_bytes_per_launch"] = per_launch["FETCH_SIZE"] * 1024.0 * ff
        out["write_bytes_per_launch"] = per_launch["WRITE_SIZE"] * 1024.0 * wf
        out["bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    hit, miss = per_launch.get("TCC_HIT_sum"), per_launch.get("TCC_MISS_sum")
    if hit is not None and miss is not None and hit + miss > 0:
        out["l2_hit_rate"] = round(hit / (hit + miss), 5)
    summary = json.load(open(PMC_FILE)) if os.path.exists(PMC_FILE) else {}
    summary.setdefault("legs", {})[leg] = out
    with open(PMC_FILE, "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(out))


COPY_MIB = 256


def attainable_copy_gbs(mib: int = 1024, reps: int = 10) -> float:
    """Measured attainable HBM bandwidth: a plain device-to-device copy of `mib`
    MiB timed with events, bytes read plus bytes written per second (GB/s)."""
    import torch

    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def attainable_peaks(dpt) -> dict:
    """Measured roofs beside the published ones: HBM (a 1 GiB device copy), the
    L2 (every workgroup rereading one 2 MiB buffer that every XCD's L2 holds),
    the last-level cache (each of 8 workgroups per CU rereading its own 64 KiB,
    128 MiB in all: above the L2s, inside the 256 MB cache) and the FP32 FMA
    rate of the vector units as the library compiles (no packed FP32)."""
    n_wg = 8 * 256
    return {"hbm_copy_gbs": round(attainable_copy_gbs(), 1),
            "l2_read_gbs": round(dpt.probe_read_bandwidth(2 << 20, 1, 1), 1),
            "mall_read_gbs": round(dpt.probe_read_bandwidth(64 << 10, n_wg, 16), 1),
            "fp32_fma_tflops": round(dpt.probe_fp32_fma(4096), 2)}


def calibrate_copy(mib: int):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch

    n = mib << 20
    torch.cuda.set_device(0)
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}))


def decode_place(v: int) -> dict:
    """XCC id << 32 | HW_ID of gfx9: wave [3:0], SIMD [5:4], CU [11:8], SH [12], SE [15:13]."""
    hw = v & 0xFFFFFFFF
    return {"xcc": v >> 32, "se": (hw >> 13) & 7, "sh": (hw >> 12) & 1, "cu": (hw >> 8) & 15, "simd": (hw >> 4) & 3}


def cycle_split(args, legs):
    """Per-phase cycle split of the headline track (and, with the batched leg
    named, of the 64-stream window batch) from the instrumented library: mean
    cycles per Gauss-Newton iteration of thread 0 of each workgroup, over every
    launch of `steps` keyframe windows, and where each workgroup ran.  Prints one
    JSON line; the timings of an instrumented build are not the headline's."""
    os.environ.setdefault("DPT_LIBRARY", os.path.join(ROOT, "paper_2607_16897_amd", "libdptrack_cycles.so"))
    import torch

    import paper_2607_16897_amd as dpt
    import synth

    global CAM
    CAM = synth.CAM_752
    dpt.load()
    torch.cuda.set_device(0)
    wins = make_windows(min(args.steps + args.warmup, 24))
    dev = to_device(wins)
    out = {"library": os.path.basename(dpt.LIB_PATH), "workload": "headline: 752x480, 2000 points, 4 levels, "
           f"{'window' if args.mode == 'window' else 'frame-by-frame'} tracks of {args.steps} keyframe windows"}

    def summarise(rows, n_slots):
        used = rows[rows[:, 5] > 0]
        it = used[:, 4].astype(np.float64)
        per = {f: float(np.mean(used[:, k] / np.maximum(it, 1))) for k, f in enumerate(dpt.CYCLE_FIELDS[:4])}
        per["total"] = float(sum(per.values()))
        clock_mhz = float(np.mean(used[:, 6] / np.maximum(used[:, 7], 1)) * 100.0)
        places = [decode_place(int(v)) for v in used[:, 8]]
        cus = {(p["xcc"], p["se"], p["sh"], p["cu"]) for p in places}
        return {"cycles_per_iteration": per, "per_slot": {f: [round(float(x), 1) for x in used[:, k] / np.maximum(it, 1)]
                                                          for k, f in enumerate(dpt.CYCLE_FIELDS[:4])},
                "us_per_iteration_at_shader_clock": per["total"] / clock_mhz if clock_mhz > 0 else None,
                "polls_per_exchange": float(np.mean(used[:, 9] / np.maximum(it, 1))),
                "cycles_per_frame": {f: float(np.mean(used[:, k] / np.maximum(used[:, 13], 1)))
                                     for k, f in ((10, "frame_start"), (11, "level_starts"), (12, "final_pass"),
                                                  (14, "frame_end"))}
                | {"iterations": float(np.mean(used[:, 4] / np.maximum(used[:, 13], 1))),
                   "kernel": float(np.mean(used[:, 6] / np.maximum(used[:, 13], 1)))},
                "shader_clock_mhz": round(clock_mhz, 1), "workgroups": int(len(used)),
                "distinct_cus": len(cus), "xccs": sorted({p["xcc"] for p in places}), "places": places[:64]}

    launch = {"auto": dpt.LAUNCH_AUTO, "coop": dpt.LAUNCH_COOP, "pairs": dpt.LAUNCH_COOP_PAIRS}[args.launch]
    prm = dpt.make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5)
    dpt_slots = 1024
    dpt.cycle_profile(dpt_slots, reset=True)
    timed_plain(dpt, synth, wins, dev, args.steps, args.warmup, prm, launch, args.chunk, window=args.mode == "window")
    out["headline"] = summarise(dpt.cycle_profile(dpt_slots, reset=True), dpt_slots)
    if "batched" in legs:
        cams = [CAM] * args.batch_streams
        bt = dpt.BatchTracker(cams, prm, [N_POINTS] * args.batch_streams)
        bt.set_launch_config(dpt.LAUNCH_COOP, 256)
        for w in range(args.steps):
            win = wins[w % len(wins)]
            stack = dev[w % len(wins)][2]
            bt.build_pyramids(dpt.SLOT_REF, stack[0:1].expand(args.batch_streams, -1, -1).contiguous())
            depth = dev[w % len(wins)][1].unsqueeze(0).expand(args.batch_streams, -1, -1).contiguous()
            bt.set_reference_from_depth_all(N_POINTS, depth, np.stack([win["gts"][0]] * args.batch_streams))
            bt.set_pose_history_all(np.stack([win["T_prev"]] * args.batch_streams),
                                    np.stack([win["gts"][0]] * args.batch_streams))
            bt.track_window_enqueue(stack[1:].unsqueeze(0).expand(args.batch_streams, -1, -1, -1).contiguous())
            bt.synchronize()
        bt.close()
        out["batched_64_window"] = summarise(dpt.cycle_profile(dpt_slots, reset=True), dpt_slots)
        for k in ("per_slot", "places"):
            out["batched_64_window"].pop(k)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB")
    ap.add_argument("--launch", choices=["auto", "coop", "pairs"], default="pairs",
                    help="track launch (the GPU-side constant-velocity start needs the cooperative track); "
                         "pairs: cooperative with two threads per point (--chunk 64 or 128)")
    ap.add_argument("--chunk", type=int, default=128, help="points per chunk (pairs: 64 or 128)")
    ap.add_argument("--mode", choices=["window", "frame"], default="window",
                    help="headline launch form: one window track per keyframe window (9 frames, bitwise the same "
                         "poses) or frame by frame; the other form is measured beside it")
    ap.add_argument("--batch-streams", type=int, default=64)
    ap.add_argument("--single-stream", action="store_true",
                    help="reference updates on the context's own stream instead of a second one")
    ap.add_argument("--only-headline", action="store_true", help="skip the batched, precision, fixed-H and initialiser legs")
    ap.add_argument("--legs", default="mixed,fixed,paper,tween,batched,init",
                    help="legs after the headline: any of mixed, fixed, paper, tween, batched, init (comma separated)")
    ap.add_argument("--batch-launch", nargs=2, type=int, default=[2, 256], metavar=("MODE", "CHUNK"),
                    help="launch configuration of the batched legs under --pmc-leg (the bench tunes it)")
    ap.add_argument("--pmc-leg", choices=PMC_LEGS,
                    help="run only this leg's track launches (for rocprofv3 --pmc) and exit")
    ap.add_argument("--pmc-meta", default="pmc_meta.json", help="where --pmc-leg writes its launch count")
    ap.add_argument("--pmc-summary", nargs="+", metavar="ARG",
                    help="LEG META COPY_FETCH_DIR COPY_WRITE_DIR DIR...: add the leg's per-launch counters (HBM "
                         "traffic from FETCH_SIZE / WRITE_SIZE) from rocprofv3 --pmc output to the summary and exit")
    ap.add_argument("--cycle-split", action="store_true",
                    help="per-phase cycles per Gauss-Newton iteration from the instrumented library "
                         "(libdptrack_cycles.so) on the headline workload (and the batch with --legs batched); "
                         "prints that instead of the benchmark line")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent streams would shard across GPUs one process per GPU)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.pmc_summary:
        if len(args.pmc_summary) < 5:
            ap.error("--pmc-summary takes LEG META COPY_FETCH_DIR COPY_WRITE_DIR and at least one DIR")
        pmc_summary(*args.pmc_summary)
        return
    if args.pmc_leg:
        pmc_leg(args, args.pmc_leg, args.pmc_meta)
        return
    legs = set() if args.only_headline else set(x for x in args.legs.split(",") if x)
    global REF_STREAM
    REF_STREAM = not args.single_stream
    if args.cycle_split:
        cycle_split(args, legs)
        return

    import torch

    import paper_2607_16897_amd as dpt
    import synth

    global CAM
    CAM = synth.CAM_752
    dpt.load()
    torch.cuda.set_device(0)
    n_render = min(args.steps + args.warmup, 24)
    t_r = time.perf_counter()
    wins = make_windows(n_render)
    render_s = time.perf_counter() - t_r
    dev = to_device(wins)
    torch.cuda.synchronize()
    print(f"# rendered {n_render} windows in {render_s:.1f} s", file=sys.stderr, flush=True)

    launch = {"auto": dpt.LAUNCH_AUTO, "coop": dpt.LAUNCH_COOP, "pairs": dpt.LAUNCH_COOP_PAIRS}[args.launch]
    prm = dpt.make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5)
    window = args.mode == "window"
    elapsed, stats, prof = timed_plain(dpt, synth, wins, dev, args.steps, args.warmup, prm, launch, args.chunk,
                                       window=window)
    print(f"# headline leg done ({elapsed:.2f} s)", file=sys.stderr, flush=True)
    # the same windows frame by frame (a pyramid and a track launch per frame): the
    # rate of a live camera whose frames arrive one at a time
    el_f, st_f, prof_f = timed_plain(dpt, synth, wins, dev, args.steps, args.warmup, prm, launch, args.chunk,
                                     window=not window)
    same = bool(np.array_equal(np.asarray(stats["T"]), np.asarray(st_f["T"])))
    print(f"# other launch form done ({el_f:.2f} s)", file=sys.stderr, flush=True)

    tracked = args.steps * (WINDOW - 1)
    samples = float(np.sum(stats["samples"]))
    fpl = prof["frames_per_launch"]
    launch_ms = prof["track_ms"] / prof["n_track"]
    track_ms = launch_ms / fpl
    samp_launch = float(np.mean(stats["samples"])) * fpl
    alg_bytes = samp_launch * BYTES_PER_SAMPLE_F32
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    kname = track_kernel_name(args.launch, args.chunk, window)
    iters = float(np.mean(stats["iters"]))

    def pyr_ms(pr):  # None where the pyramids ran on the reference stream (not timed there)
        return round(pr["pyramid_ms"] / pr["n_pyramid"], 5) if pr["n_pyramid"] else None

    def form(el, st, pr, w):
        lm = pr["track_ms"] / pr["n_track"]
        return {"launch_form": "window" if w else "frame", "frames_per_s": round(tracked / el, 2),
                "track_launch_ms": round(lm, 5), "track_ms_per_frame": round(lm / pr["frames_per_launch"], 5),
                "pyramid_launch_ms": pyr_ms(pr),
                "kernel": track_kernel_name(args.launch, args.chunk, w)}

    att = attainable_peaks(dpt)  # after the timed region
    att_gbs = att["hbm_copy_gbs"]
    out = {
        "metric": METRIC,
        "value": round(tracked / elapsed, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "752x480 seeded 3-plane sequence, 2000 points, 8-px pattern, 4 levels, "
                               "Huber 9, <=10 iters/level, sigma=2 noise, keyframe every 10 frames, "
                               "plain FP32, one stream",
                   "tracked_frames_per_step": WINDOW - 1, "frames_per_step": WINDOW, "parallelism": "none",
                   "launch": args.launch, "chunk": args.chunk, "launch_form": args.mode},
        "samples_per_s": round(samples / elapsed, 1),
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 3),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": traffic_from_profile("headline" if window else "headline_frame",
                                                     {"mode": launch, "chunk": args.chunk}),
                     "attainable_copy": round(att_gbs, 1), "frac_of_attainable": round(achieved / att_gbs, 6),
                     "bytes_per_launch_algorithmic": round(alg_bytes, 1), "samples_per_launch": round(samp_launch, 1),
                     "frames_per_launch": fpl, "avg_launch_ms": round(launch_ms, 5),
                     "note": f"one launch tracks {fpl} frame(s); a single stream is latency-bound by its ~16 "
                             "dependent Gauss-Newton iterations per frame, each a grid-wide reduction"},
        "kernels_ms": {"track_kernel_per_launch": round(launch_ms, 5),
                       "pyramid_kernel_per_launch": pyr_ms(prof),
                       "pyramid_note": "window pyramids of a keyframe's first window are built on the reference "
                                       "stream behind its update and are not timed there (null)"},
        "track_only_frames_per_s": round(1.0 / (track_ms * 1e-3), 1),
        "iterations_per_frame": round(iters, 3),
        "track_us_per_iteration": round(track_ms * 1e3 / (iters + 1), 3),
        "status_counts": {str(k): int(v) for k, v in zip(*np.unique(stats["status"], return_counts=True))},
        "pose_error_vs_gt": err_summary([pose_error(T, G) for T, G in zip(stats["T"], stats["gt"])]),
        "launch_forms": {"this": form(elapsed, stats, prof, window), "other": form(el_f, st_f, prof_f, not window),
                         "poses_bitwise_equal": same},
        "setup_render_s": round(render_s, 2),
        "attainable": att,
    }
    nc = WINDOW - 1  # the first timed window of each leg is compared with the oracle
    comparisons = {"headline_fp32": ([(args.warmup % n_render, j) for j in range(1, WINDOW)], stats["init"][:nc],
                                     stats["T"][:nc], CAM, wins, N_POINTS, LEVELS)}
    if "mixed" in legs:
        mp, st_m = bench_mixed_precision(dpt, synth, wins, dev, max(4, args.steps // 2), launch, args.chunk)
        comparisons["headline_mixed"] = ([(1 % n_render, j) for j in range(1, WINDOW)], st_m["init"][:nc],
                                         st_m["T"][:nc], CAM, wins, N_POINTS, LEVELS)
        sw, so, sraw = bench_stress(dpt, synth)
        mp["stress_1280x720_16k"] = so
        for k, st in sraw.items():
            comparisons[f"stress_1280x720_16k_{k}"] = ([(0, j) for j in range(1, WINDOW)], st["init"][:nc],
                                                       st["T"][:nc], synth.CAM_1280, sw, 16000, 4)
        out["mixed_precision"] = mp
        print("# precision legs done", file=sys.stderr, flush=True)
    if "fixed" in legs:
        fh, st_f = bench_fixed_h(dpt, synth, wins, dev, max(4, args.steps // 2), launch, args.chunk)
        comparisons["headline_fixed_h"] = ([(1 % n_render, j) for j in range(1, WINDOW)], st_f["init"][:nc],
                                           st_f["T"][:nc], CAM, wins, N_POINTS, LEVELS, {"fixed_h": True})
        out["fixed_h"] = fh
        print("# fixed-H leg done", file=sys.stderr, flush=True)
    if "paper" in legs:
        ps, st_p = bench_paper_shape(dpt, synth, wins, dev, max(4, args.steps // 4))
        comparisons["paper_shape"] = ([(1 % n_render, j) for j in range(1, WINDOW)], st_p["init"][:nc],
                                      st_p["T"][:nc], CAM, wins, N_POINTS, 6,
                                      {"gauss": True, "pattern": synth.square_pattern(7)})
        out["paper_shape"] = ps
        print("# paper-shape leg done", file=sys.stderr, flush=True)
    tween_run = None
    if "tween" in legs:
        out["tween"], tw_frames, tw_dec = bench_tween(dpt, synth, 200)
        tween_run = (tw_frames, tw_dec)
        print("# tween leg done", file=sys.stderr, flush=True)
    c3_keep = []
    if "batched" in legs:
        out["batched"] = {
            "sequences": bench_batched_sequences(dpt, synth, args.batch_streams, max(2, args.steps // 4), 1),
            "mixed": bench_batched_mixed(dpt, synth, args.batch_streams, 32, 3, keep=c3_keep),
        }
        for o in (out["batched"]["sequences"], out["batched"]["sequences"]["mixed_precision"]):
            r = o["roofline"]  # the window launches' working set lives in L2 and the last-level cache
            r["frac_of_l2_read"] = round(r["achieved"] / att["l2_read_gbs"], 5)
            r["frac_of_mall_read"] = round(r["achieved"] / att["mall_read_gbs"], 5)
        print("# batched legs done", file=sys.stderr, flush=True)
    if "init" in legs:
        out["learned_init"] = bench_learned_init(dpt, args.batch_streams, 100)
        print("# initialiser leg done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["pose_diff_vs_oracle"] = cpu_baseline(wins, args.cpu_seconds, comparisons,
                                                                        tween_run, c3_keep)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
