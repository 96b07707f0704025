#!/usr/bin/env python3
"""Benchmark of the MI355X direct photometric tracker; prints one JSON line.

Workload (one GPU, one stream, plain FP32): the 752x480 sequence of the seeded
3-plane scene (fx = fy = 458, cx = 367, cy = 248), smooth 200 Hz trajectory,
Gaussian pixel noise sigma = 2, 4 pyramid levels, 2000 map points with the
8-pixel pattern, Huber k = 9, <= 10 iterations per level.  A step is one
keyframe window: the reference frame's pyramid, point selection and IC
precompute, then 9 frames each with its pyramid and coarse-to-fine track
(constant-velocity start from the previous estimates).  All frames are
resident in device memory before the timed region.

value = tracked frames / wall time (reference refreshes amortised in).
Residual samples/s counts every residual evaluated, final cost pass included.
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
# algorithmic bytes per residual sample of the FP32 track pass (K = 8): template
# intensity and gradient (3 x 4 B), the point's x0 shared by its 8 samples
# (12 B / 8) and four uint8 bilinear taps
BYTES_PER_SAMPLE_F32 = 12.0 + 12.0 / 8 + 4.0
PMC_FILE = os.path.join(ROOT, "profiles", "track_kernel_pmc.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2607_16897_amd", "csrc", "dpt_kernels.hip")

CAM = None  # set in main (synth.CAM_752)
LEVELS, N_POINTS, WINDOW = 4, 2000, 10


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def make_windows(n_windows: int, seed: int = 2607):
    """Render n_windows keyframe windows of the sequence (10 frames each)."""
    import synth

    traj = synth.Trajectory(seed)
    scene = synth.Scene(seed)
    wins = []
    for w in range(n_windows):
        k0 = WINDOW * w
        imgs, gts, depth = [], [], None
        for j in range(WINDOW):
            k = k0 + j
            T = traj.T_cw(k)
            img, dep = scene.render(CAM, T, synth.pixel_noise(seed, k, CAM, 2.0), want_depth=(j == 0))
            if j == 0:
                depth = dep
            imgs.append(img)
            gts.append(T)
        wins.append(dict(k0=k0, imgs=imgs, gts=gts, depth=depth, T_prev=traj.T_cw(k0 - 1)))
    return wins


def cv_init(prev2, prev1):
    """Constant-velocity prediction T_k = T_{k-1} T_{k-2}^-1 T_{k-1}."""
    return prev1 @ np.linalg.inv(prev2) @ prev1


def run_window_gpu(dpt, synth, trk, win, dev_imgs, stats):
    trk.build_pyramid(dpt.SLOT_REF, dev_imgs[0])
    idx = trk.select_points(N_POINTS, 8)
    P = synth.backproject(CAM, win["depth"], idx, win["gts"][0])
    trk.set_reference_points(P, win["gts"][0])
    prev2, prev1 = win["T_prev"], win["gts"][0]
    for j in range(1, WINDOW):
        trk.build_pyramid(dpt.SLOT_CUR, dev_imgs[j])
        r = trk.track(cv_init(prev2, prev1))
        prev2, prev1 = prev1, r["T_cw"]
        if stats is not None:
            pm, tm = trk.last_kernel_ms()
            stats["track_ms"].append(tm)
            stats["pyr_ms"].append(pm)
            stats["samples"].append(r["samples"])
            stats["iters"].append(r["iterations"])
            stats["status"].append(r["status"])
            stats["T"].append(r["T_cw"])
            stats["gt"].append(win["gts"][j])


def run_window_oracle(oracle, synth, win, prm):
    idx = oracle.select_points(win["imgs"][0], N_POINTS, 8)
    P = synth.backproject(CAM, win["depth"], idx, win["gts"][0])
    ref = oracle.Reference(CAM, prm, win["imgs"][0], P, win["gts"][0])
    prev2, prev1 = win["T_prev"], win["gts"][0]
    for j in range(1, WINDOW):
        r = ref.track(win["imgs"][j], cv_init(prev2, prev1))
        prev2, prev1 = prev1, r["T_cw"]


def cpu_baseline(wins, seconds: float):
    """The FP64 oracle, single thread, on the same windows until `seconds` elapse."""
    import oracle
    import synth

    prm = oracle.make_params(levels=LEVELS)
    t0 = time.perf_counter()
    n = 0
    while True:
        run_window_oracle(oracle, synth, wins[n % len(wins)], prm)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return dict(value=(WINDOW - 1) * n / el, unit="frames/s", cores=1, kind="oracle",
                sample=f"{n} keyframe windows ({(WINDOW - 1) * n} tracked frames) of the same sequence, "
                       f"{el:.1f} s, FP64 C oracle (gcc -O2) on one host thread")


def traffic_from_profile(samples_per_launch: float):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, or None if the
    kernel source changed since the counters were taken."""
    if not os.path.exists(PMC_FILE):
        return None
    d = json.load(open(PMC_FILE))
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def calibrate_copy(mib: int):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch

    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}))


def bench_batched_sequences(dpt, synth, n_streams: int, steps: int, warmup: int, n_win: int = 2):
    """n_streams independent sequences of the headline shape (752x480, 2000 points,
    4 levels, sigma = 2), stream s on its own scene and trajectory (seed 2607 + s),
    tracked together: a step is one keyframe window of every stream."""
    import torch

    from paper_2607_16897_amd import autotune

    t_r = time.perf_counter()
    wins = [make_windows(n_win, seed=2607 + s) for s in range(n_streams)]
    render_s = time.perf_counter() - t_r
    dev = [[[torch.from_numpy(im).cuda() for im in w["imgs"]] for w in ws] for ws in wins]
    torch.cuda.synchronize()
    prm = dpt.make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5)
    bt = dpt.BatchTracker([CAM] * n_streams, prm, [N_POINTS] * n_streams)
    stats = {"track_ms": [], "samples": [], "iters": [], "status": []}

    def window(w, record):
        bt.build_pyramids(dpt.SLOT_REF, [dev[s][w][0] for s in range(n_streams)])
        prev2, prev1 = [], []
        for s in range(n_streams):
            ws = wins[s][w]
            idx = bt.select_points(s, N_POINTS, 8)
            bt.set_reference_points(s, synth.backproject(CAM, ws["depth"], idx, ws["gts"][0]), ws["gts"][0])
            prev2.append(ws["T_prev"])
            prev1.append(ws["gts"][0])
        for j in range(1, WINDOW):
            bt.build_pyramids(dpt.SLOT_CUR, [dev[s][w][j] for s in range(n_streams)])
            res = bt.track(np.stack([cv_init(a, b) for a, b in zip(prev2, prev1)]))
            prev2, prev1 = prev1, [r["T_cw"] for r in res]
            if record:
                stats["track_ms"].append(bt.last_kernel_ms()[1])
                stats["samples"].append(sum(r["samples"] for r in res))
                stats["iters"].extend(r["iterations"] for r in res)
                stats["status"].extend(r["status"] for r in res)
        return prev1

    # autotune on the last frame of the first window, started from its estimates
    last = window(0, False)
    key = autotune.shape_key([CAM] * n_streams, [N_POINTS] * n_streams, LEVELS, 8)
    mode, chunk, timings = autotune.tune(bt, np.stack(last), key, cache=None)
    for w in range(warmup):
        window(w % n_win, False)
    bt.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(steps):
        window((warmup + st) % n_win, True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    bt.set_profiling(False)
    tracked = n_streams * (WINDOW - 1) * steps
    track_ms = float(np.mean(stats["track_ms"]))
    samp_launch = float(np.mean(stats["samples"]))
    achieved = samp_launch * BYTES_PER_SAMPLE_F32 / (track_ms * 1e-3) / 1e9
    return {"workload": f"{n_streams} independent 752x480 sequences, 2000 points each, 4 levels, sigma=2, "
                        "keyframe every 10 frames, FP32, tracked together",
            "value": round(tracked / el, 1), "unit": "frames/s", "samples_per_s": round(sum(stats["samples"]) / el, 1),
            "ms_per_step": round(el * 1e3 / steps, 4), "steps": steps,
            "launch": {"mode": mode, "chunk": chunk, "autotune_ms": timings},
            "track_launch_ms": round(track_ms, 5), "iterations_per_frame": round(float(np.mean(stats["iters"])), 3),
            "status_counts": {str(k): int(v) for k, v in zip(*np.unique(stats["status"], return_counts=True))},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 5), "samples_per_launch": round(samp_launch, 1)},
            "setup_render_s": round(render_s, 2)}


def bench_batched_mixed(dpt, synth, n_streams: int, n_frames: int, reps: int):
    """The mixed batch: stream s draws its resolution from {640x480, 752x480,
    1280x720} and its map size log-uniformly in [300, 8000]; each stream has one
    reference and n_frames perturbed views (<= 1 deg, <= 2 cm), identity start.
    Batched (one launch sequence per frame index) against the same tracks through
    one plain context per stream, run one after another."""
    import torch

    from paper_2607_16897_amd import autotune
    import oracle

    t_r = time.perf_counter()
    streams = [synth.stream_frames(s, n_frames=n_frames) for s in range(n_streams)]
    render_s = time.perf_counter() - t_r
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
    batched_T, samples = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        for f in range(n_frames):
            bt.build_pyramids(dpt.SLOT_CUR, [fr[f] for fr in dev_frames])
            res = bt.track(I)
            samples += sum(x["samples"] for x in res)
            if r == 0:
                batched_T.append([x["T_cw"] for x in res])
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    # plain: one context per stream, frames one after another
    plain = []
    for s, d in enumerate(streams):
        t = dpt.Tracker(d["cam"], prm, max_points=d["n_points"])
        t.build_pyramid(dpt.SLOT_REF, dev_ref[s])
        t.set_reference_points(pts[s], np.eye(4))
        plain.append(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_T = [[None] * n_streams for _ in range(n_frames)]
    for r in range(reps):
        for f in range(n_frames):
            for s in range(n_streams):
                plain[s].build_pyramid(dpt.SLOT_CUR, dev_frames[s][f])
                x = plain[s].track(np.eye(4))
                if r == 0:
                    plain_T[f][s] = x["T_cw"]
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    diff = max(max(oracle.pose_error(a, b)) for fa, fb in zip(batched_T, plain_T) for a, b in zip(fa, fb))
    tracked = n_streams * n_frames * reps
    return {"workload": f"{n_streams} streams, resolutions U{{640x480, 752x480, 1280x720}}, map sizes log-uniform "
                        f"300-8000 (total {sum(npts)} points), 3 levels, {n_frames} perturbed frames per stream",
            "batched_frames_per_s": round(tracked / t_b, 1), "plain_frames_per_s": round(tracked / t_p, 1),
            "speedup": round(t_p / t_b, 2), "batched_samples_per_s": round(samples / t_b, 1),
            "max_pose_diff_batched_vs_plain": diff, "launch": {"mode": mode, "chunk": chunk, "autotune_ms": timings},
            "setup_render_s": round(render_s, 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB")
    ap.add_argument("--launch", choices=["auto", "workgroup", "coop"], default="auto")
    ap.add_argument("--chunk", type=int, default=256)
    ap.add_argument("--batch-streams", type=int, default=64)
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (the tracker shards by stream, see DESIGN.md); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
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
    dev = [[torch.from_numpy(im).cuda() for im in w["imgs"]] for w in wins]
    torch.cuda.synchronize()

    prm = dpt.make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5)
    trk = dpt.Tracker(CAM, prm, max_points=N_POINTS)
    trk.set_launch_config({"auto": dpt.LAUNCH_AUTO, "workgroup": dpt.LAUNCH_WORKGROUP,
                           "coop": dpt.LAUNCH_COOP}[args.launch], args.chunk)
    for w in range(args.warmup):
        run_window_gpu(dpt, synth, trk, wins[w % n_render], dev[w % n_render], None)
    trk.set_profiling(True)
    stats = {k: [] for k in ("track_ms", "pyr_ms", "samples", "iters", "status", "T", "gt")}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        w = (args.warmup + s) % n_render
        run_window_gpu(dpt, synth, trk, wins[w], dev[w], stats)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    trk.set_profiling(False)

    tracked = args.steps * (WINDOW - 1)
    fps = tracked / elapsed
    coop = args.launch == "coop" or (args.launch == "auto" and N_POINTS <= 64 * args.chunk)
    track_kernel_name = f"coop_track_kernel<{args.chunk}>" if coop else "track_kernel<8,*>"
    samples = float(np.sum(stats["samples"]))
    track_ms = float(np.mean(stats["track_ms"]))
    samp_launch = float(np.mean(stats["samples"]))
    alg_bytes = samp_launch * BYTES_PER_SAMPLE_F32
    achieved = alg_bytes / (track_ms * 1e-3) / 1e9
    import oracle

    errs = np.array([oracle.pose_error(T, G) for T, G in zip(stats["T"], stats["gt"])])
    out = {
        "metric": METRIC,
        "value": round(fps, 2),
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
                   "tracked_frames_per_step": WINDOW - 1, "frames_per_step": WINDOW, "parallelism": "none"},
        "samples_per_s": round(samples / elapsed, 1),
        "roofline": {"kernel": track_kernel_name, "bound": "hbm", "achieved": round(achieved, 3),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": traffic_from_profile(samp_launch),
                     "bytes_per_launch_algorithmic": round(alg_bytes, 1), "samples_per_launch": round(samp_launch, 1),
                     "avg_launch_ms": round(track_ms, 5), "note": "single stream: one workgroup per frame, "
                     "latency-bound by the dependent Gauss-Newton chain"},
        "kernels_ms": {"track_kernel": round(track_ms, 5), "pyramid_kernel": round(float(np.mean(stats["pyr_ms"])), 5)},
        "iterations_per_frame": round(float(np.mean(stats["iters"])), 3),
        "status_counts": {str(k): int(v) for k, v in zip(*np.unique(stats["status"], return_counts=True))},
        "pose_error_vs_gt": {"rot_deg_median": round(float(np.rad2deg(np.median(errs[:, 0]))), 5),
                             "rot_deg_max": round(float(np.rad2deg(errs[:, 0].max())), 5),
                             "trans_mm_median": round(float(np.median(errs[:, 1]) * 1e3), 4),
                             "trans_mm_max": round(float(errs[:, 1].max() * 1e3), 4)},
        "setup_render_s": round(render_s, 2),
    }
    if not args.no_batched:
        out["batched"] = {
            "sequences": bench_batched_sequences(dpt, synth, args.batch_streams, max(2, args.steps // 4), 1),
            "mixed": bench_batched_mixed(dpt, synth, args.batch_streams, 4, 2),
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wins, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
