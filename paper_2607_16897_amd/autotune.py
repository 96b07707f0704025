"""Launch-configuration autotuner for the track kernels.

For a tracker or batch whose reference maps and current pyramids are loaded,
time every candidate launch configuration (one workgroup per frame; cooperative
chunks of 64, 128 or 256 points per workgroup, one thread per point; chunks of 64
or 128 points with two threads per point) with the library's own HIP
event timing, check that the candidates agree on the poses, and keep the
fastest.  Choices are cached in a JSON file keyed by GPU architecture and a
shape bucket (streams, resolution mix, map-size bucket, levels, pattern size).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import LAUNCH_COOP, LAUNCH_COOP_PAIRS, LAUNCH_WORKGROUP

CANDIDATES = ((LAUNCH_WORKGROUP, 256), (LAUNCH_COOP, 64), (LAUNCH_COOP, 128), (LAUNCH_COOP, 256),
              (LAUNCH_COOP_PAIRS, 64), (LAUNCH_COOP_PAIRS, 128))
# the cooperative configurations only (the constant-velocity start computed on
# the GPU needs the cooperative track)
COOP_CANDIDATES = tuple(c for c in CANDIDATES if c[0] in (LAUNCH_COOP, LAUNCH_COOP_PAIRS))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dptrack", "autotune.json")


def arch_name() -> str:
    try:
        import torch

        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # pragma: no cover - no GPU
        return "unknown"


def shape_key(cams, n_points, levels: int, n_pattern: int) -> str:
    """Bucket: stream count, sorted distinct resolutions, log2 bucket of the mean and
    the largest map, levels, pattern size."""
    res = sorted({f"{c.width}x{c.height}" for c in cams})
    mean = float(np.mean(n_points)) if len(n_points) else 0.0
    b = lambda v: int(math.log2(max(v, 1.0)) * 2)  # half-octave buckets
    return (f"{arch_name()}|n={len(cams)}|res={','.join(res)}|mean={b(mean)}|max={b(max(n_points, default=0))}"
            f"|L={levels}|K={n_pattern}")


def _load(path):
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(tracker, T_init, key: str, reps: int = 5, cache: str | None = DEFAULT_CACHE, pose_tol: float = 1e-4,
         candidates=CANDIDATES):
    """Pick the fastest launch configuration for `tracker` (a Tracker or a
    BatchTracker, references and CUR pyramids already loaded) and apply it.

    T_init: start pose(s) passed to track().  Returns (mode, chunk, timings),
    timings = {"mode:chunk": median track ms}.  With a cache path, a stored
    choice for `key` is applied without timing."""
    if cache:
        stored = _load(cache).get(key)
        if stored and (stored["mode"], stored["chunk"]) in candidates:
            tracker.set_launch_config(stored["mode"], stored["chunk"])
            return stored["mode"], stored["chunk"], stored.get("timings", {})
    timings, poses = {}, {}
    tracker.set_profiling(True)
    try:
        for mode, chunk in candidates:
            try:
                tracker.set_launch_config(mode, chunk)
                res = tracker.track(T_init)
            except RuntimeError:
                continue  # not available for this shape (e.g. exceeds the co-resident capacity)
            ms = []
            for _ in range(reps):
                tracker.track(T_init)
                ms.append(tracker.last_kernel_ms()[1])
            timings[f"{mode}:{chunk}"] = float(np.median(ms))
            poses[(mode, chunk)] = [r["T_cw"] for r in (res if isinstance(res, list) else [res])]
    finally:
        tracker.set_profiling(False)
    if not timings:
        raise RuntimeError("no launch configuration ran")
    best = min(timings, key=timings.get)
    mode, chunk = (int(v) for v in best.split(":"))
    ref = poses[(mode, chunk)]
    for cfg, ps in poses.items():  # every candidate must reach the same poses
        for a, b in zip(ps, ref):
            if np.abs(a[:3] - b[:3]).max() > pose_tol * 10:
                raise RuntimeError(f"launch configuration {cfg} disagrees with {mode}:{chunk}")
    tracker.set_launch_config(mode, chunk)
    if cache:
        data = _load(cache)
        data[key] = {"mode": mode, "chunk": chunk, "timings": timings}
        _save(cache, data)
    return mode, chunk, timings
