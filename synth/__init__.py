"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

Input generation only: three textured planes (y=-1, z=3, x=2 in the world
frame, which is the first reference camera's frame: x right, y down, z
forward) ray-cast into a pinhole camera, camera trajectories, perturbations,
pixel noise and the back-projection of chosen pixels to 3-D map points.  None
of the tracking method's arithmetic lives here: pyramids, point selection,
sampling, Jacobians, weighting and the solve belong to the oracle and to the
HIP library, which never import each other.

Random numbers come from ``numpy.random.default_rng`` (PCG64) and are passed
to the C renderer as explicit arrays; the value-noise lattice uses a
counter-based splitmix64 hash of (seed, plane, ix, iy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the renderer with gcc + OpenMP into synth/libsynth.so."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-Werror",
               os.path.join(_HERE, "render.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_GPU_LIB_PATH = os.path.join(_HERE, "libsynth_gpu.so")
_gpu_lib = None


def build_gpu(force: bool = True) -> str:
    """Compile the GPU port of the renderer (training-set generation) for gfx950."""
    if force or not os.path.exists(_GPU_LIB_PATH):
        cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               os.path.join(_HERE, "render_gpu.hip"), "-o", _GPU_LIB_PATH + ".tmp"]
        subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
        os.replace(_GPU_LIB_PATH + ".tmp", _GPU_LIB_PATH)
    return _GPU_LIB_PATH


def render_gpu(scene: "Scene", cam: "Camera", poses: np.ndarray, imgs, depths=None, stream: int = 0):
    """Render len(poses) views of `scene` on the GPU into torch uint8 tensor `imgs`
    [views, H, W] (and float32 `depths`, optional).  Noiseless."""
    global _gpu_lib
    if _gpu_lib is None:
        build_gpu(force=False)
        import torch  # noqa: F401  (bind to PyTorch's HIP runtime, one per process)

        _gpu_lib = ctypes.CDLL(_GPU_LIB_PATH)
        _gpu_lib.syn_gpu_render.restype = ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        _gpu_lib.syn_gpu_render.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, dp, ctypes.c_int32, ctypes.c_int32,
                                            dp, dp, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    P = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(-1, 16))
    assert tuple(imgs.shape) == (len(P), cam.height, cam.width) and imgs.is_contiguous()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _gpu_lib.syn_gpu_render(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, P.ctypes.data_as(dp), len(P),
                                 scene.blobs.shape[1], scene.blobs.ctypes.data_as(dp),
                                 np.ascontiguousarray(_WINDOWS).ctypes.data_as(dp), scene.noise_seed,
                                 scene.noise_amp, scene.noise_cell, imgs.data_ptr(),
                                 depths.data_ptr() if depths is not None else None, stream)
    if rc != 0:
        raise RuntimeError(f"GPU render failed ({rc})")


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.syn_render.restype = ctypes.c_int
        lib.syn_render.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, dp, ctypes.c_int32, dp, dp,
                                   ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint8), dp]
        _lib = lib
    return _lib


# --------------------------------------------------------------------------- cameras
@dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def K(self) -> np.ndarray:
        return np.array([[self.fx, 0, self.cx], [0, self.fy, self.cy], [0, 0, 1.0]])


CAM_640 = Camera(640, 480, 460.0, 460.0, 320.0, 240.0)   # single-pair workload
CAM_752 = Camera(752, 480, 458.0, 458.0, 367.0, 248.0)   # sequence workload
CAM_1280 = Camera(1280, 720, 920.0, 920.0, 640.0, 360.0)  # keeps the 640 camera's horizontal FOV
RESOLUTIONS = (CAM_640, CAM_752, CAM_1280)

# pattern used throughout: point-symmetric radius-2 diamond, same offsets at every level
PATTERN8 = np.array([(-2, 0), (2, 0), (0, -2), (0, 2), (-1, -1), (1, -1), (-1, 1), (1, 1)], dtype=np.int32)


def square_pattern(p: int) -> np.ndarray:
    """p x p patch offsets (p odd), row-major."""
    h = p // 2
    return np.array([(dx, dy) for dy in range(-h, h + 1) for dx in range(-h, h + 1)], dtype=np.int32)


# --------------------------------------------------------------------------- poses (generation only)
def pose_matrix(R: np.ndarray, t) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def rigid_inverse(T: np.ndarray) -> np.ndarray:
    R = T[:3, :3]
    return pose_matrix(R.T, -R.T @ T[:3, 3])


def random_perturbation(rng: np.random.Generator, max_deg: float, max_m: float) -> np.ndarray:
    """Rotation: axis uniform on S^2, angle U(0, max_deg); translation: direction
    uniform, magnitude U(0, max_m).  Built with scipy's rotation-vector map."""
    from scipy.spatial.transform import Rotation

    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = np.deg2rad(rng.uniform(0.0, max_deg))
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    mag = rng.uniform(0.0, max_m)
    return pose_matrix(Rotation.from_rotvec(axis * ang).as_matrix(), d * mag)


# --------------------------------------------------------------------------- scene
_WINDOWS = np.array([[-4.0, 4.0, -1.0, 6.0],    # floor (x, z)
                     [-6.0, 6.0, -4.0, 4.0],    # wall (x, y)
                     [-1.0, 6.0, -4.0, 4.0]])   # side (z, y)


class Scene:
    """Seeded 3-plane textured scene: 200 Gaussian blobs per plane plus value noise."""

    def __init__(self, seed: int, n_blobs: int = 200, noise_amp: float = 12.0, noise_cell: float = 0.02):
        rng = np.random.default_rng(seed)
        blobs = np.empty((3, n_blobs, 4))
        for p in range(3):
            blobs[p, :, 0] = rng.uniform(-90.0, 90.0, n_blobs)
            blobs[p, :, 1] = rng.uniform(0.05, 0.40, n_blobs)
            blobs[p, :, 2] = rng.uniform(_WINDOWS[p, 0], _WINDOWS[p, 1], n_blobs)
            blobs[p, :, 3] = rng.uniform(_WINDOWS[p, 2], _WINDOWS[p, 3], n_blobs)
        self.seed = seed
        self.blobs = np.ascontiguousarray(blobs)
        self.noise_seed = int(rng.integers(0, 2**63 - 1))
        self.noise_amp = noise_amp
        self.noise_cell = noise_cell

    def render(self, cam: Camera, T_cw: np.ndarray, noise: np.ndarray | None = None,
               want_depth: bool = True):
        lib = _load()
        img = np.empty((cam.height, cam.width), np.uint8)
        depth = np.empty((cam.height, cam.width), np.float64) if want_depth else None
        T = np.ascontiguousarray(T_cw, dtype=np.float64)
        nz = None
        if noise is not None:
            noise = np.ascontiguousarray(noise, dtype=np.float32)
            assert noise.shape == img.shape
            nz = noise.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        dp = ctypes.POINTER(ctypes.c_double)
        misses = lib.syn_render(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                                T.ctypes.data_as(dp), self.blobs.shape[1], self.blobs.ctypes.data_as(dp),
                                np.ascontiguousarray(_WINDOWS).ctypes.data_as(dp), self.noise_seed,
                                self.noise_amp, self.noise_cell, nz,
                                img.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                depth.ctypes.data_as(dp) if depth is not None else None)
        if misses:
            raise RuntimeError(f"{misses} pixels hit no plane")
        return img, depth


def backproject(cam: Camera, depth: np.ndarray, idx: np.ndarray, T_rw: np.ndarray) -> np.ndarray:
    """World points of the given level-0 pixel indices (y*W + x) from exact depth,
    computed in FP64 and rounded to FP32 (the map points both sides consume)."""
    idx = np.asarray(idx, np.int64)
    y, x = np.divmod(idx, cam.width)
    z = depth.reshape(-1)[idx]
    if np.any(z <= 0):
        raise ValueError("selected pixel without depth")
    Pc = np.stack([(x - cam.cx) / cam.fx * z, (y - cam.cy) / cam.fy * z, z], axis=1)
    R, t = T_rw[:3, :3], T_rw[:3, 3]
    Pw = (Pc - t) @ R  # R^T (Pc - t), row-vector form
    return np.ascontiguousarray(Pw.astype(np.float32))


def pixel_noise(seed, frame: int, cam: Camera, sigma: float) -> np.ndarray:
    rng = np.random.default_rng([int(seed), int(frame), 77])
    return rng.normal(0.0, sigma, (cam.height, cam.width)).astype(np.float32)


# --------------------------------------------------------------------------- workloads
def pair(seed: int, cam: Camera = CAM_640, max_deg: float = 1.0, max_m: float = 0.02, noise_sigma: float = 0.0):
    """Single reference/current pair: reference at identity, current after a seeded
    SE(3) perturbation (rotation <= max_deg, translation <= max_m)."""
    scene = Scene(seed)
    T_rw = np.eye(4)
    ref, depth = scene.render(cam, T_rw, pixel_noise(seed, 0, cam, noise_sigma) if noise_sigma > 0 else None)
    rng = np.random.default_rng([seed, 1])
    T_cw = random_perturbation(rng, max_deg, max_m)
    cur, _ = scene.render(cam, T_cw, pixel_noise(seed, 1, cam, noise_sigma) if noise_sigma > 0 else None,
                          want_depth=False)
    return dict(scene=scene, cam=cam, ref=ref, cur=cur, depth=depth, T_rw=T_rw, T_cw_gt=T_cw)


class Trajectory:
    """Smooth seeded trajectory: periodic cubic spline through 12 waypoints
    (x in [-0.8, 0.8], y in [-0.4, 0.4], z in [-1.0, 0.8]) traversed at constant
    speed, orientations slerped between per-waypoint yaw/pitch/roll keys
    (+-15, +-8, +-5 deg), redrawn until every segment turns at <= max_rate deg/s."""

    def __init__(self, seed: int = 2607, rate_hz: float = 200.0, speed: float = 0.5, n_way: int = 12,
                 max_rate_dps: float = 30.0):
        from scipy.interpolate import CubicSpline
        from scipy.spatial.transform import Rotation, Slerp

        rng = np.random.default_rng(seed)
        for _ in range(10000):
            P = np.column_stack([rng.uniform(-0.8, 0.8, n_way), rng.uniform(-0.4, 0.4, n_way),
                                 rng.uniform(-1.0, 0.8, n_way)])
            ypr = np.column_stack([rng.uniform(-15, 15, n_way), rng.uniform(-8, 8, n_way),
                                   rng.uniform(-5, 5, n_way)])
            Pc = np.vstack([P, P[:1]])
            s = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(Pc, axis=0), axis=1))])
            cs = CubicSpline(s, Pc, bc_type="periodic")
            dense = np.linspace(0.0, s[-1], 40001)
            pts = cs(dense)
            arc = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(pts, axis=0), axis=1))])
            keys = Rotation.from_euler("YXZ", np.vstack([ypr, ypr[:1]]), degrees=True)
            arc_at_way = np.interp(s, dense, arc)
            ok = True
            for j in range(n_way):
                ang = np.rad2deg((keys[j].inv() * keys[j + 1]).magnitude())
                dt = (arc_at_way[j + 1] - arc_at_way[j]) / speed
                if ang / dt > max_rate_dps:
                    ok = False
                    break
            if ok:
                break
        else:  # pragma: no cover
            raise RuntimeError("no admissible trajectory")
        self._cs, self._dense, self._arc, self._s = cs, dense, arc, s
        self._slerp = Slerp(s, keys)
        self.rate_hz, self.speed, self.length = rate_hz, speed, arc[-1]

    def T_cw(self, k: int) -> np.ndarray:
        a = (self.speed * k / self.rate_hz) % self.length
        s = np.interp(a, self._arc, self._dense)
        c = self._cs(s)
        R_wc = self._slerp([s]).as_matrix()[0]
        return pose_matrix(R_wc.T, -R_wc.T @ c)


def sequence_frames(seed: int = 2607, cam: Camera = CAM_752, n_frames: int = 2000, noise_sigma: float = 2.0,
                    start: int = 0, scene_seed: int | None = None):
    """Frames of the sequence workload: yields (k, img, depth, T_cw_gt)."""
    traj = Trajectory(seed)
    scene = Scene(seed if scene_seed is None else scene_seed)
    for k in range(start, start + n_frames):
        T = traj.T_cw(k)
        noise = pixel_noise(seed, k, cam, noise_sigma) if noise_sigma > 0 else None
        img, depth = scene.render(cam, T, noise, want_depth=(k % 10 == 0))
        yield k, img, depth, T


def tween_frames(seed: int = 2607, cam: Camera = CAM_752, n_frames: int = 200, noise_sigma: float = 2.0,
                 p_jump: float = 0.04, jump=(15, 40), p_flicker: float = 0.05, gain=(1.15, 1.35)):
    """A sequence for the tween-window schedule: the sequence trajectory sampled
    at 200 Hz, except that with probability p_jump a frame skips ahead by a
    seeded 15-40 samples (dropped frames: a large, unpredicted motion), and with
    probability p_flicker a frame's intensities are scaled by a seeded gain
    (exposure flicker, which the photometric model does not absorb).  Every frame
    comes with its depth.  Yields (k, img, depth, T_cw_gt, events)."""
    rng = np.random.default_rng([seed, 31])
    traj = Trajectory(seed)
    scene = Scene(seed)
    t = 0
    for k in range(n_frames):
        step = 0
        if k > 0:
            step = int(rng.integers(jump[0], jump[1] + 1)) if rng.random() < p_jump else 1
            t += step
        g = float(rng.uniform(*gain)) if (k > 0 and rng.random() < p_flicker) else 1.0
        T = traj.T_cw(t)
        noise = pixel_noise(seed, t, cam, noise_sigma) if noise_sigma > 0 else None
        img, depth = scene.render(cam, T, noise)
        if g != 1.0:
            img = np.clip(np.rint(img.astype(np.float64) * g), 0, 255).astype(np.uint8)
        yield k, img, depth, T, dict(step=step, gain=g)


def stream_spec(s: int):
    """Per-stream draw of the batched workload: camera and map size for stream s."""
    rng = np.random.default_rng(1000 + s)
    cam = RESOLUTIONS[int(rng.integers(0, 3))]
    n_points = int(round(np.exp(rng.uniform(np.log(300.0), np.log(8000.0)))))
    return cam, n_points


def stream_frames(s: int, n_frames: int = 32, max_deg: float = 1.0, max_m: float = 0.02):
    """Reference (identity pose) plus n_frames perturbed views of stream s."""
    cam, n_points = stream_spec(s)
    scene = Scene(1000 + s)
    ref, depth = scene.render(cam, np.eye(4))
    rng = np.random.default_rng([1000 + s, 5])
    frames, gts = [], []
    for _ in range(n_frames):
        T = random_perturbation(rng, max_deg, max_m)
        img, _ = scene.render(cam, T, want_depth=False)
        frames.append(img)
        gts.append(T)
    return dict(cam=cam, n_points=n_points, ref=ref, depth=depth, frames=frames, T_cw_gt=gts)
