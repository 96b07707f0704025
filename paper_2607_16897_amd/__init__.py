"""Python binding of the MI355X direct photometric tracker (libdptrack.so).

Argument marshalling only: every step of the tracking path runs in the HIP
kernels behind the C ABI declared in ``include/dptrack.h``.  Host inputs are
NumPy arrays; device inputs are torch CUDA tensors (``data_ptr()``), and the
HIP stream defaults to torch's current stream.  There is no CPU fallback: if
the library is not built, :func:`load` raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DPT_LIBRARY") or os.path.join(_HERE, "libdptrack.so")
_lib = None

DPT_OK, DPT_E_ARG, DPT_E_HIP, DPT_E_STATE, DPT_E_OOM = 0, -1, -2, -3, -4
TRACK_OK, TRACK_MAX_ITERS, TRACK_TOO_FEW_POINTS, TRACK_NOT_PD, TRACK_TIMEOUT = 0, 1, 2, 3, 4
PREC_FP32, PREC_MIXED = 0, 1
FLAG_FIXED_H = 1  # dpt_params.flags: the paper's constant-H track
FLAG_GAUSS_F32 = 2  # dpt_params.flags: track on the floating-point Gaussian pyramid
SLOT_REF, SLOT_CUR = 0, 1
LAUNCH_AUTO, LAUNCH_WORKGROUP, LAUNCH_COOP, LAUNCH_COOP_PAIRS = 0, 1, 2, 3
INIT_GIVEN, INIT_CONST_VELOCITY, INIT_PROPOSED = 0, 1, 2
MAX_WINDOW = 32  # most frames one window track covers
MAX_IN_FLIGHT = 256  # most tracks enqueued and not yet synchronised
DEFAULT_PATTERN = ((-2, 0), (2, 0), (0, -2), (0, 2), (-1, -1), (1, -1), (-1, 1), (1, 1))


class DptError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dptrack error {code}: {msg}")
        self.code = code


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("huber_k", ctypes.c_float),
                ("step_eps", ctypes.c_float), ("z_min", ctypes.c_float), ("min_points", ctypes.c_int32),
                ("n_pattern", ctypes.c_int32), ("pattern", ctypes.c_int8 * 256), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("T_cw", ctypes.c_double * 16), ("final_cost", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("iters_per_level", ctypes.c_int32 * 8), ("n_valid_points", ctypes.c_int32),
                ("status", ctypes.c_int32), ("samples", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return dict(T_cw=np.array(self.T_cw[:]).reshape(4, 4), final_cost=self.final_cost,
                    iterations=self.iterations, iters_per_level=list(self.iters_per_level),
                    n_valid_points=self.n_valid_points, status=self.status, samples=self.samples)


class TweenPolicy(ctypes.Structure):
    _fields_ = [("max_cost", ctypes.c_float), ("max_baseline", ctypes.c_float), ("max_direct", ctypes.c_int32),
                ("n_points", ctypes.c_int32), ("margin", ctypes.c_int32), ("pad", ctypes.c_int32)]


class TweenResult(ctypes.Structure):
    _fields_ = [("decision", ctypes.c_int32), ("direct_since_ref", ctypes.c_int32), ("tracked", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("baseline", ctypes.c_double), ("track", Result)]


TWEEN_DIRECT, TWEEN_FAILED, TWEEN_COST, TWEEN_BASELINE, TWEEN_MAX_FRAMES = 0, 1, 2, 3, 4

# NumPy view of dpt_result (zero-copy reads of result arrays)
RESULT_DTYPE = np.dtype({
    "names": ["T_cw", "final_cost", "iterations", "iters_per_level", "n_valid_points", "status", "samples"],
    "formats": [("<f8", (16,)), "<f8", "<i4", ("<i4", (8,)), "<i4", "<i4", "<i8"],
    "offsets": [Result.T_cw.offset, Result.final_cost.offset, Result.iterations.offset,
                Result.iters_per_level.offset, Result.n_valid_points.offset, Result.status.offset,
                Result.samples.offset],
    "itemsize": ctypes.sizeof(Result)})

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64

# name -> (restype, argtypes); the ABI test checks this list against include/dptrack.h
SIGNATURES = {
    "dpt_last_error": (ctypes.c_char_p, []),
    "dpt_create": (ctypes.c_int, [ctypes.POINTER(Camera), ctypes.POINTER(Params), _i32, _vp, ctypes.POINTER(_vp)]),
    "dpt_destroy": (None, [_vp]),
    "dpt_build_pyramid": (ctypes.c_int, [_vp, _i32, _vp, _i64, _i32]),
    "dpt_get_pyramid": (ctypes.c_int, [_vp, _i32, _i32, _vp]),
    "dpt_get_pyramid_f32": (ctypes.c_int, [_vp, _i32, _i32, _vp]),
    "dpt_tween_set_policy": (ctypes.c_int, [_vp, ctypes.POINTER(TweenPolicy)]),
    "dpt_tween_anchor": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _i64, _i32, ctypes.POINTER(ctypes.c_double)]),
    "dpt_tween_frame": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.POINTER(TweenResult)]),
    "dpt_select_points": (ctypes.c_int, [_vp, _i32, _i32, _vp, ctypes.POINTER(_i32)]),
    "dpt_select_points_noalloc": (ctypes.c_int, [_vp, _i32, _i32, _i64, _i32, _i32, _vp, _vp, _vp]),
    "dpt_set_reference_points": (ctypes.c_int, [_vp, _vp, _i32, ctypes.POINTER(ctypes.c_double), _i32]),
    "dpt_set_reference_from_depth": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, _i32,
                                                    ctypes.POINTER(ctypes.c_double)]),
    "dpt_batch_set_reference_from_depth": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _i64, _i32,
                                                          ctypes.POINTER(ctypes.c_double)]),
    "dpt_track_frame": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Result)]),
    "dpt_track_enqueue": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_double), _vp]),
    "dpt_collect": (ctypes.c_int, [_vp, _i32]),
    "dpt_tracks_in_flight": (ctypes.c_int, [_vp]),
    "dpt_track_window_enqueue": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i32, _i32, _i32,
                                                ctypes.POINTER(ctypes.c_double), _vp]),
    "dpt_synchronize": (ctypes.c_int, [_vp]),
    "dpt_set_pose_history": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "dpt_get_profile": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]),
    "dpt_get_reference_cache": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "dpt_normal_equations": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_double), _vp, _vp,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64),
                                            ctypes.POINTER(_i32)]),
    "dpt_get_fixed_hessian": (ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_i32)]),
    "dpt_set_profiling": (ctypes.c_int, [_vp, _i32]),
    "dpt_set_launch_config": (ctypes.c_int, [_vp, _i32, _i32]),
    "dpt_cycle_profile": (ctypes.c_int, [_vp, _i32, _i32]),
    "dpt_set_spin_limit": (ctypes.c_int, [_vp, _i32]),
    "dpt_batch_create": (ctypes.c_int, [_i32, _vp, ctypes.POINTER(Params), _vp, _vp, ctypes.POINTER(_vp)]),
    "dpt_batch_destroy": (None, [_vp]),
    "dpt_batch_build_pyramids": (ctypes.c_int, [_vp, _i32, _vp, _vp, _i32]),
    "dpt_batch_select_points": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, ctypes.POINTER(_i32)]),
    "dpt_batch_set_reference_points": (ctypes.c_int, [_vp, _i32, _vp, _i32, ctypes.POINTER(ctypes.c_double), _i32]),
    "dpt_batch_track": (ctypes.c_int, [_vp, _vp, _vp]),
    "dpt_batch_track_enqueue": (ctypes.c_int, [_vp, _i32, _vp, _vp]),
    "dpt_batch_collect": (ctypes.c_int, [_vp, _i32]),
    "dpt_batch_tracks_in_flight": (ctypes.c_int, [_vp]),
    "dpt_batch_track_window_enqueue": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    "dpt_batch_synchronize": (ctypes.c_int, [_vp]),
    "dpt_batch_set_reference_from_depth_all": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    "dpt_batch_set_pose_history_all": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                                      ctypes.POINTER(ctypes.c_double)]),
    "dpt_batch_set_pose_history": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(ctypes.c_double)]),
    "dpt_batch_get_profile": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64),
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]),
    "dpt_batch_set_launch_config": (ctypes.c_int, [_vp, _i32, _i32]),
    "dpt_batch_set_spin_limit": (ctypes.c_int, [_vp, _i32]),
    "dpt_batch_set_profiling": (ctypes.c_int, [_vp, _i32]),
    "dpt_batch_last_kernel_ms": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "dpt_batch_get_level": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i32]),
    "dpt_cnn_num_params": (_i32, []),
    "dpt_cnn_create": (ctypes.c_int, [_i32, _vp, ctypes.POINTER(_vp)]),
    "dpt_cnn_destroy": (None, [_vp]),
    "dpt_cnn_set_params": (ctypes.c_int, [_vp, _vp]),
    "dpt_cnn_get_params": (ctypes.c_int, [_vp, _vp]),
    "dpt_cnn_get_grads": (ctypes.c_int, [_vp, _vp]),
    "dpt_cnn_forward": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp]),
    "dpt_cnn_train_step": (ctypes.c_int, [_vp, _vp, _vp, _i32, ctypes.c_float, _i32, ctypes.POINTER(ctypes.c_float)]),
    "dpt_cnn_get_activation": (ctypes.c_int, [_vp, _i32, _i32, _vp]),
    "dpt_cnn_predict": (ctypes.c_int, [_vp, _vp, _vp]),
    "dpt_cnn_predict_batch": (ctypes.c_int, [_vp, _vp, _vp]),
    "dpt_cnn_propose": (ctypes.c_int, [_vp, _vp]),
    "dpt_set_reference_stream": (ctypes.c_int, [_vp, _vp]),
    "dpt_stream_create": (ctypes.c_int, [_vp]),
    "dpt_stream_destroy": (ctypes.c_int, [_vp]),
    "dpt_batch_set_reference_stream": (ctypes.c_int, [_vp, _vp]),
    "dpt_probe_read_bandwidth": (ctypes.c_int, [_i64, _i32, _i32, ctypes.POINTER(ctypes.c_double)]),
    "dpt_probe_fp32_fma": (ctypes.c_int, [_i32, ctypes.POINTER(ctypes.c_double)]),
    "dpt_cnn_propose_batch": (ctypes.c_int, [_vp, _vp]),
    "dpt_last_kernel_ms": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
}


def load():
    """Load libdptrack.so (built by ``paper_2607_16897_amd.build``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
        try:  # one HIP runtime per process: let the library bind to the one PyTorch ships
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


# Every open Tracker, BatchTracker and Cnn.  An interpreter exit closes the ones
# still open from an atexit hook, which runs before module teardown while torch
# and the HIP runtime are fully alive; a handle reached by __del__ during the
# interpreter's own finalisation is left to the process exit instead of calling
# into HIP at an undefined point of the teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_live():
    for obj in list(_live):
        obj.close()


def _check(code: int):
    if code != DPT_OK:
        raise DptError(code, load().dpt_last_error().decode())


def _mat(T) -> ctypes.Array:
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(16))
    return (ctypes.c_double * 16)(*T.tolist())


def _ptr(x):
    """(pointer, on_device, keepalive) for a NumPy array or a torch CUDA tensor."""
    if isinstance(x, np.ndarray):
        x = np.ascontiguousarray(x)
        return x.ctypes.data, 0, x
    import torch

    if isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            x = x.contiguous()
        return x.data_ptr(), int(x.is_cuda), x
    raise TypeError(f"unsupported buffer type {type(x)}")


def _frames(x):
    """(n_frames, pointer, row pitch, frame stride, on_device, keepalive) of a
    [F, H, W] uint8 NumPy array or torch tensor (device tensors at their own
    strides; rows must be contiguous)."""
    if isinstance(x, np.ndarray):
        x = np.ascontiguousarray(x, dtype=np.uint8)
        if x.ndim != 3:
            raise ValueError("frames must be [F, H, W]")
        return x.shape[0], x.ctypes.data, x.strides[1], x.strides[0], 0, x
    import torch

    if isinstance(x, torch.Tensor):
        if x.dim() != 3 or x.dtype != torch.uint8:
            raise ValueError("frames must be a [F, H, W] uint8 tensor")
        if x.stride(2) != 1:
            x = x.contiguous()
        return x.shape[0], x.data_ptr(), x.stride(1), x.stride(0), int(x.is_cuda), x
    raise TypeError(f"unsupported buffer type {type(x)}")


def make_camera(cam) -> Camera:
    return Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)


def make_params(levels=3, max_iters=10, huber_k=9.0, step_eps=1e-5, z_min=1e-3, min_points=10,
                pattern=DEFAULT_PATTERN, precision=PREC_FP32, flags=0, fixed_h=False, gauss=False) -> Params:
    """fixed_h=True sets FLAG_FIXED_H (the paper's constant-H track, no weights);
    gauss=True sets FLAG_GAUSS_F32 (the floating-point Gaussian pyramid)."""
    if fixed_h:
        flags |= FLAG_FIXED_H
    if gauss:
        flags |= FLAG_GAUSS_F32
    p = Params()
    p.levels, p.max_iters, p.huber_k, p.step_eps, p.z_min = levels, max_iters, huber_k, step_eps, z_min
    p.min_points, p.precision, p.flags = min_points, precision, flags
    pat = np.asarray(pattern, np.int32).reshape(-1, 2)
    p.n_pattern = len(pat)
    for i, v in enumerate(pat.reshape(-1)):
        p.pattern[i] = int(v)
    return p


def current_stream() -> int:
    import torch

    return int(torch.cuda.current_stream().cuda_stream) if torch.cuda.is_available() else 0


class Stream:
    """A HIP stream the library creates (dpt_stream_create) for reference
    updates: default priority, not ordered with the null stream.  Pass it to
    Tracker/BatchTracker.set_reference_stream; it is destroyed by close() or
    when the last holder lets it go."""

    def __init__(self):
        h = _vp()
        _check(load().dpt_stream_create(ctypes.byref(h)))
        self.cuda_stream = int(h.value)

    def close(self):
        if getattr(self, "cuda_stream", 0):
            _check(load().dpt_stream_destroy(self.cuda_stream))
            self.cuda_stream = 0

    def __del__(self, _finalising=sys.is_finalizing):
        if not _finalising():
            self.close()


CYCLE_FIELDS = ("accumulate", "reduce", "exchange", "solve", "iterations", "launches", "kernel", "realtime", "place",
                "polls", "frame_start", "level_start", "final", "frames", "frame_end", "spare")


def cycle_profile(n_slots: int, reset: bool = True) -> np.ndarray:
    """Per-slot cycle split of the cooperative track (dpt_cycle_profile): an
    int64 array (n_slots, 16) with columns CYCLE_FIELDS.  Needs the
    instrumented library (DPT_LIBRARY=.../libdptrack_cycles.so)."""
    out = np.zeros((n_slots, len(CYCLE_FIELDS)), np.int64)
    _check(load().dpt_cycle_profile(out.ctypes.data, n_slots, int(bool(reset))))
    return out


def probe_read_bandwidth(slice_bytes: int, n_slices: int, reps: int) -> float:
    """dpt_probe_read_bandwidth: attainable read GB/s of a buffer of n_slices
    slices of slice_bytes, each workgroup rereading one slice reps times."""
    gbs = ctypes.c_double()
    _check(load().dpt_probe_read_bandwidth(int(slice_bytes), int(n_slices), int(reps), ctypes.byref(gbs)))
    return gbs.value


def probe_fp32_fma(iters: int = 4096) -> float:
    """dpt_probe_fp32_fma: attainable FP32 FMA TFLOP/s of the vector units."""
    tf = ctypes.c_double()
    _check(load().dpt_probe_fp32_fma(int(iters), ctypes.byref(tf)))
    return tf.value


def select_points_noalloc(img, n: int, margin: int, idx, count, stream: int | None = None):
    """dpt_select_points_noalloc: top-n gradient-score pixels of a uint8 CUDA
    tensor img (H x W, rows at any stride) into the int32 CUDA tensors idx (>= n
    entries) and count (>= 1 entry), enqueued on `stream` (torch's current one
    by default); allocates nothing and does not wait."""
    lib = load()
    if not (img.is_cuda and idx.is_cuda and count.is_cuda):
        raise ValueError("img, idx and count must be CUDA tensors")
    if img.dim() != 2 or img.stride(1) != 1 or idx.numel() < n or count.numel() < 1:
        raise ValueError("img must be H x W with unit column stride; idx needs n entries, count one")
    H, W = int(img.shape[0]), int(img.shape[1])
    s = current_stream() if stream is None else stream
    _check(lib.dpt_select_points_noalloc(img.data_ptr(), W, H, int(img.stride(0)), n, margin, idx.data_ptr(),
                                         count.data_ptr(), s))


class Tracker:
    """One camera stream: pyramids, reference IC cache and the per-frame track."""

    def __init__(self, cam, params: Params, max_points: int, stream: int | None = None):
        self._lib = load()
        self.cam = cam if isinstance(cam, Camera) else make_camera(cam)
        self.params = params
        self.stream = current_stream() if stream is None else stream
        h = _vp()
        _check(self._lib.dpt_create(ctypes.byref(self.cam), ctypes.byref(params), max_points, self.stream,
                                    ctypes.byref(h)))
        self._h = h
        self.n_points = 0
        self._pending = []
        self._frames_keep = []  # window frames until their tracks are synchronised
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dpt_destroy(self._h)
            self._h = None
            self._pending, self._frames_keep = [], []
        _live.discard(self)

    def __del__(self, _finalising=sys.is_finalizing):  # bound now: module globals are gone at shutdown
        if not _finalising():
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def build_pyramid(self, slot: int, img, pitch: int | None = None):
        p, dev, keep = _ptr(img)
        pitch = self.cam.width if pitch is None else pitch
        _check(self._lib.dpt_build_pyramid(self._h, slot, p, pitch, dev))

    def get_pyramid(self, slot: int, level: int) -> np.ndarray:
        w, h = self.cam.width >> level, self.cam.height >> level
        out = np.empty((h, w), np.uint8)
        _check(self._lib.dpt_get_pyramid(self._h, slot, level, out.ctypes.data))
        return out

    def get_pyramid_f32(self, slot: int, level: int) -> np.ndarray:
        """Level of the floating-point Gaussian pyramid (FLAG_GAUSS_F32 contexts)."""
        w, h = self.cam.width >> level, self.cam.height >> level
        out = np.empty((h, w), np.float32)
        _check(self._lib.dpt_get_pyramid_f32(self._h, slot, level, out.ctypes.data))
        return out

    def select_points(self, n: int, margin: int = 8) -> np.ndarray:
        out = np.empty(n, np.int32)
        cnt = _i32()
        _check(self._lib.dpt_select_points(self._h, n, margin, out.ctypes.data, ctypes.byref(cnt)))
        return out[:cnt.value].copy()

    def set_reference_points(self, xyz, T_rw):
        if isinstance(xyz, np.ndarray):
            xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        p, dev, keep = _ptr(xyz)
        n = int(xyz.shape[0])
        _check(self._lib.dpt_set_reference_points(self._h, p, n, _mat(T_rw), dev))
        self.n_points = n

    def set_reference_from_depth(self, n: int, depth, T_rw, margin: int = 8, pitch: int | None = None):
        """Select n points on the REF level 0 and back-project them with `depth`
        (float32 H x W, NumPy or a torch CUDA tensor), all on the stream."""
        if isinstance(depth, np.ndarray):
            depth = np.ascontiguousarray(depth, dtype=np.float32)
        p, dev, keep = _ptr(depth)
        pitch = self.cam.width if pitch is None else pitch
        _check(self._lib.dpt_set_reference_from_depth(self._h, n, margin, p, pitch, dev, _mat(T_rw)))
        self.n_points = n

    def track(self, T_cw_init) -> dict:
        r = Result()
        _check(self._lib.dpt_track_frame(self._h, _mat(T_cw_init), ctypes.byref(r)))
        return r.as_dict()

    # tween-window schedule (Sec. III, Sec. IV-D)
    def tween_set_policy(self, max_cost: float, max_direct: int, n_points: int, max_baseline: float = 0.0,
                         margin: int = 8):
        p = TweenPolicy(max_cost, max_baseline, max_direct, n_points, margin, 0)
        _check(self._lib.dpt_tween_set_policy(self._h, ctypes.byref(p)))
        self.n_points = n_points

    def tween_anchor(self, img, depth, T_cw):
        """The indirect pipeline's frame: image, level-0 depth and pose become the reference."""
        pi, di, k1 = _ptr(img)
        if isinstance(depth, np.ndarray):
            depth = np.ascontiguousarray(depth, dtype=np.float32)
        pd, dd, k2 = _ptr(depth)
        _check(self._lib.dpt_tween_anchor(self._h, pi, self.cam.width, di, pd, self.cam.width, dd, _mat(T_cw)))

    def tween_frame(self, img) -> dict:
        """Direct attempt on a tween frame and the schedule's decision (TWEEN_*)."""
        p, dev, keep = _ptr(img)
        r = TweenResult()
        _check(self._lib.dpt_tween_frame(self._h, p, self.cam.width, dev, ctypes.byref(r)))
        return dict(decision=r.decision, direct_since_ref=r.direct_since_ref, tracked=bool(r.tracked),
                    baseline=r.baseline, track=r.track.as_dict() if r.tracked else None)

    def set_reference_stream(self, stream=None):
        """Reference updates on a second stream (a Stream, a torch.cuda.Stream or
        a raw handle; None: back to the context's stream), overlapping the tracks
        of the previous reference; an update then starts with build_pyramid(SLOT_REF)."""
        handle = getattr(stream, "cuda_stream", stream)
        _check(self._lib.dpt_set_reference_stream(self._h, handle))
        self.ref_stream = stream

    def track_enqueue(self, T_cw_init=None, proposed: bool = False):
        """Enqueue a track without waiting: from T_cw_init, (None) from the
        constant-velocity prediction of the pose history, or (proposed=True) from
        the learned proposal of the last Cnn.propose(self).  Results come back, in
        order, from synchronize()."""
        r = Result()
        if proposed:
            _check(self._lib.dpt_track_enqueue(self._h, INIT_PROPOSED, None, ctypes.byref(r)))
        elif T_cw_init is None:
            _check(self._lib.dpt_track_enqueue(self._h, INIT_CONST_VELOCITY, None, ctypes.byref(r)))
        else:
            _check(self._lib.dpt_track_enqueue(self._h, INIT_GIVEN, _mat(T_cw_init), ctypes.byref(r)))
        self._pending.append(r)
        self._frames_keep.append(None)

    def track_window_enqueue(self, frames, T_cw_init=None):
        """Enqueue the track of consecutive frames (a [F, H, W] uint8 NumPy array on
        the host or torch CUDA tensor, rows and frames at any stride) in one pyramid
        and one track launch: frame 0 from T_cw_init or (None) the constant-velocity
        prediction of the pose history, every later frame from the prediction of
        the two before it.  Results come back, in order, from synchronize()."""
        F, p, pitch, fstride, dev, keep = _frames(frames)
        res = (Result * F)()
        T = None if T_cw_init is None else _mat(T_cw_init)
        _check(self._lib.dpt_track_window_enqueue(self._h, p, pitch, fstride, F, dev,
                                                  INIT_CONST_VELOCITY if T is None else INIT_GIVEN, T,
                                                  ctypes.cast(res, _vp)))
        self._pending.extend(res[f] for f in range(F))
        # device frames are read by the track launch too: kept with the window's last result
        self._frames_keep.extend([None] * (F - 1) + [keep])

    def collect(self, n: int, arrays: bool = False):
        """Results of the oldest n enqueued tracks as soon as they have finished; the
        later ones keep running.  Same forms as synchronize()."""
        if not 0 <= n <= len(self._pending):
            raise ValueError(f"{n} results asked, {len(self._pending)} enqueued")
        ready = len(self._pending) - self._lib.dpt_tracks_in_flight(self._h)  # filled by an earlier wait
        try:
            if n > ready:
                _check(self._lib.dpt_collect(self._h, n - ready))
        except DptError as err:  # all results travel with the error
            err.results = [r.as_dict() for r in self._pending]
            self._drop_pending(self._lib.dpt_tracks_in_flight(self._h))
            raise
        got, self._pending = self._pending[:n], self._pending[n:]
        self._frames_keep = self._frames_keep[n:]
        if arrays:
            return np.concatenate([np.frombuffer(r, dtype=RESULT_DTYPE) for r in got]) if got \
                else np.empty(0, RESULT_DTYPE)
        return [r.as_dict() for r in got]

    def synchronize(self, arrays: bool = False):
        """Results of the enqueued tracks, in order: a list of dicts, or (arrays=True)
        one structured array with the fields of RESULT_DTYPE."""
        try:
            _check(self._lib.dpt_synchronize(self._h))
        except DptError as err:  # the results travel with the error (err.results)
            err.results = [r.as_dict() for r in self._pending]
            self._drop_pending(self._lib.dpt_tracks_in_flight(self._h))
            raise
        if arrays:
            out = np.concatenate([np.frombuffer(r, dtype=RESULT_DTYPE) for r in self._pending]) if self._pending \
                else np.empty(0, RESULT_DTYPE)
        else:
            out = [r.as_dict() for r in self._pending]
        self._pending = []
        self._frames_keep = []
        return out

    def tracks_in_flight(self) -> int:
        """Enqueued tracks whose results the library has not filled yet."""
        n = self._lib.dpt_tracks_in_flight(self._h)
        _check(min(n, 0))
        return n

    def _drop_pending(self, in_flight: int):
        """After a failed wait the library has filled or marked every result and
        holds no pointer to them (dpt_tracks_in_flight() == 0): the result buffers
        and the window frames are released.  Should it still report tracks in
        flight, they stay referenced, since the library may still write them."""
        if in_flight == 0:
            self._pending, self._frames_keep = [], []

    def set_pose_history(self, T_older, T_newer):
        _check(self._lib.dpt_set_pose_history(self._h, _mat(T_older), _mat(T_newer)))

    def set_launch_config(self, mode: int, chunk: int = 256):
        _check(self._lib.dpt_set_launch_config(self._h, mode, chunk))

    def set_spin_limit(self, polls: int = 4194304):
        """Polls before a cooperative wait gives up (0: at once; the default restores it)."""
        _check(self._lib.dpt_set_spin_limit(self._h, polls))

    def set_profiling(self, enable: bool = True, every: int = 1):
        """Time every `every`-th pyramid and track launch with HIP events (off: enable=False)."""
        _check(self._lib.dpt_set_profiling(self._h, int(every) if enable else 0))

    def last_kernel_ms(self):
        """(pyramid_ms, track_ms) of the most recent timed kernels (-1 if none)."""
        a, b = ctypes.c_float(), ctypes.c_float()
        _check(self._lib.dpt_last_kernel_ms(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def profile(self) -> dict:
        """Totals (ms) and counts of the timed pyramid and track kernels."""
        pm, pn, tm, tn = ctypes.c_double(), _i64(), ctypes.c_double(), _i64()
        _check(self._lib.dpt_get_profile(self._h, ctypes.byref(pm), ctypes.byref(pn), ctypes.byref(tm),
                                         ctypes.byref(tn)))
        return dict(pyramid_ms=pm.value, n_pyramid=pn.value, track_ms=tm.value, n_track=tn.value)

    def reference_cache(self, level: int) -> dict:
        n, K = self.n_points, self.params.n_pattern
        valid = np.empty(max(n, 1), np.uint8)
        I0, gx, gy = (np.empty(max(n * K, 1), np.float32) for _ in range(3))
        x0 = np.empty(max(n * 3, 1), np.float32)
        _check(self._lib.dpt_get_reference_cache(self._h, level, valid.ctypes.data, I0.ctypes.data, gx.ctypes.data,
                                                 gy.ctypes.data, x0.ctypes.data))
        return dict(valid=valid[:n].astype(bool), I0=I0[:n * K].reshape(n, K), gx=gx[:n * K].reshape(n, K),
                    gy=gy[:n * K].reshape(n, K), x0=x0[:n * 3].reshape(n, 3))

    def normal_equations(self, level: int, T_rel) -> dict:
        H21, b6 = np.empty(21, np.float32), np.empty(6, np.float32)
        E, n, npts = ctypes.c_double(), _i64(), _i32()
        _check(self._lib.dpt_normal_equations(self._h, level, _mat(T_rel), H21.ctypes.data, b6.ctypes.data,
                                              ctypes.byref(E), ctypes.byref(n), ctypes.byref(npts)))
        H = np.zeros((6, 6))
        q = 0
        for i in range(6):
            for j in range(i, 6):
                H[i, j] = H[j, i] = H21[q]
                q += 1
        return dict(H=H, b=b6.astype(np.float64), E=E.value, n=n.value, npts=npts.value)

    def fixed_hessian(self, level: int):
        """Fixed-H mode: (H 6x6 float64 of the current reference at `level`, not_pd)."""
        H = np.empty((6, 6), np.float64)
        bad = _i32()
        _check(self._lib.dpt_get_fixed_hessian(self._h, level, H.ctypes.data, ctypes.byref(bad)))
        return H, bool(bad.value)


class BatchTracker:
    """Many independent camera streams tracked in one launch sequence."""

    def __init__(self, cams, params: Params, max_points, stream: int | None = None):
        self._lib = load()
        self.n = len(cams)
        self.cams = (Camera * self.n)(*[c if isinstance(c, Camera) else make_camera(c) for c in cams])
        self.params = params
        self.stream = current_stream() if stream is None else stream
        mp = (_i32 * self.n)(*[int(m) for m in max_points])
        h = _vp()
        _check(self._lib.dpt_batch_create(self.n, ctypes.cast(self.cams, _vp), ctypes.byref(params),
                                          ctypes.cast(mp, _vp), self.stream, ctypes.byref(h)))
        self._h = h
        self._pending = []
        self._frames_keep = []  # window frames until their tracks are synchronised
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dpt_batch_destroy(self._h)
            self._h = None
            self._pending, self._frames_keep = [], []
        _live.discard(self)

    def __del__(self, _finalising=sys.is_finalizing):  # bound now: module globals are gone at shutdown
        if not _finalising():
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _stacked(self, x):
        """(pointer array, row pitch in elements) of a contiguous [n, H, W] CUDA tensor."""
        base, step = x.data_ptr(), x.stride(0) * x.element_size()
        ptrs = np.arange(self.n, dtype=np.uint64) * np.uint64(step) + np.uint64(base)
        return ptrs, int(x.stride(1))

    def build_pyramids(self, slot: int, imgs, pitches=None):
        """imgs: list of NumPy arrays (host) or torch CUDA tensors (device), one per
        stream, or one contiguous [n, H, W] CUDA tensor (same resolution)."""
        if hasattr(imgs, "dim") and imgs.dim() == 3 and imgs.is_cuda and imgs.is_contiguous():
            ptrs, pitch = self._stacked(imgs)
            pp = np.full(self.n, pitch, np.int64)
            _check(self._lib.dpt_batch_build_pyramids(self._h, slot, ptrs.ctypes.data, pp.ctypes.data, 1))
            return
        ptrs, devs, keep = zip(*[_ptr(x) for x in imgs])
        if len(set(devs)) != 1:
            raise ValueError("all images must be on the same side (host or device)")
        pitches = [self.cams[s].width for s in range(self.n)] if pitches is None else pitches
        pa = (ctypes.c_void_p * self.n)(*ptrs)
        pp = (_i64 * self.n)(*[int(p) for p in pitches])
        _check(self._lib.dpt_batch_build_pyramids(self._h, slot, ctypes.cast(pa, _vp), ctypes.cast(pp, _vp), devs[0]))

    def select_points(self, s: int, n: int, margin: int = 8) -> np.ndarray:
        out = np.empty(n, np.int32)
        cnt = _i32()
        _check(self._lib.dpt_batch_select_points(self._h, s, n, margin, out.ctypes.data, ctypes.byref(cnt)))
        return out[:cnt.value].copy()

    def set_reference_points(self, s: int, xyz, T_rw):
        if isinstance(xyz, np.ndarray):
            xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        p, dev, keep = _ptr(xyz)
        _check(self._lib.dpt_batch_set_reference_points(self._h, s, p, int(xyz.shape[0]), _mat(T_rw), dev))

    def set_reference_from_depth(self, s: int, n: int, depth, T_rw, margin: int = 8, pitch: int | None = None):
        """As Tracker.set_reference_from_depth, for stream s."""
        if isinstance(depth, np.ndarray):
            depth = np.ascontiguousarray(depth, dtype=np.float32)
        p, dev, keep = _ptr(depth)
        pitch = self.cams[s].width if pitch is None else pitch
        _check(self._lib.dpt_batch_set_reference_from_depth(self._h, s, n, margin, p, pitch, dev, _mat(T_rw)))

    def track(self, T_cw_init) -> list[dict]:
        T = np.ascontiguousarray(np.asarray(T_cw_init, np.float64).reshape(self.n, 16))
        res = (Result * self.n)()
        _check(self._lib.dpt_batch_track(self._h, T.ctypes.data, ctypes.cast(res, _vp)))
        return [r.as_dict() for r in res]

    def track_enqueue(self, T_cw_init=None, proposed: bool = False):
        """Enqueue a track of every stream without waiting: from T_cw_init (n x 4 x 4),
        (None) from each stream's constant-velocity prediction, or (proposed=True)
        from the learned proposals of the last Cnn.propose(self)."""
        res = (Result * self.n)()
        if proposed:
            _check(self._lib.dpt_batch_track_enqueue(self._h, INIT_PROPOSED, None, ctypes.cast(res, _vp)))
        elif T_cw_init is None:
            _check(self._lib.dpt_batch_track_enqueue(self._h, INIT_CONST_VELOCITY, None, ctypes.cast(res, _vp)))
        else:
            T = np.ascontiguousarray(np.asarray(T_cw_init, np.float64).reshape(self.n, 16))
            _check(self._lib.dpt_batch_track_enqueue(self._h, INIT_GIVEN, T.ctypes.data, ctypes.cast(res, _vp)))
        self._pending.append(res)
        self._frames_keep.append(None)

    def track_window_enqueue(self, frames, T_cw_init=None):
        """Window tracking of every stream (Tracker.track_window_enqueue): frames is
        one [F, H_s, W_s] array or tensor per stream, all with the same F, or one
        [n, F, H, W] CUDA tensor.  synchronize() returns one list of n results per
        frame."""
        if hasattr(frames, "dim") and frames.dim() == 4:
            frames = [frames[s] for s in range(frames.shape[0])]
        if len(frames) != self.n:
            raise ValueError(f"{len(frames)} frame stacks for {self.n} streams")
        parts = [_frames(x) for x in frames]
        F = parts[0][0]
        if any(q[0] != F for q in parts) or len({q[4] for q in parts}) != 1:
            raise ValueError("every stream needs the same number of frames, all on one side (host or device)")
        ptrs = (ctypes.c_void_p * self.n)(*[q[1] for q in parts])
        pitches = (_i64 * self.n)(*[q[2] for q in parts])
        strides = (_i64 * self.n)(*[q[3] for q in parts])
        res = (Result * (F * self.n))()
        if T_cw_init is None:
            mode, T = INIT_CONST_VELOCITY, None
        else:
            mode = INIT_GIVEN
            T = np.ascontiguousarray(np.asarray(T_cw_init, np.float64).reshape(self.n, 16))
        _check(self._lib.dpt_batch_track_window_enqueue(
            self._h, ctypes.cast(ptrs, _vp), ctypes.cast(pitches, _vp), ctypes.cast(strides, _vp), F, parts[0][4],
            mode, None if T is None else T.ctypes.data, ctypes.cast(res, _vp)))
        size = ctypes.sizeof(Result) * self.n
        self._pending.extend((Result * self.n).from_buffer(res, f * size) for f in range(F))
        # device frames are read by the track launch too: kept with the window's last results
        self._frames_keep.extend([None] * (F - 1) + [[q[5] for q in parts]])

    def collect(self, k: int, arrays: bool = False):
        """Results of the oldest k enqueued batched tracks as soon as they have
        finished; the later ones keep running.  Same forms as synchronize()."""
        if not 0 <= k <= len(self._pending):
            raise ValueError(f"{k} results asked, {len(self._pending)} enqueued")
        ready = len(self._pending) - self._lib.dpt_batch_tracks_in_flight(self._h)  # filled by an earlier wait
        try:
            if k > ready:
                _check(self._lib.dpt_batch_collect(self._h, k - ready))
        except DptError as err:  # all results travel with the error
            err.results = [[r.as_dict() for r in res] for res in self._pending]
            self._drop_pending(self._lib.dpt_batch_tracks_in_flight(self._h))
            raise
        got, self._pending = self._pending[:k], self._pending[k:]
        self._frames_keep = self._frames_keep[k:]
        if arrays:
            return np.stack([np.frombuffer(res, dtype=RESULT_DTYPE) for res in got]) if got \
                else np.empty((0, self.n), RESULT_DTYPE)
        return [[r.as_dict() for r in res] for res in got]

    def synchronize(self, arrays: bool = False):
        """Results of the enqueued tracks, in order: one list of n per enqueue, or
        (arrays=True) one structured array of shape (enqueues, n) with the fields of
        RESULT_DTYPE."""
        try:
            _check(self._lib.dpt_batch_synchronize(self._h))
        except DptError as err:  # the results travel with the error (err.results)
            err.results = [[r.as_dict() for r in res] for res in self._pending]
            self._drop_pending(self._lib.dpt_batch_tracks_in_flight(self._h))
            raise
        if arrays:
            out = np.stack([np.frombuffer(res, dtype=RESULT_DTYPE) for res in self._pending]) if self._pending \
                else np.empty((0, self.n), RESULT_DTYPE)
        else:
            out = [[r.as_dict() for r in res] for res in self._pending]
        self._pending = []
        self._frames_keep = []
        return out

    _drop_pending = Tracker._drop_pending

    def tracks_in_flight(self) -> int:
        """Enqueued batched tracks (each of all streams) whose results are not filled yet."""
        n = self._lib.dpt_batch_tracks_in_flight(self._h)
        _check(min(n, 0))
        return n

    def set_pose_history(self, s: int, T_older, T_newer):
        _check(self._lib.dpt_batch_set_pose_history(self._h, s, _mat(T_older), _mat(T_newer)))

    def set_pose_history_all(self, T_older, T_newer):
        """Histories of every stream: T_older, T_newer of shape (n, 4, 4)."""
        a = np.ascontiguousarray(np.asarray(T_older, np.float64).reshape(self.n * 16))
        b = np.ascontiguousarray(np.asarray(T_newer, np.float64).reshape(self.n * 16))
        _check(self._lib.dpt_batch_set_pose_history_all(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                        b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def set_reference_from_depth_all(self, n_points, depths, T_rw, margin: int = 8):
        """Reference update of every stream in one launch sequence: n_points (int or
        one per stream), depths a list of float32 torch CUDA tensors (H x W), T_rw (n, 4, 4)."""
        n = (_i32 * self.n)(*([int(n_points)] * self.n if np.isscalar(n_points) else [int(v) for v in n_points]))
        if hasattr(depths, "dim") and depths.dim() == 3:
            if not (depths.is_cuda and depths.is_contiguous()):
                raise ValueError("stacked depths must be a contiguous CUDA tensor")
            p, pitch = self._stacked(depths)
            ptrs = (ctypes.c_void_p * self.n)(*[int(v) for v in p])
            pitches = (_i64 * self.n)(*([pitch] * self.n))
        else:
            ptrs = (ctypes.c_void_p * self.n)(*[d.data_ptr() for d in depths])
            pitches = (_i64 * self.n)(*[int(d.stride(0)) for d in depths])
        T = np.ascontiguousarray(np.asarray(T_rw, np.float64).reshape(self.n * 16))
        _check(self._lib.dpt_batch_set_reference_from_depth_all(self._h, ctypes.cast(n, _vp), margin,
                                                                ctypes.cast(ptrs, _vp), ctypes.cast(pitches, _vp),
                                                                T.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self._keep = depths

    def profile(self) -> dict:
        pm, pn, tm, tn = ctypes.c_double(), _i64(), ctypes.c_double(), _i64()
        _check(self._lib.dpt_batch_get_profile(self._h, ctypes.byref(pm), ctypes.byref(pn), ctypes.byref(tm),
                                               ctypes.byref(tn)))
        return dict(pyramid_ms=pm.value, n_pyramid=pn.value, track_ms=tm.value, n_track=tn.value)

    def set_reference_stream(self, stream=None):
        """Reference updates of every stream on a second stream (Tracker.set_reference_stream)."""
        handle = getattr(stream, "cuda_stream", stream)
        _check(self._lib.dpt_batch_set_reference_stream(self._h, handle))
        self.ref_stream = stream

    def set_launch_config(self, mode: int, chunk: int = 256):
        _check(self._lib.dpt_batch_set_launch_config(self._h, mode, chunk))

    def set_spin_limit(self, polls: int = 4194304):
        """Polls before a cooperative wait gives up, for every stream."""
        _check(self._lib.dpt_batch_set_spin_limit(self._h, polls))

    def get_level(self, slot: int, level: int, dst=None):
        """Pyramid level of every stream, packed [n][H_l][W_l]: into `dst` (a torch CUDA
        tensor) on the device, else returned as a NumPy array."""
        h, w = self.cams[0].height >> level, self.cams[0].width >> level
        if dst is None:
            out = np.empty((self.n, h, w), np.uint8)
            _check(self._lib.dpt_batch_get_level(self._h, slot, level, out.ctypes.data, 0))
            return out
        assert dst.is_cuda and dst.is_contiguous() and dst.numel() == self.n * h * w
        _check(self._lib.dpt_batch_get_level(self._h, slot, level, dst.data_ptr(), 1))
        return dst

    def set_profiling(self, enable: bool = True, every: int = 1):
        """Time every `every`-th batched pyramid and track launch (off: enable=False)."""
        _check(self._lib.dpt_batch_set_profiling(self._h, int(every) if enable else 0))

    def last_kernel_ms(self):
        a, b = ctypes.c_float(), ctypes.c_float()
        _check(self._lib.dpt_batch_last_kernel_ms(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


CNN_TWIST_SCALE = np.array([np.deg2rad(5.0)] * 3 + [0.1] * 3)
CNN_SHAPES = (("w1", (16, 2, 3, 3)), ("b1", (16,)), ("w2", (32, 16, 3, 3)), ("b2", (32,)), ("w3", (64, 32, 3, 3)),
              ("b3", (64,)), ("w4", (64, 64, 3, 3)), ("b4", (64,)), ("fw1", (64, 64)), ("fb1", (64,)),
              ("fw2", (6, 64)), ("fb2", (6,)))


def cnn_flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k, _ in CNN_SHAPES])


def cnn_unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for k, shp in CNN_SHAPES:
        n = int(np.prod(shp))
        out[k] = flat[o:o + n].reshape(shp)
        o += n
    return out


class Cnn:
    """The learned start-pose network (BF16 MFMA forward, FP32 master weights)."""

    def __init__(self, max_batch: int = 256, stream: int | None = None):
        self._lib = load()
        self.n_params = int(self._lib.dpt_cnn_num_params())
        self.stream = current_stream() if stream is None else stream
        h = _vp()
        _check(self._lib.dpt_cnn_create(max_batch, self.stream, ctypes.byref(h)))
        self._h = h
        self.max_batch = max_batch
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dpt_cnn_destroy(self._h)
            self._h = None
        _live.discard(self)

    def __del__(self, _finalising=sys.is_finalizing):  # bound now: module globals are gone at shutdown
        if not _finalising():
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, params):
        flat = cnn_flatten(params) if isinstance(params, dict) else np.ascontiguousarray(params, np.float32)
        assert flat.size == self.n_params
        _check(self._lib.dpt_cnn_set_params(self._h, flat.ctypes.data))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(self._lib.dpt_cnn_get_params(self._h, out.ctypes.data))
        return out

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(self._lib.dpt_cnn_get_grads(self._h, out.ctypes.data))
        return out

    def forward(self, pairs) -> np.ndarray:
        """pairs: (B, 2, 60, 94) uint8, NumPy (host) or torch CUDA tensor."""
        p, dev, keep = _ptr(pairs)
        B = int(pairs.shape[0])
        out = np.empty((B, 6), np.float32)
        _check(self._lib.dpt_cnn_forward(self._h, p, B, dev, out.ctypes.data))
        return out

    def train_step(self, pairs, targets, lr: float) -> float:
        p, dev, keep = _ptr(pairs)
        if dev:
            import torch

            targets = torch.as_tensor(targets, dtype=torch.float32, device=pairs.device).contiguous()
        else:
            targets = np.ascontiguousarray(targets, np.float32)
        t, tdev, keep2 = _ptr(targets)
        assert tdev == dev
        loss = ctypes.c_float()
        _check(self._lib.dpt_cnn_train_step(self._h, p, t, int(pairs.shape[0]), float(lr), dev, ctypes.byref(loss)))
        return loss.value

    def activation(self, layer: int, B: int) -> np.ndarray:
        shapes = {1: (30, 47, 16), 2: (15, 24, 32), 3: (8, 12, 64), 4: (4, 6, 64), 5: (6,)}
        out = np.empty((B,) + shapes[layer], np.float32)
        _check(self._lib.dpt_cnn_get_activation(self._h, layer, B, out.ctypes.data))
        return out

    def propose(self, tracker):
        """Enqueue the learned start of a Tracker or every stream of a BatchTracker
        on its stream, kept on the device for track_enqueue(proposed=True)."""
        if isinstance(tracker, BatchTracker):
            _check(self._lib.dpt_cnn_propose_batch(self._h, tracker._h))
        else:
            _check(self._lib.dpt_cnn_propose(self._h, tracker._h))

    def predict(self, tracker) -> np.ndarray:
        """Start pose(s) T_cw from a Tracker (4x4) or a BatchTracker (n x 4 x 4)."""
        if isinstance(tracker, BatchTracker):
            T = np.empty((tracker.n, 16))
            _check(self._lib.dpt_cnn_predict_batch(self._h, tracker._h, T.ctypes.data))
            return T.reshape(-1, 4, 4)
        T = np.empty(16)
        _check(self._lib.dpt_cnn_predict(self._h, tracker._h, T.ctypes.data))
        return T.reshape(4, 4)
