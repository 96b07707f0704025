"""FP64 CPU oracle of the direct photometric tracker (test infrastructure).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It is a plain, slow, double-precision
implementation written from the paper (Sec. IV, Eq.(1)-(6)); see the header of
``dpt_oracle.c`` for the readings taken where the paper is silent.  It shares
no code with the HIP library.

The tracker itself is plain C (``dpt_oracle.c``) built with gcc into
``liboracle.so``; this module only marshals NumPy arrays through ctypes.  The
CNN initialiser's oracle is ``oracle.cnn`` (NumPy, FP64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, MAX_ITERS, TOO_FEW_POINTS, NOT_PD = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile dpt_oracle.c with gcc (-O2, strict IEEE: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99", "-Wall", "-Werror",
               os.path.join(_HERE, "dpt_oracle.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("huber_k", ctypes.c_double),
                ("step_eps", ctypes.c_double), ("min_points", ctypes.c_int32), ("n_pattern", ctypes.c_int32),
                ("pattern", ctypes.c_int32 * 256), ("z_min", ctypes.c_double), ("fixed_h", ctypes.c_int32),
                ("pyramid", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("T_cw", ctypes.c_double * 16), ("final_cost", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("iters_per_level", ctypes.c_int32 * 8), ("n_valid_points", ctypes.c_int32),
                ("status", ctypes.c_int32), ("samples", ctypes.c_int64)]

    def as_dict(self):
        return dict(T_cw=np.array(self.T_cw[:]).reshape(4, 4), final_cost=self.final_cost,
                    iterations=self.iterations, iters_per_level=list(self.iters_per_level),
                    n_valid_points=self.n_valid_points, status=self.status, samples=self.samples)


_u8p = ctypes.POINTER(ctypes.c_uint8)
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_pyramid_bytes.restype = ctypes.c_int64
        L.orc_pyramid_bytes.argtypes = [ctypes.c_int32] * 3
        L.orc_pyramid.restype = None
        L.orc_pyramid.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _u8p]
        L.orc_pyramid_gauss.restype = None
        L.orc_pyramid_gauss.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _dp]
        L.orc_sample_f.restype = ctypes.c_double
        L.orc_sample_f.argtypes = [_dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.orc_gradient_f.restype = None
        L.orc_gradient_f.argtypes = [_dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_select_points.restype = ctypes.c_int32
        L.orc_select_points.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, _i32p]
        L.orc_sample.restype = ctypes.c_double
        L.orc_sample.argtypes = [_u8p, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.orc_gradient.restype = None
        L.orc_gradient.argtypes = [_u8p, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_se3_exp.restype = None
        L.orc_se3_exp.argtypes = [_dp, _dp]
        L.orc_se3_log.restype = None
        L.orc_se3_log.argtypes = [_dp, _dp]
        L.orc_cholesky_solve.restype = ctypes.c_int
        L.orc_cholesky_solve.argtypes = [_dp, _dp, _dp, ctypes.c_double]
        L.orc_warp_jacobian.restype = None
        L.orc_warp_jacobian.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_ref_create.restype = ctypes.c_void_p
        L.orc_ref_create.argtypes = [ctypes.POINTER(Camera), ctypes.POINTER(Params), _u8p, ctypes.c_int64, _fp,
                                     ctypes.c_int32, _dp]
        L.orc_ref_free.restype = None
        L.orc_ref_free.argtypes = [ctypes.c_void_p]
        L.orc_ref_cache.restype = None
        L.orc_ref_cache.argtypes = [ctypes.c_void_p, ctypes.c_int32, _u8p, _dp, _dp, _dp, _dp]
        L.orc_ref_fixed_h.restype = None
        L.orc_ref_fixed_h.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp]
        L.orc_ref_normal_equations.restype = None
        L.orc_ref_normal_equations.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_int64, ctypes.c_int32, _dp, _dp, _dp,
                                               _dp, _i64p, _i32p]
        L.orc_ref_track.restype = ctypes.c_int32
        L.orc_ref_track.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_int64, _dp, ctypes.POINTER(Result)]
        _lib = L
    return _lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(_u8p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


# ----------------------------------------------------------------- small primitives
def pyramid(img: np.ndarray, levels: int) -> list[np.ndarray]:
    lib = _load()
    img, p = _u8(img)
    H, W = img.shape
    out = np.empty(lib.orc_pyramid_bytes(W, H, levels), np.uint8)
    lib.orc_pyramid(p, W, W, H, levels, out.ctypes.data_as(_u8p))
    res, off = [], 0
    for l in range(levels):
        w, h = W >> l, H >> l
        res.append(out[off:off + w * h].reshape(h, w))
        off += w * h
    return res


def pyramid_gauss(img: np.ndarray, levels: int) -> list[np.ndarray]:
    """The floating-point Gaussian pyramid (binomial [1 3 3 1]/8, clamped), FP64."""
    lib = _load()
    img, p = _u8(img)
    H, W = img.shape
    out = np.empty(lib.orc_pyramid_bytes(W, H, levels), np.float64)
    lib.orc_pyramid_gauss(p, W, W, H, levels, out.ctypes.data_as(_dp))
    res, off = [], 0
    for l in range(levels):
        w, h = W >> l, H >> l
        res.append(out[off:off + w * h].reshape(h, w))
        off += w * h
    return res


def select_points(img: np.ndarray, n: int, margin: int = 8) -> np.ndarray:
    lib = _load()
    img, p = _u8(img)
    H, W = img.shape
    out = np.empty(max(n, 1), np.int32)
    k = lib.orc_select_points(p, W, W, H, n, margin, out.ctypes.data_as(_i32p))
    return out[:k].copy()


def sample(img, x, y) -> float:
    img, p = _u8(img)
    return _load().orc_sample(p, img.shape[1], float(x), float(y))


def gradient(img, x, y):
    img, p = _u8(img)
    gx, gy = ctypes.c_double(), ctypes.c_double()
    _load().orc_gradient(p, img.shape[1], float(x), float(y), ctypes.byref(gx), ctypes.byref(gy))
    return gx.value, gy.value


def sample_f(img, x, y) -> float:
    """Bilinear sample of a level stored as doubles."""
    img, p = _f64(img)
    return _load().orc_sample_f(p, img.shape[1], float(x), float(y))


def gradient_f(img, x, y):
    img, p = _f64(img)
    gx, gy = ctypes.c_double(), ctypes.c_double()
    _load().orc_gradient_f(p, img.shape[1], float(x), float(y), ctypes.byref(gx), ctypes.byref(gy))
    return gx.value, gy.value


def se3_exp(xi) -> np.ndarray:
    xi, p = _f64(xi)
    T = np.empty(16)
    _load().orc_se3_exp(p, T.ctypes.data_as(_dp))
    return T.reshape(4, 4)


def se3_log(T) -> np.ndarray:
    T, p = _f64(T)
    xi = np.empty(6)
    _load().orc_se3_log(p, xi.ctypes.data_as(_dp))
    return xi


def cholesky_solve(H, b, rel_tol=1e-12):
    H, hp = _f64(H)
    b, bp = _f64(b)
    x = np.empty(6)
    fail = _load().orc_cholesky_solve(hp, bp, x.ctypes.data_as(_dp), rel_tol)
    return (None if fail else x)


def warp_jacobian(fx, fy, x0) -> np.ndarray:
    x0, p = _f64(x0)
    Jw = np.empty(12)
    _load().orc_warp_jacobian(fx, fy, p, Jw.ctypes.data_as(_dp))
    return Jw.reshape(2, 6)


# ----------------------------------------------------------------- tracker
DEFAULT_PATTERN = ((-2, 0), (2, 0), (0, -2), (0, 2), (-1, -1), (1, -1), (-1, 1), (1, 1))


def make_params(levels=3, max_iters=10, huber_k=9.0, step_eps=1e-5, min_points=10, pattern=DEFAULT_PATTERN,
                z_min=1e-3, fixed_h=False, gauss=False) -> Params:
    """gauss=True: track on the floating-point Gaussian pyramid instead of the uint8 box pyramid."""
    p = Params()
    p.levels, p.max_iters, p.huber_k, p.step_eps = levels, max_iters, huber_k, step_eps
    p.min_points, p.z_min, p.fixed_h = min_points, z_min, int(bool(fixed_h))
    p.pyramid = 1 if gauss else 0
    pat = np.asarray(pattern, np.int32).reshape(-1, 2)
    p.n_pattern = len(pat)
    for i, v in enumerate(pat.reshape(-1)):
        p.pattern[i] = int(v)
    return p


def make_camera(cam) -> Camera:
    return Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)


class Reference:
    """A reference frame with its IC precompute cache (Sec. IV-C)."""

    def __init__(self, cam, params: Params, ref_img: np.ndarray, points: np.ndarray, T_rw: np.ndarray):
        lib = _load()
        self._lib = lib
        self.cam = make_camera(cam) if not isinstance(cam, Camera) else cam
        self.params = params
        self.T_rw = np.array(T_rw, np.float64)
        self.n = int(len(points))
        img, ip = _u8(ref_img)
        pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
        T, tp = _f64(T_rw)
        self._h = lib.orc_ref_create(ctypes.byref(self.cam), ctypes.byref(params), ip, img.shape[1],
                                     pts.ctypes.data_as(_fp), self.n, tp)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_ref_free(self._h)
            self._h = None

    def cache(self, level: int):
        K = self.params.n_pattern
        n = self.n
        rv = np.empty(max(n, 1), np.uint8)
        I0 = np.empty(max(n * K, 1))
        g = np.empty(max(n * K * 2, 1))
        J = np.empty(max(n * K * 6, 1))
        x0 = np.empty(max(n * 3, 1))
        self._lib.orc_ref_cache(self._h, level, rv.ctypes.data_as(_u8p), I0.ctypes.data_as(_dp),
                                g.ctypes.data_as(_dp), J.ctypes.data_as(_dp), x0.ctypes.data_as(_dp))
        return dict(refvalid=rv[:n].astype(bool), I0=I0[:n * K].reshape(n, K), g=g[:n * K * 2].reshape(n, K, 2),
                    J=J[:n * K * 6].reshape(n, K, 6), x0=x0[:n * 3].reshape(n, 3))

    def fixed_h(self, level: int) -> np.ndarray:
        H = np.empty(36)
        self._lib.orc_ref_fixed_h(self._h, level, H.ctypes.data_as(_dp))
        return H.reshape(6, 6)

    def normal_equations(self, cur_img, level: int, T_rel: np.ndarray):
        img, ip = _u8(cur_img)
        T, tp = _f64(T_rel)
        H, b = np.empty(36), np.empty(6)
        E, n, npts = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int32()
        self._lib.orc_ref_normal_equations(self._h, ip, img.shape[1], level, tp, H.ctypes.data_as(_dp),
                                           b.ctypes.data_as(_dp), ctypes.byref(E), ctypes.byref(n), ctypes.byref(npts))
        return dict(H=H.reshape(6, 6), b=b, E=E.value, n=n.value, npts=npts.value)

    def track(self, cur_img: np.ndarray, T_cw_init: np.ndarray) -> dict:
        img, ip = _u8(cur_img)
        T, tp = _f64(T_cw_init)
        r = Result()
        self._lib.orc_ref_track(self._h, ip, img.shape[1], tp, ctypes.byref(r))
        return r.as_dict()


def track(cam, params: Params, ref_img, cur_img, points, T_rw, T_cw_init) -> dict:
    return Reference(cam, params, ref_img, points, T_rw).track(cur_img, T_cw_init)


def pose_error(T_a: np.ndarray, T_b: np.ndarray):
    """(rotation angle in rad, translation norm in m) of T_a T_b^-1."""
    Rb, tb = T_b[:3, :3], T_b[:3, 3]
    Ra, ta = T_a[:3, :3], T_a[:3, 3]
    R = Ra @ Rb.T
    t = ta - R @ tb
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    return float(np.arctan2(s, c)), float(np.linalg.norm(t))
