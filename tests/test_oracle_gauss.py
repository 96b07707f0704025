"""Pins of the oracle's floating-point Gaussian pyramid (Sec. IV-C, image
pyramids: a frame in floating point, blurred by a vertical and a horizontal
pass, then downsampled) and of the tracker running on it.  Each check compares
with something other than the oracle: SciPy's 1-D correlation, a brute-force
2-D sum, closed forms on constant and ramp images, and the tracker invariants."""
import numpy as np
import pytest
from scipy.ndimage import correlate1d, map_coordinates

import oracle
import synth

W4 = np.array([1.0, 3.0, 3.0, 1.0]) / 8.0


def _scipy_level(prev):
    """One level with SciPy: taps at 2y-1 .. 2y+2 (origin -1 of a 4-tap
    correlation), clamped borders ('nearest'), then every second sample."""
    h2, w2 = prev.shape[0] // 2, prev.shape[1] // 2
    v = correlate1d(prev, W4, axis=0, mode="nearest", origin=-1)[0:2 * h2:2]
    return correlate1d(v, W4, axis=1, mode="nearest", origin=-1)[:, 0:2 * w2:2]


def _brute_level(prev):
    h, w = prev.shape
    out = np.zeros((h // 2, w // 2))
    for y in range(h // 2):
        for x in range(w // 2):
            s = 0.0
            for i in range(4):
                for j in range(4):
                    yy = min(max(2 * y - 1 + i, 0), h - 1)
                    xx = min(max(2 * x - 1 + j, 0), w - 1)
                    s += W4[i] * W4[j] * prev[yy, xx]
            out[y, x] = s
    return out


@pytest.mark.parametrize("shape,levels", [((37, 53), 4), ((480, 752), 6), ((31, 16), 2), ((64, 64), 7)])
def test_gauss_pyramid_matches_scipy(shape, levels):
    img = np.random.default_rng(shape[0]).integers(0, 256, shape, dtype=np.uint8)
    pyr = oracle.pyramid_gauss(img, levels)
    np.testing.assert_array_equal(pyr[0], img.astype(np.float64))
    for l in range(1, levels):
        assert pyr[l].shape == (shape[0] >> l, shape[1] >> l)
        np.testing.assert_allclose(pyr[l], _scipy_level(pyr[l - 1]), rtol=0, atol=1e-10)


def test_gauss_pyramid_brute_force_2d():
    img = np.random.default_rng(5).integers(0, 256, (23, 30), dtype=np.uint8)
    pyr = oracle.pyramid_gauss(img, 3)
    np.testing.assert_allclose(pyr[1], _brute_level(img.astype(np.float64)), rtol=0, atol=1e-10)
    np.testing.assert_allclose(pyr[2], _brute_level(pyr[1]), rtol=0, atol=1e-10)


def test_gauss_pyramid_constant_and_ramp():
    flat = np.full((40, 60), 137, np.uint8)
    for lev in oracle.pyramid_gauss(flat, 4):
        assert np.all(lev == 137.0)
    # a linear ramp stays linear; level-1 pixel x lies at level-0 position 2x + 1/2
    ys, xs = np.mgrid[0:48, 0:64]
    ramp = (10 + xs + 2 * ys).astype(np.uint8)  # at most 167: no wrap
    p1 = oracle.pyramid_gauss(ramp, 2)[1]
    y1, x1 = np.mgrid[1:23, 1:31]  # away from the clamped borders
    np.testing.assert_allclose(p1[1:23, 1:31], 10 + (2 * x1 + 0.5) + 2 * (2 * y1 + 0.5), atol=1e-12)


def test_sample_and_gradient_on_float_levels():
    rng = np.random.default_rng(9)
    img = rng.uniform(0, 255, (40, 50))
    pts = rng.uniform([1, 1], [46.999, 36.999], (200, 2))
    got = np.array([oracle.sample_f(img, x, y) for x, y in pts])
    np.testing.assert_allclose(got, map_coordinates(img, [pts[:, 1], pts[:, 0]], order=1), atol=1e-10)
    gyi, gxi = np.gradient(img)
    g = np.array([oracle.gradient_f(img, x, y) for x, y in pts])
    np.testing.assert_allclose(g[:, 0], map_coordinates(gxi, [pts[:, 1], pts[:, 0]], order=1), atol=1e-10)
    np.testing.assert_allclose(g[:, 1], map_coordinates(gyi, [pts[:, 1], pts[:, 0]], order=1), atol=1e-10)
    # on uint8 data the float path equals the uint8 one exactly
    u8 = rng.integers(0, 256, (40, 50), dtype=np.uint8)
    for x, y in pts[:50]:
        assert oracle.sample_f(u8.astype(np.float64), x, y) == oracle.sample(u8, x, y)
        assert oracle.gradient_f(u8.astype(np.float64), x, y) == oracle.gradient(u8, x, y)


def _setup(seed, n=500, levels=3, **kw):
    d = synth.pair(seed)
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(d["cam"], d["depth"], idx, d["T_rw"])
    prm = oracle.make_params(levels=levels, gauss=True, **kw)
    return d, P, oracle.Reference(d["cam"], prm, d["ref"], P, d["T_rw"])


def test_gauss_tracker_identity():
    d, P, ref = _setup(0)
    r = ref.track(d["ref"], np.eye(4))
    np.testing.assert_array_equal(r["T_cw"], np.eye(4))
    assert r["final_cost"] == 0.0 and r["status"] == oracle.OK


@pytest.mark.parametrize("seed", [0, 11, 29, 47, 83])
def test_gauss_tracker_recovers_perturbation(seed):
    d, P, ref = _setup(seed)
    r = ref.track(d["cur"], np.eye(4))
    g = ref.track(d["cur"], d["T_cw_gt"])
    rot, tr = oracle.pose_error(r["T_cw"], d["T_cw_gt"])
    assert r["status"] == oracle.OK
    assert np.rad2deg(rot) < 0.1 and tr < 4e-3
    rot2, tr2 = oracle.pose_error(r["T_cw"], g["T_cw"])
    assert rot2 < 1e-8 and tr2 < 1e-8


def test_gauss_paper_shape_six_levels_7x7():
    """The paper's own shape: 6 pyramid levels and 7x7 patches on a 752x480 pair."""
    cam = synth.CAM_752
    d = synth.pair(3, cam)
    idx = oracle.select_points(d["ref"], 400, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    prm = oracle.make_params(levels=6, gauss=True, pattern=synth.square_pattern(7))
    ref = oracle.Reference(cam, prm, d["ref"], P, d["T_rw"])
    r = ref.track(d["cur"], np.eye(4))
    rot, tr = oracle.pose_error(r["T_cw"], d["T_cw_gt"])
    assert r["status"] in (oracle.OK, oracle.MAX_ITERS)
    assert np.rad2deg(rot) < 0.1 and tr < 4e-3
