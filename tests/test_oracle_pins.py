"""Pins of the FP64 oracle against what the paper and mathematics fix.

Every check here compares the oracle with something other than itself: a
hand-worked example, a library routine (NumPy, SciPy), a closed form, an
invariant, or finite differences.  Citations name the paper's section or
equation each pinned function follows.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.special
from scipy.ndimage import map_coordinates

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _hat(xi):
    w, v = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    M[:3, 3] = v
    return M


# ------------------------------------------------------------------ pyramid (Sec. IV-C)
def test_pyramid_hand_example():
    g = json.load(open(os.path.join(GOLD, "pyramid_4x4.json")))
    levels = oracle.pyramid(np.array(g["image"], np.uint8), 3)
    for got, want in zip(levels, g["levels"]):
        np.testing.assert_array_equal(got, np.array(want, np.uint8))


@pytest.mark.parametrize("shape", [(37, 53), (480, 640), (31, 16)])
def test_pyramid_is_rounded_block_mean(shape):
    rng = np.random.default_rng(shape[0])
    img = rng.integers(0, 256, shape, dtype=np.uint8)
    levels = oracle.pyramid(img, 4)
    prev = img.astype(np.float64)
    for l in range(1, 4):
        h, w = prev.shape[0] // 2, prev.shape[1] // 2
        assert levels[l].shape == (h, w)  # floor sizes
        mean = prev[:2 * h, :2 * w].reshape(h, 2, w, 2).mean(axis=(1, 3))
        want = np.floor(mean + 0.5)  # round half up
        np.testing.assert_array_equal(levels[l], want.astype(np.uint8))
        prev = levels[l].astype(np.float64)
    np.testing.assert_array_equal(levels[0], img)


def test_pyramid_constant_and_extremes():
    for c in (0, 1, 128, 254, 255):
        for lv in oracle.pyramid(np.full((24, 40), c, np.uint8), 4):
            assert np.all(lv == c)


# ------------------------------------------------------------------ selection
def _brute_select(img, n, margin):
    gy, gx = np.gradient(img.astype(np.float64))  # central differences / 2 in the interior
    score = np.rint(4.0 * (gx * gx + gy * gy)).astype(np.int64)
    H, W = img.shape
    ys, xs = np.mgrid[0:H, 0:W]
    m = (xs >= margin) & (xs <= W - 1 - margin) & (ys >= margin) & (ys <= H - 1 - margin)
    idx = (ys * W + xs)[m]
    s = score[m]
    order = np.lexsort((idx, -s))
    return np.sort(idx[order[:n]])


@pytest.mark.parametrize("shape,n,margin", [((20, 30), 17, 1), ((20, 30), 1000, 3), ((64, 48), 100, 8)])
def test_selection_brute_force(shape, n, margin):
    rng = np.random.default_rng(7)
    img = rng.integers(0, 4, shape, dtype=np.uint8) * 20  # many ties
    np.testing.assert_array_equal(oracle.select_points(img, n, margin), _brute_select(img, n, margin))


def test_selection_rendered():
    d = synth.pair(3)
    np.testing.assert_array_equal(oracle.select_points(d["ref"], 500, 8), _brute_select(d["ref"], 500, 8))


# ------------------------------------------------------------------ sampling (Eq.(2), Sec. IV-C)
def test_bilinear_matches_map_coordinates():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (40, 50), dtype=np.uint8)
    pts = rng.uniform([1, 1], [47.999, 37.999], (300, 2))
    got = np.array([oracle.sample(img, x, y) for x, y in pts])
    want = map_coordinates(img.astype(np.float64), [pts[:, 1], pts[:, 0]], order=1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    # integer positions return the pixel
    assert oracle.sample(img, 7, 9) == img[9, 7]


def test_bilinear_and_gradient_exact_on_ramp():
    ys, xs = np.mgrid[0:30, 0:40]
    img = (10 + 3 * xs + 5 * ys).astype(np.uint8)
    rng = np.random.default_rng(2)
    for x, y in rng.uniform([1, 1], [37.99, 27.99], (100, 2)):
        assert abs(oracle.sample(img, x, y) - (10 + 3 * x + 5 * y)) < 1e-12
        gx, gy = oracle.gradient(img, x, y)
        assert abs(gx - 3) < 1e-12 and abs(gy - 5) < 1e-12


def test_gradient_is_interpolated_central_difference():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, (40, 50), dtype=np.uint8)
    gyi, gxi = np.gradient(img.astype(np.float64))
    pts = rng.uniform([1, 1], [46.999, 36.999], (300, 2))
    got = np.array([oracle.gradient(img, x, y) for x, y in pts])
    wx = map_coordinates(gxi, [pts[:, 1], pts[:, 0]], order=1)
    wy = map_coordinates(gyi, [pts[:, 1], pts[:, 0]], order=1)
    np.testing.assert_allclose(got[:, 0], wx, atol=1e-12)
    np.testing.assert_allclose(got[:, 1], wy, atol=1e-12)


# ------------------------------------------------------------------ SE(3) (Sec. IV-A update)
def test_exp_matches_expm():
    rng = np.random.default_rng(4)
    for scale in (1e-7, 1e-5, 3e-4, 0.1, 1.0, 2.5):
        for _ in range(20):
            xi = rng.normal(size=6) * scale
            np.testing.assert_allclose(oracle.se3_exp(xi), scipy.linalg.expm(_hat(xi)), rtol=0, atol=1e-13)
    np.testing.assert_array_equal(oracle.se3_exp(np.zeros(6)), np.eye(4))


def test_log_inverts_exp():
    rng = np.random.default_rng(5)
    for scale in (1e-6, 1e-3, 0.3, 1.2):
        for _ in range(20):
            xi = rng.normal(size=6) * scale
            if np.linalg.norm(xi[:3]) > 3.0:  # log is unique only for rotation angles below pi
                continue
            np.testing.assert_allclose(oracle.se3_log(oracle.se3_exp(xi)), xi, rtol=1e-9, atol=1e-12)
    # and against scipy's matrix logarithm
    xi = np.array([0.3, -0.2, 0.5, 1.0, -2.0, 0.5])
    L = scipy.linalg.logm(oracle.se3_exp(xi)).real
    np.testing.assert_allclose(oracle.se3_log(oracle.se3_exp(xi)),
                               [L[2, 1], L[0, 2], L[1, 0], L[0, 3], L[1, 3], L[2, 3]], atol=1e-10)


# ------------------------------------------------------------------ Cholesky solve (Sec. IV-C)
def test_cholesky_solve_matches_numpy():
    rng = np.random.default_rng(6)
    for _ in range(50):
        A = rng.normal(size=(6, 6)) * rng.uniform(0.1, 1e3, 6)
        H = A @ A.T + 1e-3 * np.eye(6)
        b = rng.normal(size=6)
        np.testing.assert_allclose(oracle.cholesky_solve(H, b), np.linalg.solve(H, b), rtol=1e-8)


def test_cholesky_rejects_singular_and_indefinite():
    v = np.arange(1.0, 7.0)
    assert oracle.cholesky_solve(np.outer(v, v), np.ones(6)) is None      # rank 1
    assert oracle.cholesky_solve(np.zeros((6, 6)), np.zeros(6)) is None   # constant image
    assert oracle.cholesky_solve(np.diag([1, 1, 1, 1, 1, -1.0]), np.ones(6)) is None


# ------------------------------------------------------------------ Jacobians (Eq.(6))
def test_warp_jacobian_hand_example():
    g = json.load(open(os.path.join(GOLD, "warp_jacobian_example.json")))
    np.testing.assert_allclose(np.array(g["dpi_dx"]) @ np.array(g["dx_ddelta"]), g["Jw"], atol=0)
    np.testing.assert_allclose(oracle.warp_jacobian(g["fx"], g["fy"], g["x0"]), g["Jw"], rtol=1e-15)


def test_warp_jacobian_finite_differences():
    rng = np.random.default_rng(8)
    for _ in range(30):
        x0 = rng.uniform([-2, -2, 0.5], [2, 2, 5])
        fx, fy = rng.uniform(100, 900, 2)

        def proj(xi):
            x = scipy.linalg.expm(_hat(xi)) @ np.append(x0, 1.0)
            return np.array([fx * x[0] / x[2], fy * x[1] / x[2]])

        h = 1e-6
        fd = np.column_stack([(proj(h * e) - proj(-h * e)) / (2 * h) for e in np.eye(6)])
        Jw = oracle.warp_jacobian(fx, fy, x0)
        np.testing.assert_allclose(Jw, fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())


def _params(**kw):
    kw.setdefault("levels", 3)
    return oracle.make_params(**kw)


def test_full_jacobian_finite_differences_on_ramp():
    """J_ik = grad I0 * dpi/dx * dx/ddelta: on a linear ramp the bilinear template is exactly
    linear, so finite differences of the warped template give J exactly."""
    cam = synth.Camera(64, 48, 60.0, 60.0, 31.5, 23.5)
    ys, xs = np.mgrid[0:48, 0:64]
    img = (20 + 2 * xs + 3 * ys).astype(np.uint8)
    rng = np.random.default_rng(9)
    px = rng.uniform([12, 12], [50, 34], (6, 2))
    z = rng.uniform(1, 3, 6)
    P = np.column_stack([(px[:, 0] - cam.cx) / cam.fx * z, (px[:, 1] - cam.cy) / cam.fy * z, z]).astype(np.float32)
    prm = _params(levels=1)
    ref = oracle.Reference(cam, prm, img, P, np.eye(4))
    c = ref.cache(0)
    assert c["refvalid"].all()
    pat = np.array(oracle.DEFAULT_PATTERN, float)
    for i in range(6):
        x0 = c["x0"][i]
        for k in range(8):
            def tmpl(xi):
                x = scipy.linalg.expm(_hat(xi)) @ np.append(x0, 1.0)
                u = cam.fx * x[0] / x[2] + cam.cx + pat[k, 0]
                v = cam.fy * x[1] / x[2] + cam.cy + pat[k, 1]
                return 20 + 2 * u + 3 * v
            h = 1e-6
            fd = np.array([(tmpl(h * e) - tmpl(-h * e)) / (2 * h) for e in np.eye(6)])
            np.testing.assert_allclose(c["J"][i, k], fd, rtol=1e-6, atol=1e-6)


# ------------------------------------------------------------------ normal equations (Eq.(2),(5))
def _level_camera(cam, l):
    s = 2.0 ** l
    return cam.fx / s, cam.fy / s, (cam.cx + 0.5) / s - 0.5, (cam.cy + 0.5) / s - 0.5


def _brute_normal_equations(d, P, l, T_rel, k_huber, prm):
    """Independent assembly: gradients from np.gradient, sampling from map_coordinates,
    Jw from finite differences of scipy's expm, weights from scipy.special.huber."""
    cam = d["cam"]
    ref_l = oracle.pyramid(d["ref"], prm.levels)[l].astype(np.float64)
    cur_l = oracle.pyramid(d["cur"], prm.levels)[l].astype(np.float64)
    Hl, Wl = ref_l.shape
    fx, fy, cx, cy = _level_camera(cam, l)
    gyi, gxi = np.gradient(ref_l)
    pat = np.array(oracle.DEFAULT_PATTERN, float)
    H = np.zeros((6, 6))
    b = np.zeros(6)
    E, n, npts = 0.0, 0, 0

    def inside(u, v):
        return np.all((u >= 1) & (u < Wl - 2) & (v >= 1) & (v < Hl - 2))

    def rho(r):
        return scipy.special.huber(k_huber, r) if k_huber > 0 else 0.5 * r * r

    for p in P.astype(np.float64):
        x0 = p  # T_rw = I
        u0, v0 = fx * x0[0] / x0[2] + cx + pat[:, 0], fy * x0[1] / x0[2] + cy + pat[:, 1]
        if not inside(u0, v0):
            continue
        x = T_rel[:3, :3] @ x0 + T_rel[:3, 3]
        u, v = fx * x[0] / x[2] + cx + pat[:, 0], fy * x[1] / x[2] + cy + pat[:, 1]
        if not (x[2] > 1e-3 and inside(u, v)):
            continue
        npts += 1

        def proj(xi):
            y = scipy.linalg.expm(_hat(xi)) @ np.append(x0, 1.0)
            return np.array([fx * y[0] / y[2], fy * y[1] / y[2]])

        h = 1e-7
        Jw = np.column_stack([(proj(h * e) - proj(-h * e)) / (2 * h) for e in np.eye(6)])
        I0 = map_coordinates(ref_l, [v0, u0], order=1)
        g = np.column_stack([map_coordinates(gxi, [v0, u0], order=1), map_coordinates(gyi, [v0, u0], order=1)])
        r = I0 - map_coordinates(cur_l, [v, u], order=1)
        for kk in range(len(pat)):
            J = g[kk] @ Jw
            hh = 1e-6
            w = (rho(r[kk] + hh) - rho(r[kk] - hh)) / (2 * hh) / r[kk] if abs(r[kk]) > 1e-3 else 1.0
            H += w * np.outer(J, J)
            b -= w * J * r[kk]
            E += rho(r[kk])
            n += 1
    return H, b, E, n, npts


@pytest.mark.parametrize("k_huber", [9.0, 0.0])
def test_normal_equations_brute_force(k_huber):
    d = synth.pair(11)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(oracle.select_points(d["ref"], 400, 8), 12, replace=False))
    P = synth.backproject(d["cam"], d["depth"], idx, d["T_rw"])
    prm = _params(levels=3, huber_k=k_huber)
    ref = oracle.Reference(d["cam"], prm, d["ref"], P, np.eye(4))
    T_rel = oracle.se3_exp(np.array([0.002, -0.003, 0.001, 0.004, -0.002, 0.003]))
    for l in (0, 1):
        ne = ref.normal_equations(d["cur"], l, T_rel)
        H, b, E, n, npts = _brute_normal_equations(d, P, l, T_rel, k_huber, prm)
        assert ne["npts"] == npts and ne["n"] == n and npts > 3
        scale = np.abs(H).max()
        np.testing.assert_allclose(ne["H"], H, atol=2e-6 * scale)
        np.testing.assert_allclose(ne["b"], b, atol=2e-6 * np.abs(b).max())
        assert abs(ne["E"] - E) <= 1e-9 * max(1.0, E)


@pytest.mark.parametrize("k_huber", [9.0, 0.0])
def test_final_cost_brute_force(k_huber):
    """The returned cost is the mean rho over the level-0 samples valid at the
    returned pose, and the valid-point count is theirs (Sec. IV-C: the track
    hands back a valid pose with its robust photometric error); checked against
    the independent assembly above at that pose."""
    d = synth.pair(14)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(oracle.select_points(d["ref"], 400, 8), 30, replace=False))
    P = synth.backproject(d["cam"], d["depth"], idx, d["T_rw"])
    prm = _params(levels=3, huber_k=k_huber)
    ref = oracle.Reference(d["cam"], prm, d["ref"], P, np.eye(4))
    r = ref.track(d["cur"], oracle.se3_exp(np.array([0.001, 0.0, -0.001, 0.002, 0.0, 0.001])))
    assert r["status"] in (oracle.OK, oracle.MAX_ITERS)
    assert r["iterations"] == sum(r["iters_per_level"][:3])
    _, _, E, n, npts = _brute_normal_equations(d, P, 0, r["T_cw"], k_huber, prm)
    assert r["n_valid_points"] == npts and n == 8 * npts and npts >= 10
    assert abs(r["final_cost"] - E / n) <= 1e-9 * max(1.0, E / n)


def test_fixed_h_equals_irls_without_weights():
    """Paper mode (H reduced once per reference, Sec. IV-B) equals the re-reduced H
    when no weights apply and every reference-valid point stays valid."""
    d = synth.pair(12)
    P = synth.backproject(d["cam"], d["depth"], oracle.select_points(d["ref"], 200, 8), d["T_rw"])
    ref = oracle.Reference(d["cam"], _params(huber_k=0.0), d["ref"], P, np.eye(4))
    for l in range(3):
        ne = ref.normal_equations(d["ref"], l, np.eye(4))
        assert ne["npts"] == ref.cache(l)["refvalid"].sum()
        np.testing.assert_allclose(ne["H"], ref.fixed_h(l), rtol=1e-12, atol=1e-9)


def test_huber_weights_from_library_rho():
    """IRLS weight w = rho'(r)/r for scipy.special.huber: at k = 9 the weighted residual
    sum b and cost E of a single large residual follow the linear branch."""
    d = synth.pair(13)
    P = synth.backproject(d["cam"], d["depth"], oracle.select_points(d["ref"], 50, 8), d["T_rw"])
    big = oracle.Reference(d["cam"], _params(huber_k=1e9), d["ref"], P, np.eye(4))
    hub = oracle.Reference(d["cam"], _params(huber_k=0.5), d["ref"], P, np.eye(4))
    a = big.normal_equations(d["cur"], 0, np.eye(4))
    c = hub.normal_equations(d["cur"], 0, np.eye(4))
    assert a["n"] == c["n"]
    assert c["E"] < a["E"]  # Huber grows linearly past k
    np.testing.assert_allclose(np.linalg.eigvalsh(c["H"]).max() <= np.linalg.eigvalsh(a["H"]).max() + 1e-9, True)


# ------------------------------------------------------------------ whole tracker (Sec. IV-A, IV-C)
def _setup(seed, n=500, **kw):
    d = synth.pair(seed)
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(d["cam"], d["depth"], idx, d["T_rw"])
    prm = _params(**kw)
    return d, P, oracle.Reference(d["cam"], prm, d["ref"], P, d["T_rw"])


def test_identity_on_identical_frames():
    d, P, ref = _setup(0)
    r = ref.track(d["ref"], np.eye(4))
    np.testing.assert_array_equal(r["T_cw"], np.eye(4))
    assert r["final_cost"] == 0.0 and r["iterations"] == 3 and r["status"] == oracle.OK
    assert r["iters_per_level"][:3] == [1, 1, 1]


@pytest.mark.parametrize("seed", list(range(0, 100, 9)))
def test_perturbation_recovery(seed):
    """Rendered GT perturbation (<= 1 deg, <= 2 cm) is recovered, and the result is the same
    fixed point as when starting at GT.  A wrong update sign or side diverges."""
    d, P, ref = _setup(seed)
    r = ref.track(d["cur"], np.eye(4))
    g = ref.track(d["cur"], d["T_cw_gt"])
    rot, tr = oracle.pose_error(r["T_cw"], d["T_cw_gt"])
    assert r["status"] == oracle.OK
    # the floor left by rasterisation, quantisation and bilinear error is
    # ~0.002-0.015 deg / 0.2-0.8 mm on these seeds
    assert np.rad2deg(rot) < 0.05 and tr < 2e-3
    rot0, tr0 = oracle.pose_error(np.eye(4), d["T_cw_gt"])
    # where the start is well above that floor, the error shrinks at least 8x
    if np.rad2deg(rot0) > 0.05:
        assert rot < rot0 / 8
    if tr0 > 4e-3:
        assert tr < tr0 / 8
    rot2, tr2 = oracle.pose_error(r["T_cw"], g["T_cw"])
    assert rot2 < 1e-8 and tr2 < 1e-8


def test_near_zero_residual_at_ground_truth():
    d, P, ref = _setup(1)
    at_gt = ref.normal_equations(d["cur"], 0, d["T_cw_gt"])
    at_id = ref.normal_equations(d["cur"], 0, np.eye(4))
    assert at_gt["E"] / at_gt["n"] < 2.0          # mean rho, intensity levels^2 / 2
    assert at_id["E"] / at_id["n"] > 10 * at_gt["E"] / at_gt["n"]


def test_world_frame_equivariance():
    """Moving the world by G (points G P, reference T_rw G^-1, start T_init G^-1) maps the
    result to T_out G^-1."""
    d, P, ref = _setup(2)
    r = ref.track(d["cur"], np.eye(4))
    G = oracle.se3_exp(np.array([0.3, -0.5, 0.2, 1.0, -2.0, 0.5]))
    Gi = np.linalg.inv(G)
    P2 = (P.astype(np.float64) @ G[:3, :3].T + G[:3, 3]).astype(np.float32)
    ref2 = oracle.Reference(d["cam"], ref.params, d["ref"], P2, d["T_rw"] @ Gi)
    r2 = ref2.track(d["cur"], Gi)
    rot, tr = oracle.pose_error(r2["T_cw"], r["T_cw"] @ Gi)
    # the moved points are rounded to float32 again (~2e-7 m), hence not 1e-12
    assert rot < 1e-8 and tr < 1e-8


def test_failure_statuses():
    d, P, ref = _setup(4)
    # constant current image: no gradients matter, but the reference still has them;
    # a constant reference gives H = 0 -> not positive definite
    flat = np.full_like(d["ref"], 100)
    ref_flat = oracle.Reference(d["cam"], ref.params, flat, P, np.eye(4))
    assert ref_flat.track(flat, np.eye(4))["status"] == oracle.NOT_PD
    # all points behind the camera
    behind = np.eye(4)
    behind[2, 3] = -10.0
    assert ref.track(d["cur"], behind)["status"] == oracle.TOO_FEW_POINTS
    # iteration cap
    capped = oracle.Reference(d["cam"], _params(max_iters=1), d["ref"], P, np.eye(4))
    assert capped.track(d["cur"], np.eye(4))["status"] == oracle.MAX_ITERS


# ------------------------------------------------------------------ fixed-H mode (Sec. IV-B, IV-C)
def _brute_fixed_h(d, P, l, prm):
    """Independent assembly of the constant H of one level: sum of J^T J over the
    points whose every pattern position lies inside the reference level (the
    precompute runs before any current frame exists), with J from np.gradient,
    map_coordinates and finite differences of scipy's expm; T_rw = I."""
    cam = d["cam"]
    ref_l = oracle.pyramid(d["ref"], prm.levels)[l].astype(np.float64)
    Hl, Wl = ref_l.shape
    fx, fy, cx, cy = _level_camera(cam, l)
    gyi, gxi = np.gradient(ref_l)
    pat = np.array(oracle.DEFAULT_PATTERN, float)
    H = np.zeros((6, 6))
    for x0 in P.astype(np.float64):
        u0, v0 = fx * x0[0] / x0[2] + cx + pat[:, 0], fy * x0[1] / x0[2] + cy + pat[:, 1]
        if not np.all((u0 >= 1) & (u0 < Wl - 2) & (v0 >= 1) & (v0 < Hl - 2)):
            continue

        def proj(xi):
            y = scipy.linalg.expm(_hat(xi)) @ np.append(x0, 1.0)
            return np.array([fx * y[0] / y[2], fy * y[1] / y[2]])

        h = 1e-7
        Jw = np.column_stack([(proj(h * e) - proj(-h * e)) / (2 * h) for e in np.eye(6)])
        g = np.column_stack([map_coordinates(gxi, [v0, u0], order=1), map_coordinates(gyi, [v0, u0], order=1)])
        for kk in range(len(pat)):
            J = g[kk] @ Jw
            H += np.outer(J, J)
    return H


def test_fixed_h_normal_equations_brute_force():
    """Fixed-H mode at a pose where some residuals exceed the Huber threshold and
    some reference-valid points leave the current level: H is the constant H of
    that level (over the reference-valid points), b and E are unweighted (w = 1,
    rho = r^2 / 2) over the points valid in the current frame, whatever huber_k is."""
    d = synth.pair(11)
    rng = np.random.default_rng(5)
    cand = oracle.select_points(d["ref"], 2000, 8)
    # half the points from the border band, so a shift moves some out of the level
    H0, W0 = d["ref"].shape
    ys, xs = cand // W0, cand % W0
    near = (xs < 40) | (xs > W0 - 41) | (ys < 40) | (ys > H0 - 41)
    idx = np.sort(np.concatenate([rng.choice(cand[near], 10, replace=False),
                                  rng.choice(cand[~near], 10, replace=False)]))
    P = synth.backproject(d["cam"], d["depth"], idx, d["T_rw"])
    prm = _params(levels=3, huber_k=9.0, fixed_h=True)
    ref = oracle.Reference(d["cam"], prm, d["ref"], P, np.eye(4))
    T_rel = oracle.se3_exp(np.array([0.01, -0.012, 0.004, 0.05, -0.03, 0.02]))
    Hs = []
    for l in range(3):
        ne = ref.normal_equations(d["cur"], l, T_rel)
        Hb = _brute_fixed_h(d, P, l, prm)
        _, b0, E0, n, npts = _brute_normal_equations(d, P, l, T_rel, 0.0, prm)
        _, b9, E9, _, _ = _brute_normal_equations(d, P, l, T_rel, 9.0, prm)
        assert ne["npts"] == npts and ne["n"] == n and npts > 3
        np.testing.assert_allclose(ne["H"], Hb, atol=2e-6 * np.abs(Hb).max())
        np.testing.assert_allclose(ne["b"], b0, atol=2e-6 * np.abs(b0).max())
        assert abs(ne["E"] - E0) <= 1e-9 * max(1.0, E0)
        # the case distinguishes the modes: weights and the Huber cost would show
        assert np.abs(b9 - b0).max() > 1e-3 * np.abs(b0).max() and E9 < 0.99 * E0
        Hs.append(Hb)
    # some reference-valid points are outside the current level 0, so the
    # constant H is not the one of the current-valid points
    assert ref.cache(0)["refvalid"].sum() > ref.normal_equations(d["cur"], 0, T_rel)["npts"]
    # every level's H is its own: a wrong level index would fail above
    for a in range(3):
        for c in range(a + 1, 3):
            assert np.abs(Hs[a] - Hs[c]).max() > 0.1 * np.abs(Hs[c]).max()


def test_fixed_h_track_equals_irls_without_weights_when_all_points_stay_valid():
    """With every reference-valid point valid in the current frame at every
    iteration, the constant H equals the re-reduced unweighted H, so the paper's
    track and the unweighted IRLS track take the same steps."""
    d = synth.pair(21)
    P = synth.backproject(d["cam"], d["depth"], oracle.select_points(d["ref"], 300, 60), d["T_rw"])
    fixed = oracle.Reference(d["cam"], _params(huber_k=9.0, fixed_h=True), d["ref"], P, d["T_rw"])
    irls = oracle.Reference(d["cam"], _params(huber_k=0.0), d["ref"], P, d["T_rw"])
    a = fixed.track(d["cur"], np.eye(4))
    b = irls.track(d["cur"], np.eye(4))
    assert a["status"] == b["status"] == oracle.OK
    assert a["iters_per_level"] == b["iters_per_level"]
    np.testing.assert_allclose(a["T_cw"], b["T_cw"], rtol=0, atol=1e-12)
    assert abs(a["final_cost"] - b["final_cost"]) <= 1e-12 * max(1.0, b["final_cost"])
    assert a["n_valid_points"] == b["n_valid_points"] == len(P)


@pytest.mark.parametrize("seed", [0, 17, 45, 80])
def test_fixed_h_perturbation_recovery(seed):
    """The paper's constant-H track recovers the rendered perturbation: from the
    identity it reaches the fixed point it reaches from the true pose."""
    d, P, ref = _setup(seed, fixed_h=True)
    r = ref.track(d["cur"], np.eye(4))
    g = ref.track(d["cur"], d["T_cw_gt"])
    rot, tr = oracle.pose_error(r["T_cw"], d["T_cw_gt"])
    rot0, tr0 = oracle.pose_error(np.eye(4), d["T_cw_gt"])
    assert r["status"] in (oracle.OK, oracle.MAX_ITERS)
    assert np.rad2deg(rot) < 0.1 and tr < 4e-3
    assert tr < 0.5 * tr0 or tr0 < 2e-3
    rot2, tr2 = oracle.pose_error(r["T_cw"], g["T_cw"])
    assert rot2 < 1e-8 and tr2 < 1e-8


def test_fixed_h_final_cost_brute_force():
    """The fixed-H track returns the unweighted mean cost r^2 / 2 over the level-0
    samples valid at the returned pose, whatever huber_k is."""
    d = synth.pair(14)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(oracle.select_points(d["ref"], 400, 8), 30, replace=False))
    P = synth.backproject(d["cam"], d["depth"], idx, d["T_rw"])
    ref = oracle.Reference(d["cam"], _params(levels=3, huber_k=1.0, fixed_h=True), d["ref"], P, np.eye(4))
    r = ref.track(d["cur"], oracle.se3_exp(np.array([0.001, 0.0, -0.001, 0.002, 0.0, 0.001])))
    assert r["status"] in (oracle.OK, oracle.MAX_ITERS)
    _, _, E0, n, npts = _brute_normal_equations(d, P, 0, r["T_cw"], 0.0, _params(levels=3))
    _, _, E1, _, _ = _brute_normal_equations(d, P, 0, r["T_cw"], 1.0, _params(levels=3))
    assert r["n_valid_points"] == npts and n == 8 * npts and npts >= 10
    assert abs(r["final_cost"] - E0 / n) <= 1e-9 * max(1.0, E0 / n)
    assert E1 < 0.99 * E0  # the Huber cost at k = 1 would differ
