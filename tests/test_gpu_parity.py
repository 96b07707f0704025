"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Bit-exact for pyramids and point selection; pose within
1e-4 rad / 1e-4 m and final cost within 1e-3 relative for the tracker."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL, COST_TOL = 1e-4, 1e-4, 1e-3


def _oparams(p):
    pat = np.array(p.pattern[:2 * p.n_pattern]).reshape(-1, 2)
    return oracle.make_params(levels=p.levels, max_iters=p.max_iters, huber_k=p.huber_k, step_eps=p.step_eps,
                              min_points=p.min_points, pattern=pat, z_min=p.z_min)


def _tracker(dpt, cam, n, **kw):
    prm = dpt.make_params(**kw)
    return dpt.Tracker(cam, prm, max_points=max(n, 1)), prm


# ------------------------------------------------------------------ pyramid
@pytest.mark.parametrize("cam,levels", [(synth.CAM_640, 3), (synth.CAM_752, 4), (synth.CAM_1280, 4),
                                        (synth.Camera(645, 483, 400, 400, 320, 240), 6),
                                        (synth.Camera(1023, 767, 500, 500, 511, 383), 7),
                                        (synth.Camera(2047, 1535, 900, 900, 1023, 767), 8),
                                        (synth.Camera(130, 70, 100, 100, 65, 35), 1)])
def test_pyramid_bit_exact(gpu_lib, cam, levels):
    import torch

    dpt = gpu_lib
    rng = np.random.default_rng(cam.width)
    img = rng.integers(0, 256, (cam.height, cam.width), dtype=np.uint8)
    trk, _ = _tracker(dpt, cam, 10, levels=levels)
    want = oracle.pyramid(img, levels)
    # host input
    trk.build_pyramid(dpt.SLOT_CUR, img)
    for l in range(levels):
        np.testing.assert_array_equal(trk.get_pyramid(dpt.SLOT_CUR, l), want[l])
    # device input with a padded pitch
    pitch = cam.width + 37
    padded = np.zeros((cam.height, pitch), np.uint8)
    padded[:, :cam.width] = img
    dev = torch.from_numpy(padded).cuda()
    trk.build_pyramid(dpt.SLOT_REF, dev, pitch=pitch)
    torch.cuda.synchronize()
    for l in range(levels):
        np.testing.assert_array_equal(trk.get_pyramid(dpt.SLOT_REF, l), want[l])


# ------------------------------------------------------------------ selection
@pytest.mark.parametrize("case", ["c1", "c2", "hd16k", "ties", "all", "odd", "m4"])
def test_selection_bit_exact(gpu_lib, case):
    """c1, c2, hd16k and m4 take the four-candidate reads (aligned rows, a
    margin that is a multiple of 4, candidate rows a multiple of 4 long; m4 at
    the smallest such margin, whose left word starts at column 0); ties, all
    and odd (45 candidates per row) the one-candidate reads."""
    dpt = gpu_lib
    if case == "c1":
        img, cam, n, m = synth.pair(0)["ref"], synth.CAM_640, 500, 8
    elif case == "c2":
        _, img, _, _ = next(synth.sequence_frames(n_frames=1))
        cam, n, m = synth.CAM_752, 2000, 8
    elif case == "hd16k":
        cam = synth.CAM_1280
        img = synth.Scene(5).render(cam, np.eye(4), want_depth=False)[0]
        n, m = 16000, 8
    elif case == "ties":
        cam = synth.Camera(200, 100, 100, 100, 100, 50)
        img = (np.random.default_rng(1).integers(0, 3, (100, 200)) * 40).astype(np.uint8)
        n, m = 3000, 3
    elif case == "odd":
        cam = synth.Camera(61, 50, 50, 50, 30, 25)
        img = np.random.default_rng(3).integers(0, 256, (50, 61), dtype=np.uint8)
        n, m = 700, 8
    elif case == "m4":
        cam = synth.Camera(68, 44, 50, 50, 34, 22)
        img = np.random.default_rng(4).integers(0, 256, (44, 68), dtype=np.uint8)
        n, m = 900, 4
    else:
        cam = synth.Camera(64, 40, 50, 50, 32, 20)
        img = np.random.default_rng(2).integers(0, 256, (40, 64), dtype=np.uint8)
        n, m = 2500, 1  # more than the 62 x 38 candidates: take all
    trk, _ = _tracker(dpt, cam, 10, levels=1)
    trk.build_pyramid(dpt.SLOT_REF, img)
    got = trk.select_points(n, m)
    np.testing.assert_array_equal(got, oracle.select_points(img, n, m))


# ------------------------------------------------------------------ precompute cache
def _pair_setup(dpt, seed=0, n=500, levels=3, cam=synth.CAM_640, launch=None, **kw):
    d = synth.pair(seed, cam)
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    trk, prm = _tracker(dpt, cam, n, levels=levels, **kw)
    if launch is not None:
        trk.set_launch_config(*launch)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    ref = oracle.Reference(cam, _oparams(prm), d["ref"], P, d["T_rw"])
    return d, P, trk, ref


def test_precompute_cache_matches_oracle(gpu_lib):
    d, P, trk, ref = _pair_setup(gpu_lib)
    for l in range(3):
        g, o = trk.reference_cache(l), ref.cache(l)
        agree = g["valid"] == o["refvalid"]
        assert agree.mean() > 0.995
        both = g["valid"] & o["refvalid"]
        np.testing.assert_allclose(g["I0"][both], o["I0"][both], atol=2e-3)
        np.testing.assert_allclose(g["gx"][both], o["g"][both][..., 0], atol=2e-3)
        np.testing.assert_allclose(g["gy"][both], o["g"][both][..., 1], atol=2e-3)
        np.testing.assert_allclose(g["x0"], o["x0"], rtol=1e-6, atol=1e-6)


def test_normal_equations_match_oracle(gpu_lib):
    d, P, trk, ref = _pair_setup(gpu_lib, seed=3)
    T_rel = oracle.se3_exp(np.array([0.002, -0.001, 0.003, 0.004, 0.002, -0.003]))
    for l in range(3):
        g = trk.normal_equations(l, T_rel)
        o = ref.normal_equations(d["cur"], l, T_rel)
        assert abs(g["npts"] - o["npts"]) <= 1
        if g["npts"] != o["npts"]:
            continue
        assert g["n"] == o["n"]
        scale = np.abs(o["H"]).max()
        np.testing.assert_allclose(g["H"], o["H"], atol=2e-4 * scale)
        np.testing.assert_allclose(g["b"], o["b"], atol=2e-4 * np.abs(o["b"]).max())
        assert abs(g["E"] - o["E"]) <= 1e-4 * o["E"]


# ------------------------------------------------------------------ tracking
def _compare(g, o):
    rot, tr = oracle.pose_error(g["T_cw"], o["T_cw"])
    rel = abs(g["final_cost"] - o["final_cost"]) / max(o["final_cost"], 1e-12)
    return rot, tr, rel


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 99])
def test_track_single_pair(gpu_lib, seed):
    d, P, trk, ref = _pair_setup(gpu_lib, seed=seed)
    g = trk.track(np.eye(4))
    o = ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    print(f"seed {seed}: rot {rot:.2e} tr {tr:.2e} cost {rel:.2e} iters {g['iterations']}/{o['iterations']}")
    assert g["status"] == o["status"] == 0
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL
    assert abs(g["n_valid_points"] - o["n_valid_points"]) <= 2


# one workgroup; cooperative chunks of one thread per point; cooperative chunks
# of two threads per point
LAUNCHES = [(1, 256), (2, 64), (2, 128), (2, 256), (3, 64), (3, 128)]


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("seed", [7, 42])
def test_track_launch_configs(gpu_lib, seed, launch):
    d, P, trk, ref = _pair_setup(gpu_lib, seed=seed, n=1500, launch=launch)
    g = trk.track(np.eye(4))
    o = ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    assert g["status"] == o["status"] == 0
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


@pytest.mark.parametrize("launch", LAUNCHES)
def test_identity_on_identical_frames(gpu_lib, launch):
    dpt = gpu_lib
    d, P, trk, ref = _pair_setup(dpt, launch=launch)
    trk.build_pyramid(dpt.SLOT_CUR, d["ref"])
    g = trk.track(np.eye(4))
    np.testing.assert_array_equal(g["T_cw"], np.eye(4))
    assert g["final_cost"] == 0.0 and g["iterations"] == 3 and g["status"] == 0


@pytest.mark.parametrize("launch", LAUNCHES)
def test_deterministic(gpu_lib, launch):
    d, P, trk, ref = _pair_setup(gpu_lib, seed=4, launch=launch)
    a, b = trk.track(np.eye(4)), trk.track(np.eye(4))
    np.testing.assert_array_equal(a["T_cw"], b["T_cw"])
    assert a["final_cost"] == b["final_cost"] and a["iterations"] == b["iterations"]


@pytest.mark.parametrize("launch", LAUNCHES)
def test_failure_statuses(gpu_lib, launch):
    dpt = gpu_lib
    d, P, trk, ref = _pair_setup(dpt, seed=4, launch=launch)
    behind = np.eye(4)
    behind[2, 3] = -10.0
    assert trk.track(behind)["status"] == dpt.TRACK_TOO_FEW_POINTS
    flat = np.full_like(d["ref"], 100)
    trk.build_pyramid(dpt.SLOT_REF, flat)
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, flat)
    assert trk.track(np.eye(4))["status"] == dpt.TRACK_NOT_PD
    d, P, trk1, ref1 = _pair_setup(dpt, seed=4, max_iters=1, launch=launch)
    g = trk1.track(np.eye(4))
    o = ref1.track(d["cur"], np.eye(4))
    assert g["status"] == o["status"] == dpt.TRACK_MAX_ITERS
    # empty map
    trk1.set_reference_points(np.zeros((0, 3), np.float32), d["T_rw"])
    assert trk1.track(np.eye(4))["status"] == dpt.TRACK_TOO_FEW_POINTS


@pytest.mark.parametrize("launch", [(1, 256), (2, 256)])
@pytest.mark.parametrize("patch", [3, 7, 11])
def test_track_square_patches(gpu_lib, patch, launch):
    """Paper-shaped p x p patches (and a 3x3 one, K = 9, not a multiple of the
    four lanes per point) through the generic-K paths: one workgroup, and the
    cooperative variant with four lanes per point."""
    d, P, trk, ref = _pair_setup(gpu_lib, seed=6, n=300, pattern=synth.square_pattern(patch), launch=launch)
    g = trk.track(np.eye(4))
    o = ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    assert g["status"] == o["status"] == 0
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


@pytest.mark.parametrize("launch", [(1, 256), (2, 256), (3, 128)])
def test_sequence_window_full_size(gpu_lib, launch):
    """752x480, 2000 points, 4 levels, sigma=2 noise: one keyframe window with the
    constant-velocity start, every frame compared with the oracle."""
    dpt = gpu_lib
    cam = synth.CAM_752
    trk, prm = _tracker(dpt, cam, 2000, levels=4)
    trk.set_launch_config(*launch)
    frames = list(synth.sequence_frames(n_frames=11, start=100))
    k0, img0, depth0, T0 = frames[0]
    trk.build_pyramid(dpt.SLOT_REF, img0)
    idx = trk.select_points(2000, 8)
    np.testing.assert_array_equal(idx, oracle.select_points(img0, 2000, 8))
    P = synth.backproject(cam, depth0, idx, T0)
    trk.set_reference_points(P, T0)
    ref = oracle.Reference(cam, _oparams(prm), img0, P, T0)
    prev2, prev1 = None, T0
    for k, img, _, Tgt in frames[1:10]:
        init = prev1 if prev2 is None else prev1 @ np.linalg.inv(prev2) @ prev1
        trk.build_pyramid(dpt.SLOT_CUR, img)
        g = trk.track(init)
        o = ref.track(img, init)
        rot, tr, rel = _compare(g, o)
        assert g["status"] == o["status"] == 0, (k, g["status"], o["status"])
        assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL, (k, rot, tr, rel)
        prev2, prev1 = prev1, o["T_cw"]


# ------------------------------------------------------------------ mixed precision


@pytest.mark.parametrize("seed", [0, 3, 21, 77])
@pytest.mark.parametrize("mode,chunk", [(2, 64), (2, 256), (3, 128)])
def test_mixed_precision_pair(gpu_lib, seed, mode, chunk):
    dpt = gpu_lib
    d, P, trk, ref = _pair_setup(dpt, seed=seed, n=1500, precision=dpt.PREC_MIXED, launch=(mode, chunk))
    g = trk.track(np.eye(4))
    o = ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    print(f"mixed seed {seed} mode {mode} chunk {chunk}: rot {rot:.2e} rad, trans {tr:.2e} m, cost {rel:.2e}")
    assert g["status"] == o["status"] == 0
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


def test_mixed_precision_identity(gpu_lib):
    dpt = gpu_lib
    d, P, trk, ref = _pair_setup(dpt, precision=dpt.PREC_MIXED, launch=(2, 256))
    trk.build_pyramid(dpt.SLOT_CUR, d["ref"])
    g = trk.track(np.eye(4))
    rot, tr = oracle.pose_error(g["T_cw"], np.eye(4))
    assert rot < 1e-6 and tr < 1e-6 and g["status"] == 0


def test_mixed_precision_stress_16k(gpu_lib):
    """1280x720, 16000 points, 4 levels: accumulation stress of the mixed variant."""
    dpt = gpu_lib
    cam = synth.CAM_1280
    d, P, trk, ref = _pair_setup(dpt, seed=5, n=16000, levels=4, cam=cam, precision=dpt.PREC_MIXED,
                                 launch=(2, 256))
    g = trk.track(np.eye(4))
    o = ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    print(f"mixed 16k: rot {rot:.2e} rad, trans {tr:.2e} m, cost {rel:.2e}")
    assert g["status"] == o["status"] == 0
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL
    trk32, _ = _tracker(dpt, cam, 16000, levels=4)
    trk32.set_launch_config(2, 256)
    trk32.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk32.set_reference_points(P, d["T_rw"])
    trk32.build_pyramid(dpt.SLOT_CUR, d["cur"])
    g32 = trk32.track(np.eye(4))
    rot32, tr32, _ = _compare(g32, o)
    print(f"fp32 16k: rot {rot32:.2e} rad, trans {tr32:.2e} m")
    assert rot32 < ROT_TOL and tr32 < TR_TOL
