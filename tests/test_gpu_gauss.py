"""GPU parity of tracking on the floating-point Gaussian pyramid (Sec. IV-C,
image pyramids) and at the paper's per-point shape (p x p patches, 6 levels),
against the oracle's Gaussian mode on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL, COST_TOL = 1e-4, 1e-4, 1e-3


def _oparams(p, fixed_h=False):
    pat = np.array(p.pattern[:2 * p.n_pattern]).reshape(-1, 2)
    return oracle.make_params(levels=p.levels, max_iters=p.max_iters, huber_k=p.huber_k, step_eps=p.step_eps,
                              min_points=p.min_points, pattern=pat, z_min=p.z_min, fixed_h=fixed_h, gauss=True)


LAUNCHES = [(1, 256), (2, 256)]  # one workgroup; cooperative (64-point chunks, four lanes per point)


def _setup(dpt, seed=0, n=500, levels=3, cam=synth.CAM_640, fixed_h=False, launch=None, **kw):
    d = synth.pair(seed, cam)
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    prm = dpt.make_params(levels=levels, gauss=True, fixed_h=fixed_h, **kw)
    trk = dpt.Tracker(cam, prm, max_points=max(n, 1))
    if launch is not None:
        trk.set_launch_config(*launch)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    ref = oracle.Reference(cam, _oparams(prm, fixed_h), d["ref"], P, d["T_rw"])
    return d, P, trk, ref


@pytest.mark.parametrize("cam,levels", [(synth.CAM_640, 3), (synth.CAM_752, 6),
                                        (synth.Camera(645, 483, 400, 400, 320, 240), 6),
                                        (synth.Camera(1023, 767, 500, 500, 511, 383), 7),
                                        (synth.Camera(130, 70, 100, 100, 65, 35), 1)])
def test_gauss_pyramid_matches_oracle(gpu_lib, cam, levels):
    """FP32 pyramid against the FP64 one: within 2e-4 intensity levels."""
    import torch

    dpt = gpu_lib
    img = np.random.default_rng(cam.width).integers(0, 256, (cam.height, cam.width), dtype=np.uint8)
    trk = dpt.Tracker(cam, dpt.make_params(levels=levels, gauss=True), max_points=10)
    want = oracle.pyramid_gauss(img, levels)
    trk.build_pyramid(dpt.SLOT_CUR, img)
    for l in range(levels):
        got = trk.get_pyramid_f32(dpt.SLOT_CUR, l)
        np.testing.assert_allclose(got, want[l], rtol=0, atol=2e-4)
        # the uint8 box pyramid is still built (point selection reads its level 0)
        np.testing.assert_array_equal(trk.get_pyramid(dpt.SLOT_CUR, l), oracle.pyramid(img, levels)[l])
    pitch = cam.width + 29
    padded = np.zeros((cam.height, pitch), np.uint8)
    padded[:, :cam.width] = img
    trk.build_pyramid(dpt.SLOT_REF, torch.from_numpy(padded).cuda(), pitch=pitch)
    torch.cuda.synchronize()
    for l in range(levels):
        np.testing.assert_allclose(trk.get_pyramid_f32(dpt.SLOT_REF, l), want[l], rtol=0, atol=2e-4)


def test_gauss_precompute_and_normal_equations(gpu_lib):
    d, P, trk, ref = _setup(gpu_lib, seed=3)
    for l in range(3):
        g, o = trk.reference_cache(l), ref.cache(l)
        assert (g["valid"] == o["refvalid"]).mean() > 0.995
        both = g["valid"] & o["refvalid"]
        np.testing.assert_allclose(g["I0"][both], o["I0"][both], atol=2e-3)
        np.testing.assert_allclose(g["gx"][both], o["g"][both][..., 0], atol=2e-3)
        np.testing.assert_allclose(g["gy"][both], o["g"][both][..., 1], atol=2e-3)
    T_rel = oracle.se3_exp(np.array([0.002, -0.001, 0.003, 0.004, 0.002, -0.003]))
    for l in range(3):
        g = trk.normal_equations(l, T_rel)
        o = ref.normal_equations(d["cur"], l, T_rel)
        assert abs(g["npts"] - o["npts"]) <= 1
        if g["npts"] != o["npts"]:
            continue
        np.testing.assert_allclose(g["H"], o["H"], atol=2e-4 * np.abs(o["H"]).max())
        np.testing.assert_allclose(g["b"], o["b"], atol=2e-4 * np.abs(o["b"]).max())
        assert abs(g["E"] - o["E"]) <= 1e-4 * o["E"]


def _compare(g, o):
    rot, tr = oracle.pose_error(g["T_cw"], o["T_cw"])
    rel = abs(g["final_cost"] - o["final_cost"]) / max(o["final_cost"], 1e-12)
    return rot, tr, rel


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("seed", [0, 5, 21, 42])
def test_gauss_track_matches_oracle(gpu_lib, seed, launch):
    d, P, trk, ref = _setup(gpu_lib, seed=seed, n=1500, launch=launch)
    g, o = trk.track(np.eye(4)), ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    print(f"seed {seed}: rot {rot:.2e} tr {tr:.2e} cost {rel:.2e} iters {g['iterations']}/{o['iterations']}")
    assert g["status"] == o["status"] == 0
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("patch,levels,fixed_h", [(7, 6, False), (11, 5, False), (7, 6, True), (11, 5, True)])
def test_gauss_paper_shape(gpu_lib, patch, levels, fixed_h, launch):
    """The paper's per-point shape: 752x480, p x p patches, 6 levels (5 for
    11x11, whose patch leaves too few valid positions in the 23x15 sixth level)."""
    d, P, trk, ref = _setup(gpu_lib, seed=3, n=600, levels=levels, cam=synth.CAM_752,
                            pattern=synth.square_pattern(patch), fixed_h=fixed_h, launch=launch)
    g, o = trk.track(np.eye(4)), ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    print(f"p={patch} fixed_h={fixed_h}: rot {rot:.2e} tr {tr:.2e} cost {rel:.2e} "
          f"iters {g['iterations']}/{o['iterations']} status {g['status']}/{o['status']}")
    assert g["status"] == o["status"]
    assert g["status"] in (0, 1)
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


@pytest.mark.parametrize("launch", LAUNCHES)
def test_gauss_paper_shape_too_few_points_at_coarsest(gpu_lib, launch):
    """A 7x7 patch fits few points into the 23x15 sixth level: with this map
    only 4 are valid there, so both sides stop with TOO_FEW_POINTS."""
    dpt = gpu_lib
    d, P, trk, ref = _setup(dpt, seed=6, n=600, levels=6, cam=synth.CAM_752, pattern=synth.square_pattern(7),
                            launch=launch)
    assert int(trk.reference_cache(5)["valid"].sum()) == int(ref.cache(5)["refvalid"].sum()) == 4
    g, o = trk.track(np.eye(4)), ref.track(d["cur"], np.eye(4))
    assert g["status"] == o["status"] == dpt.TRACK_TOO_FEW_POINTS
    assert g["iterations"] == o["iterations"] == 0


@pytest.mark.parametrize("launch", LAUNCHES)
def test_gauss_identity_and_rejections(gpu_lib, launch):
    dpt = gpu_lib
    d, P, trk, ref = _setup(dpt, seed=4, launch=launch)
    trk.build_pyramid(dpt.SLOT_CUR, d["ref"])
    g = trk.track(np.eye(4))
    np.testing.assert_array_equal(g["T_cw"], np.eye(4))
    assert g["final_cost"] == 0.0 and g["status"] == 0
    with pytest.raises(dpt.DptError):
        dpt.Tracker(synth.CAM_640, dpt.make_params(gauss=True, precision=dpt.PREC_MIXED), max_points=10)


def test_gauss_batch_equals_plain(gpu_lib):
    import torch

    dpt = gpu_lib
    cam, n = synth.CAM_640, 800
    pairs = [synth.pair(s, cam) for s in (1, 2, 3)]
    prm = dpt.make_params(levels=3, gauss=True)
    bt = dpt.BatchTracker([cam] * 3, prm, [n] * 3)
    bt.build_pyramids(dpt.SLOT_REF, [torch.from_numpy(p["ref"]).cuda() for p in pairs])
    Ps = []
    for s, p in enumerate(pairs):
        idx = oracle.select_points(p["ref"], n, 8)
        Ps.append(synth.backproject(cam, p["depth"], idx, p["T_rw"]))
        bt.set_reference_points(s, Ps[-1], p["T_rw"])
    bt.build_pyramids(dpt.SLOT_CUR, [torch.from_numpy(p["cur"]).cuda() for p in pairs])
    res = bt.track(np.stack([np.eye(4)] * 3))
    for s, p in enumerate(pairs):
        t = dpt.Tracker(cam, prm, max_points=n)
        t.build_pyramid(dpt.SLOT_REF, p["ref"])
        t.set_reference_points(Ps[s], p["T_rw"])
        t.build_pyramid(dpt.SLOT_CUR, p["cur"])
        r = t.track(np.eye(4))
        np.testing.assert_array_equal(res[s]["T_cw"], r["T_cw"])
        assert res[s]["iterations"] == r["iterations"] and r["status"] == 0
