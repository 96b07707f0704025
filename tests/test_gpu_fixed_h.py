"""GPU parity of the fixed-H mode (the paper's own inverse-compositional track,
Sec. IV-B and the precompute / track stages of Sec. IV-C): per level a constant
H reduced once per reference, b reduced per iteration, no robust weights.
Compared with the oracle run with fixed_h on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROT_TOL, TR_TOL, COST_TOL = 1e-4, 1e-4, 1e-3
LAUNCHES = [(1, 256), (2, 64), (2, 256), (3, 128)]  # one workgroup; cooperative chunks; two threads per point


def _oparams(p):
    pat = np.array(p.pattern[:2 * p.n_pattern]).reshape(-1, 2)
    return oracle.make_params(levels=p.levels, max_iters=p.max_iters, huber_k=p.huber_k, step_eps=p.step_eps,
                              min_points=p.min_points, pattern=pat, z_min=p.z_min, fixed_h=True)


def _setup(dpt, seed=0, n=500, levels=3, cam=synth.CAM_640, launch=None, **kw):
    d = synth.pair(seed, cam)
    idx = oracle.select_points(d["ref"], n, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    prm = dpt.make_params(levels=levels, fixed_h=True, **kw)
    trk = dpt.Tracker(cam, prm, max_points=max(n, 1))
    if launch is not None:
        trk.set_launch_config(*launch)
    trk.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk.set_reference_points(P, d["T_rw"])
    trk.build_pyramid(dpt.SLOT_CUR, d["cur"])
    ref = oracle.Reference(cam, _oparams(prm), d["ref"], P, d["T_rw"])
    return d, P, trk, ref


def _compare(g, o):
    rot, tr = oracle.pose_error(g["T_cw"], o["T_cw"])
    rel = abs(g["final_cost"] - o["final_cost"]) / max(o["final_cost"], 1e-12)
    return rot, tr, rel


@pytest.mark.parametrize("n", [1, 300, 1500])
def test_fixed_hessian_matches_oracle(gpu_lib, n):
    """H of every level: the FP64 sum of FP32 per-point terms against the
    oracle's FP64 sum, elementwise relative to the largest entry."""
    d, P, trk, ref = _setup(gpu_lib, seed=2, n=n)
    for l in range(3):
        H, bad = trk.fixed_hessian(l)
        Ho = ref.fixed_h(l)
        np.testing.assert_allclose(H, H.T, rtol=0, atol=0)
        scale = max(np.abs(Ho).max(), 1e-30)
        np.testing.assert_allclose(H, Ho, rtol=0, atol=2e-5 * scale)
        # one point spans at most rank 2 (its warp Jacobian has two rows)
        assert bad == (n == 1)


def test_normal_equations_fixed_mode(gpu_lib):
    d, P, trk, ref = _setup(gpu_lib, seed=3)
    T_rel = oracle.se3_exp(np.array([0.002, -0.001, 0.003, 0.004, 0.002, -0.003]))
    for l in range(3):
        g = trk.normal_equations(l, T_rel)
        o = ref.normal_equations(d["cur"], l, T_rel)
        np.testing.assert_allclose(g["H"], ref.fixed_h(l), atol=2e-5 * np.abs(o["H"]).max())
        np.testing.assert_allclose(o["H"], ref.fixed_h(l), rtol=0, atol=0)
        assert abs(g["npts"] - o["npts"]) <= 1
        if g["npts"] != o["npts"]:
            continue
        assert g["n"] == o["n"]
        np.testing.assert_allclose(g["b"], o["b"], atol=2e-4 * np.abs(o["b"]).max())
        assert abs(g["E"] - o["E"]) <= 1e-4 * o["E"]


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("seed", [0, 5, 13, 42])
def test_fixed_h_track_matches_oracle(gpu_lib, seed, launch):
    d, P, trk, ref = _setup(gpu_lib, seed=seed, n=1500, launch=launch)
    g = trk.track(np.eye(4))
    o = ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    print(f"seed {seed} {launch}: rot {rot:.2e} tr {tr:.2e} cost {rel:.2e} iters {g['iterations']}/{o['iterations']}")
    assert g["status"] == o["status"]
    assert g["status"] in (0, 1)
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


def test_fixed_h_ignores_huber_k(gpu_lib):
    """No weights in the fixed-H mode: the Huber threshold changes nothing."""
    d, P, trk, _ = _setup(gpu_lib, seed=8, huber_k=9.0)
    _, _, trk2, _ = _setup(gpu_lib, seed=8, huber_k=2.0)
    a, b = trk.track(np.eye(4)), trk2.track(np.eye(4))
    np.testing.assert_array_equal(a["T_cw"], b["T_cw"])
    assert a["final_cost"] == b["final_cost"]


@pytest.mark.parametrize("launch", LAUNCHES)
def test_fixed_h_identity_and_statuses(gpu_lib, launch):
    dpt = gpu_lib
    d, P, trk, ref = _setup(dpt, seed=4, launch=launch)
    trk.build_pyramid(dpt.SLOT_CUR, d["ref"])
    g = trk.track(np.eye(4))
    np.testing.assert_array_equal(g["T_cw"], np.eye(4))
    assert g["final_cost"] == 0.0 and g["iterations"] == 3 and g["status"] == 0
    # a single point: H of rank 2, not positive definite at the first level
    trk1 = dpt.Tracker(synth.CAM_640, dpt.make_params(levels=3, fixed_h=True, min_points=0), max_points=4)
    trk1.set_launch_config(*launch)
    trk1.build_pyramid(dpt.SLOT_REF, d["ref"])
    trk1.set_reference_points(P[:1], d["T_rw"])
    trk1.build_pyramid(dpt.SLOT_CUR, d["cur"])
    o1 = oracle.Reference(synth.CAM_640, _oparams(trk1.params), d["ref"], P[:1], d["T_rw"]).track(d["cur"], np.eye(4))
    g1 = trk1.track(np.eye(4))
    assert g1["status"] == o1["status"] == dpt.TRACK_NOT_PD
    # the camera moved behind the map: too few points
    behind = np.eye(4)
    behind[2, 3] = -10.0
    assert trk.track(behind)["status"] == dpt.TRACK_TOO_FEW_POINTS


@pytest.mark.parametrize("launch", [(1, 256), (2, 256)])
def test_fixed_h_square_patch(gpu_lib, launch):
    """7x7 patches (49 samples per point) through the generic-K paths."""
    d, P, trk, ref = _setup(gpu_lib, seed=6, n=300, pattern=synth.square_pattern(7), launch=launch)
    g = trk.track(np.eye(4))
    o = ref.track(d["cur"], np.eye(4))
    rot, tr, rel = _compare(g, o)
    assert g["status"] == o["status"]
    assert rot < ROT_TOL and tr < TR_TOL and rel < COST_TOL


def test_fixed_h_batch_equals_plain(gpu_lib):
    """Batched references (one launch sequence for every stream's H) and the
    batched track give the plain context's poses."""
    import torch

    dpt = gpu_lib
    cam, n = synth.CAM_752, 1500
    traj, scene = synth.Trajectory(2607), synth.Scene(2607)
    frames = []
    for s in range(3):
        k = 10 * s + 20
        T_rw = traj.T_cw(k)
        img, depth = scene.render(cam, T_rw, synth.pixel_noise(2607, k, cam, 2.0), want_depth=True)
        cur, _ = scene.render(cam, traj.T_cw(k + 3), synth.pixel_noise(2607, k + 3, cam, 2.0), want_depth=False)
        frames.append((img, depth.astype(np.float32), cur, T_rw, traj.T_cw(k + 2)))
    prm = dpt.make_params(levels=4, fixed_h=True)
    bt = dpt.BatchTracker([cam] * 3, prm, [n] * 3)
    bt.build_pyramids(dpt.SLOT_REF, [torch.from_numpy(f[0]).cuda() for f in frames])
    bt.set_reference_from_depth_all([n] * 3, [torch.from_numpy(f[1]).cuda() for f in frames],
                                    np.stack([f[3] for f in frames]))
    bt.build_pyramids(dpt.SLOT_CUR, [torch.from_numpy(f[2]).cuda() for f in frames])
    res = bt.track(np.stack([f[4] for f in frames]))
    for s, f in enumerate(frames):
        t = dpt.Tracker(cam, prm, max_points=n)
        t.build_pyramid(dpt.SLOT_REF, f[0])
        t.set_reference_from_depth(n, f[1], f[3])
        t.build_pyramid(dpt.SLOT_CUR, f[2])
        r = t.track(f[4])
        rot, tr = oracle.pose_error(res[s]["T_cw"], r["T_cw"])
        assert rot < 1e-5 and tr < 1e-5
        assert res[s]["iterations"] == r["iterations"]
        assert r["status"] in (0, 1)
