"""Learned start pose for the tracker: training-set generation, training and
evaluation of the BF16 CNN (``Cnn``) against the constant-velocity prior.

Training pairs: seeded 3-plane scenes rendered on the GPU at 752 x 480
(fx = fy = 458, cx = 367, cy = 248); a reference view near the scene origin and
current views displaced from it by rotations up to 5 deg (axis uniform) and
translations up to 10 cm.  The label of a pair is the pose the tracker itself
converges to when started from the true pose (4 levels, 2000 map points), as
the reference-to-current twist divided by (5 deg, 0.1 m).  The network input
is the pair's coarsest pyramid level (94 x 60) taken from the tracker's own
pyramids, so training and use see identical inputs.
"""
from __future__ import annotations

import time

import numpy as np

import synth

from . import SLOT_CUR, SLOT_REF, BatchTracker, Cnn, CNN_TWIST_SCALE, make_params

CAM = synth.CAM_752
LEVELS, N_POINTS = 4, 2000


def twist_log(T: np.ndarray) -> np.ndarray:
    """(omega, v) of a rigid transform (rotation angle below pi)."""
    from scipy.spatial.transform import Rotation

    w = Rotation.from_matrix(T[:3, :3]).as_rotvec()
    th = np.linalg.norm(w)
    W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-6:
        Vinv = np.eye(3) - 0.5 * W + W @ W / 12.0
    else:
        Vinv = np.eye(3) - 0.5 * W + (1 - th * np.sin(th) / (2 * (1 - np.cos(th)))) / th ** 2 * (W @ W)
    return np.concatenate([w, Vinv @ T[:3, 3]])


def _reference_pose(rng) -> np.ndarray:
    """A reference view near the scene origin: up to 0.3 m and 8 deg from it."""
    return synth.random_perturbation(rng, 8.0, 0.3)


def make_dataset(n_refs: int, per_ref: int, seed: int, streams: int = 128, max_deg: float = 5.0,
                 max_m: float = 0.10, log=print):
    """Returns (pairs uint8 CUDA tensor [n, 2, 60, 94], targets float32 [n, 6],
    stats).  n = n_refs * per_ref; scene of reference r has seed `seed + r`."""
    import torch

    n = n_refs * per_ref
    pairs = torch.empty((n, 2, 60, 94), dtype=torch.uint8, device="cuda")
    targets = np.empty((n, 6), np.float32)
    prm = make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5)
    S = min(streams, n_refs)
    bt = BatchTracker([CAM] * S, prm, [N_POINTS] * S)
    imgs = torch.empty((S, 1 + per_ref, CAM.height, CAM.width), dtype=torch.uint8, device="cuda")
    depth = torch.empty((S, CAM.height, CAM.width), dtype=torch.float32, device="cuda")
    ref_lv = torch.empty((S, 60, 94), dtype=torch.uint8, device="cuda")
    cur_lv = torch.empty((S, 60, 94), dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    fails, k = 0, 0
    for g0 in range(0, n_refs, S):
        cnt = min(S, n_refs - g0)
        T_ref, T_cur = [], []
        for s in range(S):
            r = g0 + min(s, cnt - 1)  # pad a short last group by repeating its last reference
            rng = np.random.default_rng([seed, r])
            Tr = _reference_pose(rng)
            Tc = [synth.random_perturbation(rng, max_deg, max_m) @ Tr for _ in range(per_ref)]
            T_ref.append(Tr)
            T_cur.append(Tc)
            scene = synth.Scene(seed + r)
            views = np.stack([Tr] + Tc)
            dep = torch.empty((1 + per_ref, CAM.height, CAM.width), dtype=torch.float32, device="cuda")
            synth.render_gpu(scene, CAM, views, imgs[s], dep)
            depth[s] = dep[0]
        bt.build_pyramids(SLOT_REF, [imgs[s, 0] for s in range(S)])
        bt.get_level(SLOT_REF, LEVELS - 1, ref_lv)
        for s in range(S):
            idx = bt.select_points(s, N_POINTS, 8)
            d = depth[s].reshape(-1)[torch.from_numpy(idx.astype(np.int64)).cuda()].double().cpu().numpy()
            full = np.zeros(CAM.width * CAM.height)
            full[idx] = d
            bt.set_reference_points(s, synth.backproject(CAM, full.reshape(CAM.height, CAM.width), idx, T_ref[s]),
                                    T_ref[s])
        for c in range(per_ref):
            bt.build_pyramids(SLOT_CUR, [imgs[s, 1 + c] for s in range(S)])
            bt.get_level(SLOT_CUR, LEVELS - 1, cur_lv)
            res = bt.track(np.stack([T_cur[s][c] for s in range(S)]))
            for s in range(cnt):
                T_rel = res[s]["T_cw"] @ np.linalg.inv(T_ref[s])
                fails += res[s]["status"] not in (0, 1)
                targets[k] = twist_log(T_rel) / CNN_TWIST_SCALE
                pairs[k, 0] = ref_lv[s]
                pairs[k, 1] = cur_lv[s]
                k += 1
        if log and (g0 // S) % 10 == 0:
            log(f"dataset: {k}/{n} pairs, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    bt.close()
    return pairs, targets, {"pairs": n, "seconds": time.perf_counter() - t0, "label_failures": int(fails)}


def train(net: Cnn, pairs, targets, epochs: int, batch: int = 256, lr: float = 1e-3, seed: int = 0, log=print,
          time_limit: float | None = None):
    """Adam on mini-batches of shuffled pairs (all on the device).  Returns the
    per-epoch mean losses."""
    import torch

    n = pairs.shape[0]
    tg = torch.from_numpy(np.ascontiguousarray(targets)).cuda()
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        losses = []
        for b0 in range(0, n - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            losses.append(net.train_step(pairs[sel].contiguous(), tg[sel].contiguous(), lr))
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f} ({time.perf_counter() - t0:.1f} s)")
        if time_limit and time.perf_counter() - t0 > time_limit:
            break
    return hist


def evaluate(net: Cnn | None, n_streams: int, n_frames: int, seed: int, jerk_deg: float = 1.5, jerk_m: float = 0.03,
             max_deg: float = 5.0, max_m: float = 0.10):
    """Streams of n_frames views each against one reference per stream.  The
    current pose drifts away from the reference along a smooth random path
    whose offset reaches (max_deg, max_m), plus per-frame jerks.  Each frame is
    tracked from the CNN's proposal (net given) or from the constant-velocity
    prediction of the previous two estimates, and from the true pose (to find
    the tracker's fixed point), every frame enqueued without a host wait.
    Returns iterations, failures (status not OK, or more than 0.1 deg / 2 mm
    from the fixed point) and frames/s."""
    import torch

    prm = make_params(levels=LEVELS, max_iters=10, huber_k=9.0, step_eps=1e-5)
    S = n_streams
    bt = BatchTracker([CAM] * S, prm, [N_POINTS] * S)
    rng = np.random.default_rng(seed)
    poses = []  # [S][n_frames + 1]
    imgs = torch.empty((S, 1 + n_frames, CAM.height, CAM.width), dtype=torch.uint8, device="cuda")
    depth = torch.empty((S, CAM.height, CAM.width), dtype=torch.float32, device="cuda")
    for s in range(S):
        Tr = _reference_pose(np.random.default_rng([seed, s]))
        end = synth.random_perturbation(rng, max_deg, max_m)
        from scipy.spatial.transform import Rotation, Slerp

        key = Rotation.from_matrix(np.stack([np.eye(3), end[:3, :3]]))
        sl = Slerp([0, 1], key)
        seq = [Tr]
        for f in range(1, n_frames + 1):
            a = f / n_frames
            J = synth.random_perturbation(rng, jerk_deg, jerk_m)
            M = synth.pose_matrix(sl([a]).as_matrix()[0], a * end[:3, 3])
            seq.append(J @ M @ Tr)
        poses.append(seq)
        dep = torch.empty((1 + n_frames, CAM.height, CAM.width), dtype=torch.float32, device="cuda")
        synth.render_gpu(synth.Scene(seed * 7919 + s), CAM, np.stack(seq), imgs[s], dep)
        depth[s] = dep[0]
    bt.build_pyramids(SLOT_REF, [imgs[s, 0] for s in range(S)])
    for s in range(S):
        idx = bt.select_points(s, N_POINTS, 8)
        d = depth[s].reshape(-1)[torch.from_numpy(idx.astype(np.int64)).cuda()].double().cpu().numpy()
        full = np.zeros(CAM.width * CAM.height)
        full[idx] = d
        bt.set_reference_points(s, synth.backproject(CAM, full.reshape(CAM.height, CAM.width), idx, poses[s][0]),
                                poses[s][0])

    T0 = np.stack([poses[s][0] for s in range(S)])

    def run(mode):
        """Every frame of every stream enqueued without a host wait: its pyramid,
        then (cnn) the network's proposal and the track from it, (cv) the track
        from the constant-velocity prediction of the two previous estimates, or
        (gt) the track from the true pose; all on the GPU.  The results are
        collected once at the end."""
        bt.set_pose_history_all(T0, T0)  # the first frame predicts the reference pose
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(1, n_frames + 1):
            bt.build_pyramids(SLOT_CUR, [imgs[s, f] for s in range(S)])
            if mode == "gt":
                bt.track_enqueue(np.stack([poses[s][f] for s in range(S)]))
            elif mode == "cnn":
                net.propose(bt)
                bt.track_enqueue(proposed=True)
            else:
                bt.track_enqueue(None)
        res = bt.synchronize(arrays=True)  # (n_frames, S)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        T_out = res["T_cw"].reshape(n_frames, S, 4, 4)
        return res["iterations"].reshape(-1).astype(np.float64), T_out, S * n_frames / el, res["status"]

    its_gt, T_gt, _, _ = run("gt")
    out = {}
    for mode in (["cv", "cnn"] if net is not None else ["cv"]):
        its, T, fps, status = run(mode)
        fail = 0
        for f in range(n_frames):
            for s in range(S):
                E = T[f][s] @ np.linalg.inv(T_gt[f][s])
                ang = np.arccos(np.clip((np.trace(E[:3, :3]) - 1) / 2, -1, 1))
                fail += (status[f, s] != 0) or (np.rad2deg(ang) > 0.1) or (np.linalg.norm(E[:3, 3]) > 2e-3)
        out[mode] = {"iterations_mean": float(its.mean()), "failure_rate": fail / (S * n_frames),
                     "frames_per_s": round(fps, 1)}
    out["gt_start_iterations_mean"] = float(its_gt.mean())
    bt.close()
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal conv / FC weights, zero biases, as the flat FP32 parameter vector."""
    from . import CNN_SHAPES

    rng = np.random.default_rng(seed)
    out = []
    for name, shp in CNN_SHAPES:
        if name.startswith("w"):
            fan_in = shp[1] * shp[2] * shp[3]
            out.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), shp))
        elif name == "fw1":
            out.append(rng.normal(0.0, np.sqrt(2.0 / shp[1]), shp))
        elif name == "fw2":
            out.append(rng.normal(0.0, np.sqrt(1.0 / shp[1]), shp))
        else:
            out.append(np.zeros(shp))
    return np.concatenate([o.reshape(-1) for o in out]).astype(np.float32)


def save_checkpoint(path: str, params: np.ndarray, meta: dict):
    """Flat FP32 parameters (tensor order of CNN_SHAPES) plus a JSON header."""
    import json

    np.save(path + ".npy", np.asarray(params, np.float32))
    with open(path + ".json", "w") as f:
        json.dump(meta, f, indent=1)


def load_checkpoint(path: str) -> np.ndarray:
    return np.load(path + ".npy", allow_pickle=False)


def validation_loss(net: Cnn, pairs, targets, batch: int = 256) -> float:
    errs = []
    for b0 in range(0, pairs.shape[0], batch):
        out = net.forward(pairs[b0:b0 + batch].contiguous())
        errs.append(((out - targets[b0:b0 + batch]) ** 2).reshape(-1))
    return float(np.mean(np.concatenate(errs)))
