"""Training-set pipeline of the learned initialiser on the GPU: the GPU scene
renderer against the CPU renderer, tracker labels against the true motion,
and the network's proposals feeding the tracker."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_gpu_renderer_matches_cpu(gpu_lib):
    import torch

    scene = synth.Scene(42)
    poses = [np.eye(4), synth.random_perturbation(np.random.default_rng(3), 5.0, 0.1)]
    imgs = torch.empty((2, 480, 752), dtype=torch.uint8, device="cuda")
    dep = torch.empty((2, 480, 752), dtype=torch.float32, device="cuda")
    synth.render_gpu(scene, synth.CAM_752, np.stack(poses), imgs, dep)
    for v, T in enumerate(poses):
        cpu, d = scene.render(synth.CAM_752, T)
        g = imgs[v].cpu().numpy().astype(int)
        diff = np.abs(g - cpu.astype(int))
        assert (diff == 0).mean() > 0.999 and diff.max() <= 1
        np.testing.assert_allclose(dep[v].cpu().numpy(), d, rtol=1e-6)


def test_dataset_labels_follow_true_motion(gpu_lib):
    from paper_2607_16897_amd import initialiser as ini
    from paper_2607_16897_amd import CNN_TWIST_SCALE

    pairs, targets, st = ini.make_dataset(4, 3, seed=123, streams=4, log=None)
    assert tuple(pairs.shape) == (12, 2, 60, 94) and st["label_failures"] == 0
    for r in range(4):  # one group of 4 streams: pair k = c * 4 + r
        rng = np.random.default_rng([123, r])
        Tr = ini._reference_pose(rng)
        for c in range(3):
            Tc = synth.random_perturbation(rng, 5.0, 0.10) @ Tr
            true = ini.twist_log(Tc @ np.linalg.inv(Tr)) / CNN_TWIST_SCALE
            # the tracker's fixed point lies within ~1 mm / 0.05 deg of the rendered motion
            k = c * 4 + r
            assert np.abs(targets[k] - true).max() < 0.02, (r, c, targets[k], true)


def test_network_proposals_feed_the_tracker(gpu_lib):
    import torch

    dpt = gpu_lib
    from paper_2607_16897_amd import initialiser as ini

    net = dpt.Cnn(max_batch=8)
    net.set_params(ini.init_params(1))
    res = ini.evaluate(net, 4, 3, seed=9)
    assert set(res) >= {"cv", "cnn", "gt_start_iterations_mean"}
    assert 0.0 <= res["cnn"]["failure_rate"] <= 1.0


def test_trained_network_beats_constant_velocity(gpu_lib):
    """The committed network (trained on 200k tracker-labelled pairs) against the
    constant-velocity prior on held-out scenes: fewer Gauss-Newton iterations and
    no more failures."""
    dpt = gpu_lib
    from paper_2607_16897_amd import initialiser as ini

    path = os.path.join(os.path.dirname(dpt.__file__), "weights", "initialiser")
    net = dpt.Cnn(max_batch=32)
    net.set_params(ini.load_checkpoint(path))
    res = ini.evaluate(net, 16, 20, seed=424242)
    print(res)
    assert res["cnn"]["iterations_mean"] < res["cv"]["iterations_mean"]
    assert res["cnn"]["failure_rate"] <= res["cv"]["failure_rate"]


def test_device_proposal_matches_host_prediction(gpu_lib):
    """The proposal kept on the device (no host round trip) starts the same
    track as the host-side prediction given as the start pose."""
    import torch

    dpt = gpu_lib
    from paper_2607_16897_amd import initialiser as ini

    S = 4
    net = dpt.Cnn(max_batch=S)
    net.set_params(ini.init_params(5))
    prm = dpt.make_params(levels=4)
    bt = dpt.BatchTracker([synth.CAM_752] * S, prm, [500] * S)
    with pytest.raises(dpt.DptError):  # no proposal yet
        bt.track_enqueue(proposed=True)
    rng = np.random.default_rng(77)
    imgs = torch.empty((S, 2, 480, 752), dtype=torch.uint8, device="cuda")
    dep = torch.empty((S, 2, 480, 752), dtype=torch.float32, device="cuda")
    refs = []
    for s in range(S):
        Tr = np.eye(4)
        Tc = synth.random_perturbation(rng, 3.0, 0.05)
        synth.render_gpu(synth.Scene(500 + s), synth.CAM_752, np.stack([Tr, Tc]), imgs[s], dep[s])
        refs.append(Tr)
    bt.build_pyramids(dpt.SLOT_REF, [imgs[s, 0] for s in range(S)])
    for s in range(S):
        idx = bt.select_points(s, 500, 8)
        d = dep[s, 0].reshape(-1)[torch.from_numpy(idx.astype(np.int64)).cuda()].double().cpu().numpy()
        full = np.zeros(480 * 752)
        full[idx] = d
        bt.set_reference_points(s, synth.backproject(synth.CAM_752, full.reshape(480, 752), idx, refs[s]), refs[s])
    bt.build_pyramids(dpt.SLOT_CUR, [imgs[s, 1] for s in range(S)])
    host = bt.track(net.predict(bt))
    net.propose(bt)
    bt.track_enqueue(proposed=True)
    dev = bt.synchronize()[0]
    for h, d in zip(host, dev):
        rot, tr = _pose_err(h["T_cw"], d["T_cw"])
        assert rot < 1e-5 and tr < 1e-5 and h["status"] == d["status"]
    bt.close()
    net.close()


def _pose_err(A, B):
    E = np.asarray(A) @ np.linalg.inv(np.asarray(B))
    ang = float(np.arccos(np.clip((np.trace(E[:3, :3]) - 1) / 2, -1, 1)))
    return ang, float(np.linalg.norm(E[:3, 3]))


def test_level_and_pair_inputs_agree(gpu_lib):
    """The proposal, which reads the coarsest levels through per-stream
    pointers and keeps its activations on chip, gives bitwise the layer-4
    activations and head outputs of the forward pass over the same levels
    handed over as planar pairs."""
    import torch

    dpt = gpu_lib
    from paper_2607_16897_amd import initialiser as ini

    S = 5
    net = dpt.Cnn(max_batch=S)
    net.set_params(ini.init_params(7))
    bt = dpt.BatchTracker([synth.CAM_752] * S, dpt.make_params(levels=4), [400] * S)
    rng = np.random.default_rng(78)
    imgs = torch.empty((S, 2, 480, 752), dtype=torch.uint8, device="cuda")
    dep = torch.empty((S, 2, 480, 752), dtype=torch.float32, device="cuda")
    for s in range(S):
        synth.render_gpu(synth.Scene(600 + s), synth.CAM_752,
                         np.stack([np.eye(4), synth.random_perturbation(rng, 4.0, 0.08)]), imgs[s], dep[s])
    bt.build_pyramids(dpt.SLOT_REF, [imgs[s, 0] for s in range(S)])
    for s in range(S):
        idx = bt.select_points(s, 400, 8)
        d = dep[s, 0].reshape(-1)[torch.from_numpy(idx.astype(np.int64)).cuda()].double().cpu().numpy()
        full = np.zeros(480 * 752)
        full[idx] = d
        bt.set_reference_points(s, synth.backproject(synth.CAM_752, full.reshape(480, 752), idx, np.eye(4)), np.eye(4))
    bt.build_pyramids(dpt.SLOT_CUR, [imgs[s, 1] for s in range(S)])
    net.propose(bt)
    fused, out = net.activation(4, S), net.activation(5, S)
    pairs = np.ascontiguousarray(np.stack([bt.get_level(dpt.SLOT_REF, 3), bt.get_level(dpt.SLOT_CUR, 3)], axis=1))
    np.testing.assert_array_equal(out, net.forward(pairs))
    np.testing.assert_array_equal(fused, net.activation(4, S))
    assert np.count_nonzero(fused) > fused.size // 10  # a live network, not all-zero activations
    bt.close()
    net.close()
