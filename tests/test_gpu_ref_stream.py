"""Reference updates on a second stream (dpt_set_reference_stream): the
keyframe's reference pyramid, selection, back-projection and IC precompute
(Sec. IV-C) run on their own stream into the reference bank the tracks in
flight do not read.  Every track must return bitwise what the single-stream
context returns on the same enqueue sequence (several keyframe windows
enqueued back to back without host waits, window and frame-by-frame forms,
FP32, mixed precision, fixed H, two threads per point), the test hooks must
read the committed reference, and an update without a new reference pyramid
must be refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FIELDS = ("T_cw", "final_cost", "iterations", "iters_per_level", "n_valid_points", "status", "samples")
N = 2000


def _windows(n_win, cam=synth.CAM_752, seed=2607):
    """Keyframe windows of the headline sequence: keyframe image and depth,
    the pose before the keyframe and the keyframe's pose, nine tween frames."""
    import torch

    traj, scene = synth.Trajectory(seed), synth.Scene(seed)
    out = []
    for w in range(n_win):
        k0 = 40 + 10 * w
        img0, depth = scene.render(cam, traj.T_cw(k0), synth.pixel_noise(seed, k0, cam, 2.0), want_depth=True)
        frames = np.stack([scene.render(cam, traj.T_cw(k0 + j), synth.pixel_noise(seed, k0 + j, cam, 2.0),
                                        want_depth=False)[0] for j in range(1, 10)])
        out.append(dict(img0=torch.from_numpy(img0).cuda(), depth=torch.from_numpy(depth.astype(np.float32)).cuda(),
                        frames=torch.from_numpy(frames).cuda(), T0=traj.T_cw(k0), T_prev=traj.T_cw(k0 - 1)))
    torch.cuda.synchronize()
    return out


def _run(dpt, wins, prm, launch, window, ref_stream):
    trk = dpt.Tracker(synth.CAM_752, prm, max_points=N)
    trk.set_launch_config(*launch)
    if ref_stream:
        trk.set_reference_stream(ref_stream)
    for w in wins:  # everything enqueued, one synchronisation at the end
        trk.build_pyramid(dpt.SLOT_REF, w["img0"])
        trk.set_reference_from_depth(N, w["depth"], w["T0"])
        trk.set_pose_history(w["T_prev"], w["T0"])
        if window:
            trk.track_window_enqueue(w["frames"])
        else:
            for j in range(9):
                trk.build_pyramid(dpt.SLOT_CUR, w["frames"][j])
                trk.track_enqueue(None)
    res = trk.synchronize()
    cache = trk.reference_cache(0)
    trk.close()
    return res, cache


def _assert_same(a, b):
    assert len(a) == len(b)
    for f, (x, y) in enumerate(zip(a, b)):
        for k in FIELDS:
            np.testing.assert_array_equal(np.asarray(x[k]), np.asarray(y[k]), err_msg=f"frame {f} field {k}")


@pytest.fixture(scope="module")
def wins(gpu_lib):
    return _windows(5)


@pytest.fixture(scope="module")
def rstream(gpu_lib):
    """One library-made stream for every case (a process that uses more streams
    than the GPU has hardware queues runs later kernels slower)."""
    s = gpu_lib.Stream()
    yield s
    s.close()


@pytest.mark.parametrize("variant,launch,window", [
    ("fp32", (3, 128), True), ("fp32", (2, 256), True), ("fp32", (3, 128), False),
    ("mixed", (3, 128), True), ("fixed_h", (2, 256), True), ("fixed_h", (3, 128), False)])
def test_reference_stream_equals_single_stream(gpu_lib, wins, rstream, variant, launch, window):
    dpt = gpu_lib
    kw = dict(levels=4)
    if variant == "mixed":
        kw["precision"] = dpt.PREC_MIXED
    elif variant == "fixed_h":
        kw["fixed_h"] = True
    prm = dpt.make_params(**kw)
    print(f"reference stream {variant} launch {launch} window {window}", flush=True)
    base, cache0 = _run(dpt, wins, prm, launch, window, None)
    piped, cache1 = _run(dpt, wins, prm, launch, window, rstream)
    _assert_same(base, piped)
    assert all(r["status"] == 0 for r in base)
    for k in ("valid", "I0", "gx", "gy", "x0"):  # the hook reads the last committed reference
        np.testing.assert_array_equal(cache0[k], cache1[k], err_msg=k)


def test_reference_stream_needs_a_new_reference_pyramid(gpu_lib, wins, rstream):
    dpt = gpu_lib
    trk = dpt.Tracker(synth.CAM_752, dpt.make_params(levels=4), max_points=N)
    trk.set_reference_stream(rstream)
    w = wins[0]
    trk.build_pyramid(dpt.SLOT_REF, w["img0"])
    trk.set_reference_from_depth(N, w["depth"], w["T0"])
    with pytest.raises(dpt.DptError):  # a second update on the same pyramid
        trk.set_reference_from_depth(N, w["depth"], w["T0"])
    # back to one stream: the same update is accepted again
    trk.set_reference_stream(None)
    trk.set_reference_from_depth(N, w["depth"], w["T0"])
    trk.set_pose_history(w["T_prev"], w["T0"])
    trk.track_window_enqueue(w["frames"])
    assert all(r["status"] == 0 for r in trk.synchronize())
    trk.close()


S = 4  # streams of the batch cases


@pytest.fixture(scope="module")
def bwins(gpu_lib):
    """Four keyframe windows of each of S streams, each stream its own scene and trajectory."""
    return [_windows(4, seed=2607 + 13 * s) for s in range(S)]


def _run_batch(dpt, bw, prm, launch, window, ref_stream, cnn=None):
    """Every window of every stream enqueued back to back; odd windows set the
    references stream by stream, even ones in one launch sequence."""
    bt = dpt.BatchTracker([synth.CAM_752] * S, prm, [N] * S)
    bt.set_launch_config(*launch)
    if ref_stream:
        bt.set_reference_stream(ref_stream)
    for w in range(len(bw[0])):
        ws = [bw[s][w] for s in range(S)]
        bt.build_pyramids(dpt.SLOT_REF, [x["img0"] for x in ws])
        if w % 2 == 0:
            bt.set_reference_from_depth_all(N, [x["depth"] for x in ws], np.stack([x["T0"] for x in ws]))
        else:
            for s, x in enumerate(ws):
                bt.set_reference_from_depth(s, N, x["depth"], x["T0"])
        bt.set_pose_history_all(np.stack([x["T_prev"] for x in ws]), np.stack([x["T0"] for x in ws]))
        if window:
            bt.track_window_enqueue([x["frames"] for x in ws])
            continue
        for j in range(9):
            bt.build_pyramids(dpt.SLOT_CUR, [x["frames"][j] for x in ws])
            if cnn is not None:
                cnn.propose(bt)
                bt.track_enqueue(proposed=True)
            else:
                bt.track_enqueue(None)
    res = bt.synchronize()
    ref_level = bt.get_level(dpt.SLOT_REF, 1)
    bt.close()
    return res, ref_level


def _assert_same_batch(a, b):
    assert len(a) == len(b)
    for f, (x, y) in enumerate(zip(a, b)):
        assert len(x) == len(y) == S
        for s, (p, q) in enumerate(zip(x, y)):
            for k in FIELDS:
                np.testing.assert_array_equal(np.asarray(p[k]), np.asarray(q[k]), err_msg=f"frame {f} stream {s} field {k}")


@pytest.mark.parametrize("variant,launch,window", [
    ("fp32", (3, 128), True), ("fp32", (2, 256), False), ("mixed", (3, 128), True), ("fixed_h", (3, 128), False)])
def test_batch_reference_stream_equals_single_stream(gpu_lib, bwins, rstream, variant, launch, window):
    dpt = gpu_lib
    kw = dict(levels=4)
    if variant == "mixed":
        kw["precision"] = dpt.PREC_MIXED
    elif variant == "fixed_h":
        kw["fixed_h"] = True
    prm = dpt.make_params(**kw)
    print(f"batch reference stream {variant} launch {launch} window {window}", flush=True)
    base, lv0 = _run_batch(dpt, bwins, prm, launch, window, None)
    piped, lv1 = _run_batch(dpt, bwins, prm, launch, window, rstream)
    _assert_same_batch(base, piped)
    assert all(r["status"] == 0 for f in base for r in f)
    np.testing.assert_array_equal(lv0, lv1)  # the last reference pyramid, read after its update


def test_learned_start_with_reference_stream(gpu_lib, bwins, rstream):
    """Proposals read the coarsest reference level of the committed bank: the
    proposed starts, and so the tracks, equal the single-stream ones."""
    dpt = gpu_lib
    from paper_2607_16897_amd import initialiser as ini

    net = dpt.Cnn(max_batch=S)
    net.set_params(ini.init_params(5))
    prm = dpt.make_params(levels=4)
    print("batch reference stream with learned starts", flush=True)
    base, _ = _run_batch(dpt, bwins, prm, (3, 128), False, None, cnn=net)
    piped, _ = _run_batch(dpt, bwins, prm, (3, 128), False, rstream, cnn=net)
    net.close()
    _assert_same_batch(base, piped)


def test_reference_reads_follow_the_update(gpu_lib, wins, rstream):
    """Reading the reference pyramid back right after an update on the second
    stream (tracks of the previous reference still in flight) returns the new
    reference, level by level, as the one-stream context does; so do the
    template cache and a batch's packed levels."""
    dpt = gpu_lib
    prm = dpt.make_params(levels=4)
    one = dpt.Tracker(synth.CAM_752, prm, max_points=N)
    two = dpt.Tracker(synth.CAM_752, prm, max_points=N)
    two.set_reference_stream(rstream)
    for w in wins[:4]:
        for t in (one, two):
            t.build_pyramid(dpt.SLOT_REF, w["img0"])
            t.set_reference_from_depth(N, w["depth"], w["T0"])
        for l in range(4):
            np.testing.assert_array_equal(one.get_pyramid(dpt.SLOT_REF, l), two.get_pyramid(dpt.SLOT_REF, l),
                                          err_msg=f"level {l}")
        c1, c2 = one.reference_cache(1), two.reference_cache(1)
        for k in ("valid", "I0", "gx", "gy", "x0"):
            np.testing.assert_array_equal(c1[k], c2[k], err_msg=k)
        for t in (one, two):  # tracks in flight while the next reference is built
            t.set_pose_history(w["T_prev"], w["T0"])
            t.track_window_enqueue(w["frames"])
    _assert_same(one.synchronize(), two.synchronize())
    one.close()
    two.close()


def test_batch_levels_follow_the_update(gpu_lib, bwins, rstream):
    dpt = gpu_lib
    prm = dpt.make_params(levels=4)
    bts = [dpt.BatchTracker([synth.CAM_752] * S, prm, [N] * S) for _ in range(2)]
    bts[1].set_reference_stream(rstream)
    for w in range(len(bwins[0])):
        ws = [bwins[s][w] for s in range(S)]
        for bt in bts:
            bt.build_pyramids(dpt.SLOT_REF, [x["img0"] for x in ws])
            bt.set_reference_from_depth_all(N, [x["depth"] for x in ws], np.stack([x["T0"] for x in ws]))
        for l in range(4):
            np.testing.assert_array_equal(bts[0].get_level(dpt.SLOT_REF, l), bts[1].get_level(dpt.SLOT_REF, l))
        for bt in bts:
            bt.set_pose_history_all(np.stack([x["T_prev"] for x in ws]), np.stack([x["T0"] for x in ws]))
            bt.track_window_enqueue([x["frames"] for x in ws])
    _assert_same_batch(bts[0].synchronize(), bts[1].synchronize())
    for bt in bts:
        bt.close()


def test_library_streams_can_be_made_and_released(gpu_lib):
    dpt = gpu_lib
    streams = [dpt.Stream() for _ in range(3)]
    assert len({s.cuda_stream for s in streams}) == 3 and all(s.cuda_stream for s in streams)
    for s in streams:
        s.close()
        assert s.cuda_stream == 0
        s.close()  # a second close is a no-op


@pytest.mark.parametrize("slow", ["reference", "tracks"])
def test_ordering_holds_when_one_stream_lags(gpu_lib, wins, rstream, slow):
    """A bounded spin kernel ahead of every reference update (the tracks must
    wait for the update) or ahead of every window track (the next update must
    wait for the tracks still reading the bank it overwrites): the tracks stay
    bitwise those of the one-stream context."""
    import torch

    dpt = gpu_lib
    prm = dpt.make_params(levels=4)
    base, _ = _run(dpt, wins, prm, (3, 128), True, None)
    trk = dpt.Tracker(synth.CAM_752, prm, max_points=N)
    trk.set_launch_config(3, 128)
    trk.set_reference_stream(rstream)
    ref_side = torch.cuda.ExternalStream(rstream.cuda_stream)
    main_side = torch.cuda.ExternalStream(trk.stream) if trk.stream else torch.cuda.default_stream()
    spin = 1_500_000  # shader clock cycles, under a millisecond
    for w in wins:
        if slow == "reference":
            with torch.cuda.stream(ref_side):
                torch.cuda._sleep(spin)
        trk.build_pyramid(dpt.SLOT_REF, w["img0"])
        trk.set_reference_from_depth(N, w["depth"], w["T0"])
        trk.set_pose_history(w["T_prev"], w["T0"])
        if slow == "tracks":
            with torch.cuda.stream(main_side):
                torch.cuda._sleep(spin)
        trk.track_window_enqueue(w["frames"])
    piped = trk.synchronize()
    trk.close()
    _assert_same(base, piped)


@pytest.mark.parametrize("slow", ["reference", "tracks"])
def test_batch_ordering_holds_when_one_stream_lags(gpu_lib, bwins, rstream, slow):
    import torch

    dpt = gpu_lib
    prm = dpt.make_params(levels=4)
    base, _ = _run_batch(dpt, bwins, prm, (3, 128), True, None)
    bt = dpt.BatchTracker([synth.CAM_752] * S, prm, [N] * S)
    bt.set_launch_config(3, 128)
    bt.set_reference_stream(rstream)
    ref_side = torch.cuda.ExternalStream(rstream.cuda_stream)
    main_side = torch.cuda.ExternalStream(bt.stream) if bt.stream else torch.cuda.default_stream()
    for w in range(len(bwins[0])):
        ws = [bwins[s][w] for s in range(S)]
        if slow == "reference":
            with torch.cuda.stream(ref_side):
                torch.cuda._sleep(1_500_000)
        bt.build_pyramids(dpt.SLOT_REF, [x["img0"] for x in ws])
        if w % 2 == 0:
            bt.set_reference_from_depth_all(N, [x["depth"] for x in ws], np.stack([x["T0"] for x in ws]))
        else:
            for s, x in enumerate(ws):
                bt.set_reference_from_depth(s, N, x["depth"], x["T0"])
        bt.set_pose_history_all(np.stack([x["T_prev"] for x in ws]), np.stack([x["T0"] for x in ws]))
        if slow == "tracks":
            with torch.cuda.stream(main_side):
                torch.cuda._sleep(1_500_000)
        bt.track_window_enqueue([x["frames"] for x in ws])
    piped = bt.synchronize()
    bt.close()
    _assert_same_batch(base, piped)
