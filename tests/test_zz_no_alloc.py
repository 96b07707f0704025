"""The allocation-free selection entry point (dpt_select_points_noalloc):
through the C ABI, bit-exact against dpt_select_points, the existing entry
point with context memory, on calls in a row of decreasing size (the static
scratch keeps the previous call's contents), a padded row pitch, and a map
asking for more points than there are candidates; sizes beyond the static
scratch are rejected before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _render(cam, seed):
    scene, traj = synth.Scene(seed), synth.Trajectory(seed)
    img, _ = scene.render(cam, traj.T_cw(40), synth.pixel_noise(seed, 40, cam, 2.0), want_depth=False)
    return img


def _with_context(dpt, cam, img, n, margin):
    trk = dpt.Tracker(cam, dpt.make_params(levels=3), max_points=min(n, 16000))
    trk.build_pyramid(dpt.SLOT_REF, img)
    idx = trk.select_points(n, margin)
    trk.close()
    return idx


def _noalloc(dpt, img_dev, n, margin):
    import torch

    idx = torch.full((n + 7,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    dpt.select_points_noalloc(img_dev, n, margin, idx, cnt)
    torch.cuda.synchronize()
    k = int(cnt.item())
    out = idx.cpu().numpy()
    assert np.all(out[k:] == -1), "entries past the count were written"
    return out[:k]


def test_noalloc_selection_equals_context_selection(gpu_lib):
    import torch

    dpt = gpu_lib
    cases = [(synth.CAM_1280, 11, 16000, 8), (synth.CAM_752, 12, 2000, 8), (synth.CAM_640, 13, 500, 8)]
    for cam, seed, n, margin in cases:  # each call smaller than the one before
        img = _render(cam, seed)
        print(f"noalloc selection {cam.width}x{cam.height} n={n}", flush=True)
        got = _noalloc(dpt, torch.from_numpy(img).cuda(), n, margin)
        want = _with_context(dpt, cam, img, n, margin)
        np.testing.assert_array_equal(got, want)
        assert len(got) == n
        if n <= 2000:
            np.testing.assert_array_equal(got, oracle.select_points(img, n, margin))


def test_noalloc_padded_pitch_and_take_all(gpu_lib):
    import torch

    dpt = gpu_lib
    img = _render(synth.CAM_640, 14)
    wide = torch.zeros((480, 704), dtype=torch.uint8, device="cuda")
    wide[:, :640] = torch.from_numpy(img).cuda()
    view = wide[:, :640]  # rows 704 bytes apart
    got = _noalloc(dpt, view, 3000, 8)
    np.testing.assert_array_equal(got, _with_context(dpt, synth.CAM_640, img, 3000, 8))
    # more points asked than candidates: every candidate, in index order
    tiny = np.ascontiguousarray(img[:40, :48])
    got = _noalloc(dpt, torch.from_numpy(tiny).cuda(), 1500, 8)
    assert len(got) == (48 - 16) * (40 - 16)
    np.testing.assert_array_equal(got, oracle.select_points(tiny, 1500, 8))


def test_noalloc_rejects_sizes_beyond_the_scratch(gpu_lib):
    import torch

    dpt = gpu_lib
    lib = dpt.load()
    idx = torch.zeros(16, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    big = ctypes.c_void_p(16)  # never dereferenced: the size check comes first
    assert lib.dpt_select_points_noalloc(big, 4097, 4096, 4097, 10, 8, idx.data_ptr(), cnt.data_ptr(),
                                         None) == dpt.DPT_E_ARG
    assert b"static scratch" in lib.dpt_last_error()
    img = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    assert lib.dpt_select_points_noalloc(img.data_ptr(), 64, 64, 63, 10, 8, idx.data_ptr(), cnt.data_ptr(),
                                         None) == dpt.DPT_E_ARG
    assert lib.dpt_select_points_noalloc(None, 64, 64, 64, 10, 8, idx.data_ptr(), cnt.data_ptr(),
                                         None) == dpt.DPT_E_ARG
    assert lib.dpt_select_points_noalloc(img.data_ptr(), 64, 64, 64, 10, 32, idx.data_ptr(), cnt.data_ptr(),
                                         None) == dpt.DPT_E_ARG
