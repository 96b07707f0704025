"""The C ABI from plain C: tests/c/track_pair.c includes include/dptrack.h as
C99, links libdptrack.so and tracks one frame with no Python in its process,
frame by frame and as a one-frame window track of the host image.  CPU: it
compiles and links warning-free.  GPU: its pose matches the oracle's and the
window track returns the same bytes."""
import os
import struct
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "c", "track_pair")


def test_c_client_compiles_and_links(tmp_path):
    import __graft_entry__ as g

    out = g.build_c_client(str(tmp_path / "track_pair"))
    assert os.path.exists(out)
    # the client links only the library's ABI: every dpt_* symbol it imports is declared in the header
    syms = subprocess.run(["nm", "-D", "--undefined-only", out], capture_output=True, text=True, check=True).stdout
    used = {line.split()[-1] for line in syms.splitlines() if "dpt_" in line}
    header = open(os.path.join(ROOT, "include", "dptrack.h")).read()
    assert used and all(f"{s}(" in header for s in used)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", [0, 7])
def test_c_client_tracks_like_the_oracle(tmp_path, seed):
    import oracle
    import synth

    if not os.path.exists(CLIENT):
        import __graft_entry__ as g

        g.build_c_client()
    cam = synth.CAM_640
    d = synth.pair(seed, cam)
    idx = oracle.select_points(d["ref"], 500, 8)
    P = synth.backproject(cam, d["depth"], idx, d["T_rw"])
    job = tmp_path / "job.bin"
    with open(job, "wb") as f:
        f.write(struct.pack("4i", cam.width, cam.height, 3, len(P)))
        f.write(struct.pack("4d", cam.fx, cam.fy, cam.cx, cam.cy))
        f.write(np.ascontiguousarray(d["T_rw"], np.float64).tobytes())
        f.write(np.eye(4).tobytes())
        f.write(np.ascontiguousarray(d["ref"], np.uint8).tobytes())
        f.write(np.ascontiguousarray(d["cur"], np.uint8).tobytes())
        f.write(np.ascontiguousarray(P, np.float32).tobytes())
    out = tmp_path / "out.bin"
    r = subprocess.run([CLIENT, str(job), str(out)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    raw = out.read_bytes()
    assert len(raw) % 2 == 0 and raw[:len(raw) // 2] == raw[len(raw) // 2:]  # the window track: bitwise the same
    T = np.frombuffer(raw[:128], np.float64).reshape(4, 4)
    final_cost = struct.unpack("d", raw[128:136])[0]
    iterations, status = struct.unpack("i", raw[136:140])[0], struct.unpack("i", raw[176:180])[0]
    o = oracle.Reference(cam, oracle.make_params(levels=3), d["ref"], P, d["T_rw"]).track(d["cur"], np.eye(4))
    rot, tr = oracle.pose_error(T, o["T_cw"])
    assert status == o["status"] == 0
    assert rot < 1e-4 and tr < 1e-4
    assert abs(final_cost - o["final_cost"]) <= 1e-3 * o["final_cost"]
    assert iterations > 0
