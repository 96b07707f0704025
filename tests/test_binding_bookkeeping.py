"""The Python binding's bookkeeping of results in flight, on the CPU against a
stub of the C library (no GPU): after a failed collect or synchronise the
binding releases its result buffers and window frames only once the library
reports that no track is in flight any more, since until then the library may
still write the results and a kernel may still read the frames."""
import ctypes

import pytest

import paper_2607_16897_amd as dpt


class StubLib:
    """Mimics the in-flight counting of the C side; `fail_with` makes the next
    collect / synchronise fail, leaving `left_after_fail` tracks in flight."""

    def __init__(self, n_streams=1):
        self.in_flight = 0
        self.fail_with = 0
        self.left_after_fail = 0
        self.n_streams = n_streams
        self.destroyed = 0

    def dpt_last_error(self):
        return b"stub failure"

    # single context
    def dpt_track_enqueue(self, h, mode, T, out):
        self.in_flight += 1
        return 0

    def dpt_tracks_in_flight(self, h):
        return self.in_flight

    def _wait(self, n):
        if self.fail_with:
            self.in_flight = self.left_after_fail
            return self.fail_with
        self.in_flight -= n
        return 0

    def dpt_collect(self, h, n):
        return self._wait(n)

    def dpt_synchronize(self, h):
        return self._wait(self.in_flight)

    def dpt_destroy(self, h):
        self.destroyed += 1

    # batch
    dpt_batch_track_enqueue = dpt_track_enqueue
    dpt_batch_tracks_in_flight = dpt_tracks_in_flight
    dpt_batch_collect = dpt_collect
    dpt_batch_synchronize = dpt_synchronize
    dpt_batch_destroy = dpt_destroy


@pytest.fixture
def stub(monkeypatch):
    lib = StubLib()
    monkeypatch.setattr(dpt, "_lib", lib)  # _check() reads the error message through load()
    return lib


def _tracker(cls, lib, n=1):
    t = object.__new__(cls)
    t._lib, t._h, t._pending, t._frames_keep = lib, ctypes.c_void_p(1), [], []
    if cls is dpt.BatchTracker:
        t.n = n
    return t


@pytest.mark.parametrize("cls", [dpt.Tracker, dpt.BatchTracker])
@pytest.mark.parametrize("how", ["collect", "synchronize"])
def test_failed_wait_releases_buffers_when_nothing_is_in_flight(stub, cls, how):
    t = _tracker(cls, stub)
    for _ in range(4):
        t.track_enqueue(None)
    stub.fail_with, stub.left_after_fail = dpt.DPT_E_HIP, 0
    with pytest.raises(dpt.DptError) as ei:
        t.collect(2) if how == "collect" else t.synchronize()
    assert ei.value.code == dpt.DPT_E_HIP and "stub failure" in str(ei.value)
    assert len(ei.value.results) == 4  # every result travels with the error
    assert t._pending == [] and t._frames_keep == []
    t.close()
    assert stub.destroyed == 1


@pytest.mark.parametrize("cls", [dpt.Tracker, dpt.BatchTracker])
@pytest.mark.parametrize("how", ["collect", "synchronize"])
def test_failed_wait_keeps_buffers_while_tracks_are_in_flight(stub, cls, how):
    t = _tracker(cls, stub)
    for _ in range(3):
        t.track_enqueue(None)
    kept = list(t._pending)
    stub.fail_with, stub.left_after_fail = dpt.DPT_E_HIP, 3
    with pytest.raises(dpt.DptError):
        t.collect(1) if how == "collect" else t.synchronize()
    assert t._pending == kept and len(t._frames_keep) == 3
    # once the library has let go, a later synchronise hands them over
    stub.fail_with = 0
    assert len(t.synchronize()) == 3
    assert t._pending == [] and t._frames_keep == []
    t.close()


def test_collect_bookkeeping_without_failure(stub):
    t = _tracker(dpt.Tracker, stub)
    for _ in range(5):
        t.track_enqueue(None)
    assert len(t.collect(2)) == 2 and stub.in_flight == 3 and len(t._pending) == 3
    assert len(t.collect(0)) == 0 and stub.in_flight == 3
    assert len(t.synchronize()) == 3 and stub.in_flight == 0
    with pytest.raises(ValueError):
        t.collect(1)
    t.close()


def test_close_at_exit_hook(stub):
    t = _tracker(dpt.Tracker, stub)
    dpt._live.add(t)
    dpt._close_live()
    assert stub.destroyed == 1 and t._h is None and t not in dpt._live
