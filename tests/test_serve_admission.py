"""Admission by footprint and continuous batching, with the GPU library
replaced by a stub (host logic only; no GPU)."""
import threading
import types

import numpy as np
import pytest


class _FakeStream:
    def synchronize(self):
        pass


class _FakeTorch(types.SimpleNamespace):
    pass


def _fake_modules(monkeypatch, log):
    from paper_2203_02228_amd import faco as F
    from paper_2203_02228_amd import serve as S

    class H:
        def __init__(self, n):
            self.n, self.it = n, 0

        def close(self):
            log.append(("close", self.n))

    monkeypatch.setattr(F, "faco_footprint_bytes", lambda n, p: 1000 * n)
    monkeypatch.setattr(F, "faco_set_batch_ants_per_block", lambda apb: None)
    monkeypatch.setattr(F, "faco_build_instance", lambda xy, stream=None, **kw: H(len(xy)))

    def set_stream(h, st):
        h.stream = st
    monkeypatch.setattr(F, "faco_set_stream", set_stream)

    def run_batch(hs, steps, stream=None):
        # a resident solve runs on its class's stream, not its builder's
        assert all(getattr(h, "stream", None) is stream for h in hs)
        log.append(("batch", sorted(h.n for h in hs), steps))
        for h in hs:
            h.it += steps
    monkeypatch.setattr(F, "faco_run_batch", run_batch)
    monkeypatch.setattr(F, "faco_get_best_tour", lambda h: (np.arange(h.n), h.n * 10 + h.it))
    fake_torch = _FakeTorch(cuda=types.SimpleNamespace(Stream=_FakeStream))
    import sys
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    return F, S


def test_admission_respects_budget_and_results_arrive(monkeypatch):
    log = []
    F, S = _fake_modules(monkeypatch, log)
    srv = S.Server(hbm_budget_bytes=10_000, chunk=4, classes=(50, 1 << 30), builders=2)
    peak = [0]
    orig = srv._admit_locked

    def watch():
        orig()
        peak[0] = max(peak[0], srv.used)
    srv._admit_locked = watch
    futs = [srv.submit(i, np.zeros((n, 2), np.int32), {}, 10)
            for i, n in enumerate([4, 6, 5, 9, 3, 8, 7])]
    res = [f.result(timeout=20) for f in futs]
    srv.close()
    assert peak[0] <= 10_000
    assert [r[1] for r in res] == [n * 10 + 10 for n in [4, 6, 5, 9, 3, 8, 7]]
    assert srv.used == 0
    # every batch advanced resident solves by at most their remaining budget
    assert all(step <= 4 for kind, *rest in log if kind == "batch" for step in [rest[1]])


def test_oversized_request_rejected(monkeypatch):
    log = []
    F, S = _fake_modules(monkeypatch, log)
    srv = S.Server(hbm_budget_bytes=5_000, chunk=4)
    fut = srv.submit(0, np.zeros((6, 2), np.int32), {}, 10)
    with pytest.raises(F.FacoError):
        fut.result(timeout=5)
    srv.close()


def test_failed_readback_resolves_every_future(monkeypatch):
    """A device error while retiring one solve fails that request only: every
    future resolves, the failed solve's handle is closed and its footprint is
    released, and the worker keeps serving the others."""
    log = []
    F, S = _fake_modules(monkeypatch, log)

    def get_best(h):
        if h.n == 6:
            raise F.FacoError(F.FACO_EDEVICE, "read-back failed")
        return np.arange(h.n), h.n * 10 + h.it
    monkeypatch.setattr(F, "faco_get_best_tour", get_best)
    srv = S.Server(hbm_budget_bytes=10_000, chunk=4, classes=(50, 1 << 30), builders=2)
    sizes = [4, 6, 5, 9, 3]
    futs = [srv.submit(i, np.zeros((n, 2), np.int32), {}, 10) for i, n in enumerate(sizes)]
    for n, f in zip(sizes, futs):
        if n == 6:
            with pytest.raises(F.FacoError):
                f.result(timeout=20)
        else:
            assert f.result(timeout=20)[1] == n * 10 + 10
    srv.close()
    assert srv.used == 0
    assert sorted(e[1] for e in log if e[0] == "close") == sorted(sizes)
    assert any(rid == 1 for rid, _ in srv.errors)


def test_failed_batch_resolves_every_future(monkeypatch):
    """A batch launch that fails fails every solve resident in it: all futures
    resolve with the error, all handles are closed, the budget is free again,
    and later requests are still served."""
    log = []
    F, S = _fake_modules(monkeypatch, log)
    calls = [0]

    def run_batch(hs, steps, stream=None):
        calls[0] += 1
        if calls[0] == 1:
            raise F.FacoError(F.FACO_EDEVICE, "launch failed")
        for h in hs:
            h.it += steps
    monkeypatch.setattr(F, "faco_run_batch", run_batch)
    srv = S.Server(hbm_budget_bytes=100_000, chunk=4, classes=(1 << 30,), builders=1)
    first = srv.submit(0, np.zeros((7, 2), np.int32), {}, 8)
    with pytest.raises(F.FacoError):
        first.result(timeout=20)
    later = srv.submit(1, np.zeros((5, 2), np.int32), {}, 8)
    assert later.result(timeout=20)[1] == 5 * 10 + 8
    srv.close()
    assert srv.used == 0
    assert sorted(e[1] for e in log if e[0] == "close") == [5, 7]
