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

    def run_batch(hs, steps, stream=None):
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
