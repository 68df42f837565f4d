"""Served stream: requests of different sizes admitted by footprint, batched
with each other while resident; each result equals the same request solved
alone."""
import sys
import time

import numpy as np
import pytest

from paper_2203_02228_amd import faco as F
from paper_2203_02228_amd import instances as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_mix_equals_alone_under_small_budget():
    import torch
    from paper_2203_02228_amd import serve as S
    torch.cuda.set_device(0)
    sizes = [1200, 300, 5000, 800, 15000, 2500, 600, 9000]
    reqs = []
    for i, n in enumerate(sizes):
        kind = "stipple" if i % 2 == 0 else "uniform"
        xy = I.make_points(kind, n, 900 + i)
        params = dict(n_ants=8 + (i % 3) * 4, min_new_edges=8, rho=0.5, seed=i + 1,
                      cl_size=16 if i % 4 else 12)
        reqs.append((xy, params, 20 + 7 * (i % 3)))
    fps = [F.faco_footprint_bytes(len(x), F.make_params(**p)) for x, p, _ in reqs]
    budget = max(fps) + sorted(fps)[len(fps) // 2]
    say(f"[gpu] serve mix sizes={sizes} budget={budget}")
    srv = S.Server(hbm_budget_bytes=budget, chunk=5, builders=2)
    peak = [0]
    futs = []
    for i, (xy, p, it) in enumerate(reqs):
        futs.append(srv.submit(i, xy, p, it))
        time.sleep(0.01)
        peak[0] = max(peak[0], srv.used)
    got = [f.result(timeout=300) for f in futs]
    srv.close()
    assert peak[0] <= budget
    assert srv.used == 0 and not srv.errors
    for (xy, p, it), (tour, L) in zip(reqs, got):
        g = F.faco_build_instance(xy, **p)
        F.faco_run_iterations(g, it)
        t2, L2 = F.faco_get_best_tour(g)
        g.close()
        assert L == L2 and np.array_equal(tour, t2)


def test_request_larger_than_budget_is_rejected():
    import torch
    from paper_2203_02228_amd import serve as S
    torch.cuda.set_device(0)
    srv = S.Server(hbm_budget_bytes=1 << 20, chunk=5, builders=1)
    fut = srv.submit(0, I.uniform(5000, 3), dict(n_ants=8), 10)
    with pytest.raises(F.FacoError):
        fut.result(timeout=60)
    srv.close()


def test_capture_alongside_other_threads():
    """A batch graph captured on one thread while another thread builds,
    reads back and releases instances (the served pattern): no call may trip
    over the capture."""
    import threading
    import torch
    from paper_2203_02228_amd import instances as I
    say("[gpu] capture alongside builds, reads and releases")
    ws = I.batch_instances(count=4, seed0=4300, n_hi=1500)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    batch = [F.faco_build_instance(w.points(), stream=s1, **w.params()) for w in ws]
    errors = []

    def runner():
        try:
            for _ in range(12):
                F.faco_run_batch(batch, 5, stream=s1)
                s1.synchronize()
        except Exception as e:  # reported below
            errors.append(repr(e))

    def churn():
        try:
            for i in range(12):
                w = ws[i % len(ws)]
                g = F.faco_build_instance(w.points(), stream=s2, **w.params())
                F.faco_get_best_tour(g)
                F.faco_debug_get(g, F.FACO_DBG_INFO)
                g.close()
        except Exception as e:
            errors.append(repr(e))

    ta, tb = threading.Thread(target=runner), threading.Thread(target=churn)
    ta.start(); tb.start(); ta.join(); tb.join()
    for g in batch:
        g.close()
    assert not errors, errors[:3]


def test_moved_handle_equals_unmoved():
    """faco_set_stream: a handle moved between streams (after a few
    iterations, then batched on a third stream, then read and destroyed on its
    new stream) ends exactly where a handle that stayed on its build stream
    ends; destroyed handles' device blocks are reused by the next builds."""
    import torch
    torch.cuda.set_device(0)
    sa, sb, sc = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    xy = I.make_points("stipple", 3000, 77)
    p = dict(n_ants=12, min_new_edges=8, rho=0.5, seed=5)
    say("[gpu] set_stream: build two handles of n=3000")
    for rep in range(2):
        g0 = F.faco_build_instance(xy, stream=sa, **p)
        g1 = F.faco_build_instance(xy, stream=sa, **p)
        F.faco_run_iterations(g0, 4)
        F.faco_run_iterations(g1, 4)
        F.faco_set_stream(g1, sb)
        F.faco_run_iterations(g0, 3)
        F.faco_run_iterations(g1, 3)
        F.faco_run_batch([g0], 2, stream=sc)
        F.faco_run_batch([g1], 2, stream=sc)
        t0, L0 = F.faco_get_best_tour(g0)
        t1, L1 = F.faco_get_best_tour(g1)
        assert L0 == L1 and np.array_equal(t0, t1)
        for what in (F.FACO_DBG_PHEROMONE, F.FACO_DBG_ANT_ROUTES):
            assert np.array_equal(F.faco_debug_get(g0, what), F.faco_debug_get(g1, what))
        g0.close()
        g1.close()
