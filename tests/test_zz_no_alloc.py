"""faco_run_batch_noalloc (the batched launches with fixed tables, no device
allocation) against faco_run_batch, through the C ABI: two calls in a row,
the second with a smaller batch, each ending in exactly the state the
allocating entry point leaves."""
import sys

import numpy as np
import pytest

from paper_2203_02228_amd import faco as F
from paper_2203_02228_amd import instances as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(g):
    return [F.faco_debug_get(g, F.FACO_DBG_ANT_ROUTES),
            F.faco_debug_get(g, F.FACO_DBG_ANT_LENGTHS),
            F.faco_debug_get(g, F.FACO_DBG_COUNTERS),
            F.faco_debug_get(g, F.FACO_DBG_PHEROMONE),
            F.faco_debug_get(g, F.FACO_DBG_SOURCE),
            F.faco_debug_get(g, F.FACO_DBG_INFO),
            F.faco_debug_get(g, F.FACO_DBG_LIMITS),
            F.faco_get_best_tour(g)[0]]


def _pair_run(ws, iterations):
    a = [F.faco_build_instance(w.points(), **w.params()) for w in ws]
    b = [F.faco_build_instance(w.points(), **w.params()) for w in ws]
    F.faco_run_batch_noalloc(a, iterations)
    F.faco_run_batch(b, iterations)
    for w, ga, gb in zip(ws, a, b):
        sa, sb = _state(ga), _state(gb)
        for x, y in zip(sa, sb):
            assert np.array_equal(x, y), w.name
        assert F.faco_debug_get(ga, F.FACO_DBG_FAULT)[0] == 0
    for g in a + b:
        g.close()


def test_noalloc_matches_batch_twice_second_smaller():
    # first call: uneven sizes up to 3000 cities (team kernel: 8 waves per ant)
    ws1 = I.batch_instances(count=7, seed0=4600, n_lo=300, n_hi=3000)
    ws1[1].cl_size = 16
    ws1[2].n_ants = 5
    say(f"[gpu] noalloc call 1 sizes={[w.n for w in ws1]}")
    _pair_run(ws1, 4)
    # second call: fewer, smaller instances (one wave per ant)
    ws2 = I.batch_instances(count=3, seed0=4700, n_lo=200, n_hi=1200)
    ws2[0].n_ants = 9
    say(f"[gpu] noalloc call 2 sizes={[w.n for w in ws2]}")
    _pair_run(ws2, 3)


def test_noalloc_limits_and_stream_rule():
    import torch
    xy = I.uniform(8, 2)
    many = [F.faco_build_instance(xy, n_ants=1, cl_size=4, bl_size=0) for _ in range(257)]
    with pytest.raises(F.FacoError) as e:
        F.faco_run_batch_noalloc(many, 1)
    assert e.value.code == F.FACO_EINVAL
    for g in many:
        g.close()
    wide = [F.faco_build_instance(xy, n_ants=4096, cl_size=4, bl_size=0) for _ in range(5)]
    with pytest.raises(F.FacoError) as e:
        F.faco_run_batch_noalloc(wide, 1)
    assert e.value.code == F.FACO_EINVAL
    for g in wide:
        g.close()
    s = torch.cuda.Stream()
    other = F.faco_build_instance(I.uniform(50, 3), n_ants=2, stream=s)
    with pytest.raises(F.FacoError) as e:
        F.faco_run_batch_noalloc([other], 1)
    assert e.value.code == F.FACO_EINVAL
    F.faco_run_batch_noalloc([other], 2, stream=s)
    s.synchronize()
    assert F.faco_debug_get(other, F.FACO_DBG_INFO)[0] == 2
    other.close()
