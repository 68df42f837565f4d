"""Tour-length verification and device faults (through the C ABI).

The verification kernel recomputes every tour's length from the stored
route and the coordinates; here those sums are checked against lengths
recomputed on the host from the dumped routes (exact integer EUC_2D) and
against the lengths the construction and local search tracked."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_02228_amd import faco as F
from paper_2203_02228_amd import instances as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host_lengths(xy, routes):
    """EUC_2D tour lengths by exact integer arithmetic (numpy)."""
    xy = xy.astype(np.int64)
    nxt = np.roll(routes, -1, axis=-1)
    d = xy[routes] - xy[nxt]
    d2 = (d * d).sum(-1)
    r = np.floor(np.sqrt(d2.astype(np.float64))).astype(np.int64)
    for _ in range(2):
        r = np.where(r * r > d2, r - 1, r)
        r = np.where((r + 1) * (r + 1) <= d2, r + 1, r)
    c = r + (d2 > r * r + r)
    return c.sum(-1)


@pytest.mark.parametrize("tw", [1, 8])
def test_verification_every_iteration(tw):
    xy = I.make_points("cluster16", 3000, 31)
    params = dict(n_ants=12, min_new_edges=10)
    say(f"[gpu] verify tw={tw}")
    F.faco_set_team_waves(tw)
    try:
        g = F.faco_build_instance(xy, **params)
    finally:
        F.faco_set_team_waves(0)
    rec0 = F.faco_debug_get(g, F.FACO_DBG_RECOMPUTED_LENGTHS)
    assert (rec0[:-1] == 0).all() and rec0[-1] == F.faco_debug_get(g, F.FACO_DBG_INFO)[6]
    F.faco_set_verify(g, True)
    F.faco_run_iterations(g, 8)
    f = F.faco_debug_get(g, F.FACO_DBG_FAULT)
    assert f[0] == 0 and f[3] == 1 + 8 * 13, f.tolist()
    routes = F.faco_debug_get(g, F.FACO_DBG_ANT_ROUTES)
    lens = F.faco_debug_get(g, F.FACO_DBG_ANT_LENGTHS)
    rec = F.faco_debug_get(g, F.FACO_DBG_RECOMPUTED_LENGTHS)
    assert np.array_equal(rec[:-1], lens)
    assert np.array_equal(host_lengths(xy, routes), lens)
    bt, bl = F.faco_get_best_tour(g)
    assert rec[-1] == bl == host_lengths(xy, bt)
    assert (np.sort(routes, axis=1) == np.arange(3000)).all()
    g.close()


def test_verification_in_batches():
    ws = I.batch_instances(count=5, seed0=4400, n_hi=3000)
    say(f"[gpu] verify batch sizes={[w.n for w in ws]}")
    hs = [F.faco_build_instance(w.points(), **w.params()) for w in ws]
    for h in hs[::2]:
        F.faco_set_verify(h, True)
    F.faco_run_batch(hs, 1)
    F.faco_run_batch(hs, 5)
    for i, (w, h) in enumerate(zip(ws, hs)):
        f = F.faco_debug_get(h, F.FACO_DBG_FAULT)
        assert f[0] == 0, (w.name, f.tolist())
        assert f[3] == (6 * (w.n_ants + 1) if i % 2 == 0 else 0), (w.name, f.tolist())
        rec = F.faco_debug_get(h, F.FACO_DBG_RECOMPUTED_LENGTHS)
        assert np.array_equal(rec[:-1], F.faco_debug_get(h, F.FACO_DBG_ANT_LENGTHS))
        h.close()


def test_threshold_range_against_oracle_with_verification():
    """calc_num_new_edges() drawn per ant: every iteration identical to the
    oracle, with the device checking every length."""
    xy = I.make_points("uniform", 2500, 33)
    params = dict(n_ants=10, min_new_edges=3, min_new_edges_max=40)
    say("[gpu] threshold range n=2500")
    o = O.Oracle(xy, threads=8, **params)
    g = F.faco_build_instance(xy, **params)
    F.faco_set_verify(g, True)
    for it in range(1, 7):
        o.run(1)
        F.faco_run_iterations(g, 1)
        assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_ANT_ROUTES), o.ant_routes()), it
        assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_COUNTERS), o.ant_counters()), it
        assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_PHEROMONE), o.pheromone()), it
    assert F.faco_debug_get(g, F.FACO_DBG_FAULT)[0] == 0
    g.close()


def test_invalid_threshold_range_rejected():
    xy = I.uniform(50, 1)
    with pytest.raises(F.FacoError) as e:
        F.faco_build_instance(xy, min_new_edges=8, min_new_edges_max=5)
    assert e.value.code == F.FACO_EINVAL
