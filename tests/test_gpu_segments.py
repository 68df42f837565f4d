"""Segment-list ant tours against the oracle.

With segment lists the local search reads each ant's tour through segment
records (a storage range, its orientation, the array position of its first
element) and a move rewrites records instead of elements; when the records
run short the tour is written out in array order and cut again.  Array
positions stay exactly those of the flat arrays, so every iteration must match
the oracle bit for bit.  Cases force segment lists on small tours, with
segments as short as 2 cities (every move splits, neighbour walks cross
records) and record limits a few above the tour's chunk count (a
materialisation every move or two), on one wave and on teams."""
import numpy as np
import pytest

from paper_2203_02228_amd import faco as F
from paper_2203_02228_amd import instances as I
from tests.test_gpu_parity import _cmp_iter, _cmp_setup, _pair, say

pytestmark = pytest.mark.gpu

# (n, kind, seed, params, segment length log2, record limit)
CASES = [
    (9, "uniform", 3, dict(n_ants=4, min_new_edges=0, rho=0.2), 1, 12),
    (64, "uniform", 4, dict(n_ants=5, min_new_edges=3), 0, 0),
    (257, "uniform", 9, dict(n_ants=7, min_new_edges=6, rho=0.9, p_source_gbest=0.5), 1, 140),
    (700, "cluster16", 13, dict(n_ants=5, min_new_edges=12, ls_flags=1), 3, 100),
    (1000, "cluster16", 5, dict(n_ants=6, min_new_edges=20, ls_flags=6, oropt_max_seg=3), 2, 300),
    (3000, "cluster16", 12, dict(n_ants=8, min_new_edges=40), 4, 200),
    (6000, "uniform", 14, dict(n_ants=6, min_new_edges=24, rho=0.8), 0, 0),
    (4000, "cluster16", 15, dict(n_ants=7, min_new_edges=4, min_new_edges_max=60), 5, 130),
    (2500, "uniform", 16, dict(n_ants=6, min_new_edges=12, ls_flags=15), 3, 2048),
]


@pytest.fixture(params=[1, 4, 8])
def team(request):
    F.faco_set_team_waves(request.param)
    try:
        yield request.param
    finally:
        F.faco_set_team_waves(0)


def _build(xy, lg, mx, **params):
    F.faco_set_tour_segments(2, lg, mx)
    try:
        return _pair(xy, threads=8, **params)
    finally:
        F.faco_set_tour_segments(0, 0, 0)


@pytest.mark.parametrize("n,kind,seed,params,lg,mx", CASES)
def test_segments_every_iteration(team, n, kind, seed, params, lg, mx):
    say(f"[gpu] segments team={team} n={n} kind={kind} log2={lg} records={mx} {params}")
    xy = I.make_points(kind, n, seed)
    o, g = _build(xy, lg, mx, **params)
    tour = F.faco_debug_get(g, F.FACO_DBG_TOUR)
    assert tour[0] == 1, tour
    F.faco_set_verify(g, True)
    _cmp_setup(o, g)
    for it in range(1, 6):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
        f = F.faco_debug_get(g, F.FACO_DBG_FAULT)
        assert f[0] == 0, f.tolist()
    tk = F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS)
    moves = int(F.faco_debug_get(g, F.FACO_DBG_COUNTER_TOTALS)[:, 6:8].sum())
    if moves:
        assert tk[:, 19].sum() > 0, "no split recorded"
    g.close()


def test_segments_many_iterations_one_setting():
    """A tour with 4-city segments and a tight record limit over 25
    iterations: epochs and storage buffers alternate many times."""
    F.faco_set_team_waves(8)
    try:
        xy = I.make_points("cluster16", 5000, 21)
        o, g = _build(xy, 2, 1300, n_ants=8, min_new_edges=30)
    finally:
        F.faco_set_team_waves(0)
    _cmp_setup(o, g)
    for it in range(1, 26):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    tk = F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS)
    assert tk[:, 16].sum() > 0  # materialisations happened
    g.close()


def test_segments_then_batch_reads_flat():
    """An instance run with segment lists and then in a batch (flat arrays):
    the batch's tours are read from the buffer its kernel wrote."""
    F.faco_set_team_waves(4)
    try:
        xy = I.make_points("uniform", 3000, 31)
        o, g = _build(xy, 3, 500, n_ants=6, min_new_edges=20)
    finally:
        F.faco_set_team_waves(0)
    _cmp_setup(o, g)
    for it in range(1, 4):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    o.run(2)
    F.faco_run_batch([g], 2)
    _cmp_iter(o, g, 5)
    g.close()


def test_default_is_flat_and_forced_segments():
    """Flat arrays unless segment lists are asked for; then the segment
    length by size (the smallest power of two >= 64 giving <= 512 chunks)."""
    F.faco_set_team_waves(0)
    g = F.faco_build_instance(I.make_points("uniform", 20000, 41), n_ants=8)
    assert F.faco_debug_get(g, F.FACO_DBG_TOUR)[0] == 0
    g.close()
    F.faco_set_tour_segments(2, 0, 0)
    try:
        g = F.faco_build_instance(I.make_points("uniform", 20000, 41), n_ants=8)
        t = F.faco_debug_get(g, F.FACO_DBG_TOUR)
        assert t[0] == 1 and t[1] == 64 and t[2] == 2048, t
        g.close()
        g = F.faco_build_instance(I.make_points("uniform", 100000, 41), n_ants=4)
        t = F.faco_debug_get(g, F.FACO_DBG_TOUR)
        assert t[1] == 256, t
        g.close()
    finally:
        F.faco_set_tour_segments(0, 0, 0)


def test_segment_setting_errors():
    for args in [(3, 0, 0), (-1, 0, 0), (2, 25, 0), (2, -1, 0), (2, 0, 7), (2, 0, 2049)]:
        with pytest.raises(F.FacoError) as e:
            F.faco_set_tour_segments(*args)
        assert e.value.code == F.FACO_EINVAL
    # too few records for the tour's chunks: the build fails
    F.faco_set_tour_segments(2, 1, 20)
    try:
        with pytest.raises(F.FacoError) as e:
            F.faco_build_instance(I.make_points("uniform", 100, 1), n_ants=4)
        assert e.value.code == F.FACO_EINVAL
    finally:
        F.faco_set_tour_segments(0, 0, 0)
    g = F.faco_build_instance(I.make_points("uniform", 100, 1), n_ants=4)
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_TOUR), [0, 0, 0])
    g.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,iters", [("uniform1k", 200), ("gmm20k", 100), ("stipple100k", 30)])
def test_segments_configured_workloads(name, iters):
    """The configured workloads with segment lists (team size and segment
    length by size), against the oracle: lengths, counters, state, limits and
    source every iteration; routes, pheromone and the best tour every 10th and
    at the end; at 100k the device also recomputes every tour length."""
    from tests.test_gpu_configs import HOST_THREADS, _cmp_heavy, _cmp_light
    from oracle import oracle as O
    w = I.WORKLOADS[name]
    xy = w.points()
    say(f"[gpu] segments {name}: n={w.n} iterations={iters}")
    o = O.Oracle(xy, threads=HOST_THREADS, **w.params())
    F.faco_set_tour_segments(2, 0, 0)
    try:
        g = F.faco_build_instance(xy, **w.params())
    finally:
        F.faco_set_tour_segments(0, 0, 0)
    assert F.faco_debug_get(g, F.FACO_DBG_TOUR)[0] == 1
    F.faco_set_verify(g, name == "stipple100k")
    _cmp_setup(o, g)
    for it in range(1, iters + 1):
        F.faco_run_iterations(g, 1)
        o.run(1)
        _cmp_light(o, g, it)
        if it % 10 == 0 or it == iters:
            _cmp_heavy(o, g, it)
    tk = F.faco_debug_get(g, F.FACO_DBG_PHASE_TICKS)
    assert tk[:, 19].sum() > 0  # moves split records
    g.close()
    o.close()
