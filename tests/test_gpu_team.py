"""Ant teams (several waves per ant) against the oracle.

With 4 or 8 waves per ant the speculative windows span 256 or 512 steps, the
2-opt reversals and Or-opt block moves above one wave's round are split
across the waves, and sweep tests run 64 cities per wave.  None of that may
change a result: every iteration must match the oracle bit for bit, as the
one-wave kernel does.  Cases cover tours shorter than one window, the
window-only regime (m larger than n), Or-opt-only and 2-opt-only searches, and
tours long enough (n >= 4096) for team reversals and shifts."""
import pytest

from paper_2203_02228_amd import faco as F
from paper_2203_02228_amd import instances as I
from tests.test_gpu_parity import _cmp_iter, _cmp_setup, _pair, say

pytestmark = pytest.mark.gpu

CASES = [
    (5, "uniform", 2, dict(n_ants=4, min_new_edges=0, rho=0.2)),
    (33, "cluster16", 5, dict(n_ants=4, min_new_edges=5, cl_size=7, bl_size=5,
                              ls_flags=6, oropt_max_seg=2)),
    (257, "uniform", 9, dict(n_ants=7, min_new_edges=6, rho=0.9, p_source_gbest=0.5)),
    (300, "uniform", 11, dict(n_ants=6, min_new_edges=10**6, cl_size=5, bl_size=2)),
    (700, "cluster16", 13, dict(n_ants=5, min_new_edges=12, ls_flags=1)),
    (3000, "cluster16", 12, dict(n_ants=8, min_new_edges=40)),
    (6000, "uniform", 14, dict(n_ants=6, min_new_edges=24, rho=0.8)),
    (4000, "cluster16", 15, dict(n_ants=7, min_new_edges=4, min_new_edges_max=60)),
    (2500, "uniform", 16, dict(n_ants=6, min_new_edges=12, ls_flags=15)),
]


@pytest.fixture(params=[4, 8])
def team(request):
    F.faco_set_team_waves(request.param)
    try:
        yield request.param
    finally:
        F.faco_set_team_waves(0)


@pytest.mark.parametrize("n,kind,seed,params", CASES)
def test_team_every_iteration(team, n, kind, seed, params):
    say(f"[gpu] team={team} n={n} kind={kind} params={params}")
    xy = I.make_points(kind, n, seed)
    o, g = _pair(xy, threads=8, **params)
    assert int(F.faco_debug_get(g, F.FACO_DBG_TEAM_WAVES)[0]) == team
    _cmp_setup(o, g)
    for it in range(1, 6):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    g.close()


def test_team_setting_errors():
    with pytest.raises(F.FacoError) as e:
        F.faco_set_team_waves(3)
    assert e.value.code == F.FACO_EINVAL
    F.faco_set_team_waves(0)


@pytest.mark.parametrize("tw,n,kind,seed,params", [
    (1, 700, "cluster16", 13, dict(n_ants=5, min_new_edges=30)),
    (4, 3000, "cluster16", 12, dict(n_ants=8, min_new_edges=40)),
    (8, 6000, "uniform", 14, dict(n_ants=6, min_new_edges=60, rho=0.8)),
])
def test_small_lds_queue_spills(tw, n, kind, seed, params):
    """A 64-entry LDS queue: the initial search starts in the global ring and
    iterations overflow the LDS ring into it; results must not change."""
    say(f"[gpu] lds queue 64 team={tw} n={n} params={params}")
    F.faco_set_team_waves(tw)
    F.faco_set_queue_lds_capacity(64)
    try:
        xy = I.make_points(kind, n, seed)
        o, g = _pair(xy, threads=8, **params)
    finally:
        F.faco_set_queue_lds_capacity(0)
        F.faco_set_team_waves(0)
    _cmp_setup(o, g)
    for it in range(1, 5):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    g.close()


def test_queue_capacity_errors():
    for bad in (1, 63, 16385, -5):
        with pytest.raises(F.FacoError) as e:
            F.faco_set_queue_lds_capacity(bad)
        assert e.value.code == F.FACO_EINVAL
    F.faco_set_queue_lds_capacity(0)


def test_team_nearest_on_grid(team):
    """A 64 x 64 integer grid with one backup city: the nearest-unvisited scan
    runs often, its bound and box pruning meet massive distance ties (settled
    by original number), and the results must match the oracle's."""
    import numpy as np
    g1 = np.arange(64, dtype=np.int32) * 3 + 7
    xy = np.stack(np.meshgrid(g1, g1, indexing="ij"), -1).reshape(-1, 2).astype(np.int32)
    xy = xy[np.random.default_rng(5).permutation(len(xy))].copy()
    say(f"[gpu] team={team} grid 64x64 nearest")
    o, g = _pair(xy, threads=8, n_ants=5, min_new_edges=20, cl_size=4, bl_size=1)
    _cmp_setup(o, g)
    fallbacks = 0
    for it in range(1, 4):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
        fallbacks += int(F.faco_debug_get(g, F.FACO_DBG_COUNTERS)[:, 3].sum())
    assert fallbacks > 0
    g.close()
