"""The initial solution's phase ticks (FACO_DBG_INIT_TICKS), and the record
of an attempt to share its sweeps with helper workgroups."""
import numpy as np
import pytest

from paper_2203_02228_amd import faco as F
from paper_2203_02228_amd import instances as I
from tests.test_gpu_parity import _cmp_iter, _cmp_setup, say

pytestmark = pytest.mark.gpu


def test_initial_solution_ticks():
    """Every sweep of the initial search tests all n cities (the whole tour is
    touched), the phases fit inside the kernel's time, and the search made
    evaluation rounds and sweeps."""
    n = 5000
    say(f"[gpu] init ticks n={n}")
    g = F.faco_build_instance(I.make_points("uniform", n, 71), n_ants=4, min_new_edges=8)
    tk = F.faco_debug_get(g, F.FACO_DBG_INIT_TICKS)
    cnt = F.faco_debug_get(g, F.FACO_DBG_INIT_COUNTERS)
    sweeps = cnt[F.CNT_NAMES.index("sweeps")]
    assert sweeps > 0 and tk[26] == n * sweeps
    assert tk[12] > 0                      # evaluation rounds
    assert 0 < tk[0] + tk[1] + tk[2] + tk[3] <= tk[4]
    g.close()


@pytest.mark.skip(reason="sharing the initial solution's sweeps with helper workgroups of its "
                         "launch was removed: its first GPU run printed nothing for 180 s on "
                         "this first case (16384 cities, 8-wave team) and was stopped, and no "
                         "cause was found by reading the code; the build's normal path is "
                         "compared with the oracle by the configured-workload tests")
@pytest.mark.parametrize("tw", [8, 4, 1])
@pytest.mark.parametrize("n,kind,seed", [(16384, "uniform", 61), (40000, "stipple", 62)])
def test_initial_solution_with_shared_sweeps(tw, n, kind, seed):
    from oracle import oracle as O
    say(f"[gpu] shared init sweeps: tw={tw} n={n} kind={kind}")
    xy = I.make_points(kind, n, seed)
    params = dict(n_ants=4, min_new_edges=8, rho=0.5, seed=seed)
    F.faco_set_team_waves(tw)
    try:
        g = F.faco_build_instance(xy, **params)
    finally:
        F.faco_set_team_waves(0)
    o = O.Oracle(xy, threads=8, **params)
    f = F.faco_debug_get(g, F.FACO_DBG_FAULT)
    assert f[0] == 0, f.tolist()
    _cmp_setup(o, g)
    tk = F.faco_debug_get(g, F.FACO_DBG_INIT_TICKS)
    init_cnt = F.faco_debug_get(g, F.FACO_DBG_INIT_COUNTERS)
    assert init_cnt[F.CNT_NAMES.index("sweeps")] > 0
    assert tk[26] == n * init_cnt[F.CNT_NAMES.index("sweeps")]
    o.run(1)
    F.faco_run_iterations(g, 1)
    _cmp_iter(o, g, 1)
    g.close()
    o.close()
