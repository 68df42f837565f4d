"""The C oracle against the independent pure-Python statement (tests/pyref.py)
on tiny instances: every array must agree exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_02228_amd import instances as I
from tests import pyref

CASES = [
    # n, kind, seed, params
    (30, "uniform", 1, dict(cl_size=8, bl_size=6, n_ants=4, min_new_edges=3, rho=0.5)),
    (40, "cluster16", 2, dict(cl_size=6, bl_size=4, n_ants=3, min_new_edges=0, rho=0.02)),
    (25, "uniform", 3, dict(cl_size=16, bl_size=64, n_ants=5, min_new_edges=4, rho=0.3,
                            p_source_gbest=0.5)),
    (36, "cluster16", 4, dict(cl_size=5, bl_size=2, n_ants=4, min_new_edges=10**6, rho=0.7)),
    (12, "uniform", 5, dict(cl_size=4, bl_size=0, n_ants=6, min_new_edges=2, rho=0.5,
                            ls_flags=O.LS_2OPT)),
    (33, "uniform", 6, dict(cl_size=7, bl_size=5, n_ants=4, min_new_edges=5, rho=0.5,
                            ls_flags=O.LS_OROPT | O.LS_SWEEP, oropt_max_seg=2)),
    (34, "cluster16", 7, dict(cl_size=6, bl_size=4, n_ants=5, min_new_edges=1, rho=0.4,
                              min_new_edges_max=9)),
    # initial solution with 3-opt
    (38, "uniform", 8, dict(cl_size=7, bl_size=4, n_ants=4, min_new_edges=3, rho=0.5,
                            ls_flags=15)),
    (30, "cluster16", 9, dict(cl_size=5, bl_size=3, n_ants=3, min_new_edges=2, rho=0.5,
                              ls_flags=O.LS_2OPT | O.LS_SWEEP | O.LS_INIT_3OPT)),
]


@pytest.mark.parametrize("n,kind,seed,params", CASES)
def test_oracle_matches_python_statement(n, kind, seed, params):
    xy = I.make_points(kind, n, seed)
    o = O.Oracle(xy, **params)
    r = pyref.Ref(xy, **params)
    cl, bl = o.lists()
    assert cl.tolist() == r.cl
    assert bl.tolist() == [list(x) for x in r.bll]
    nn, _ = o.nearest_neighbour()
    assert nn.tolist() == r.nn
    gb, L = o.best()
    assert gb.tolist() == r.gb and L == r.gb_len
    tmin, tmax, _ = o.limits()
    assert tmin == r.tau_min and tmax == r.tau_max
    for it in range(6):
        o.run(1)
        r.run(1)
        assert o.ant_routes().tolist() == r.routes, it
        assert o.ant_lengths().tolist() == r.lens
        src, Ls = o.source()
        assert src.tolist() == r.src and Ls == r.src_len
        assert np.array_equal(o.pheromone(), np.array(r.tau, np.float32))
        assert o.best()[0].tolist() == r.gb
        tmin, tmax, delta = o.limits()
        assert (tmin, tmax, delta) == (r.tau_min, r.tau_max, r.delta)


def test_local_search_arrays_match_python_statement():
    n = 45
    xy = I.make_points("cluster16", n, 9)
    for flags in (O.LS_2OPT, O.LS_2OPT | O.LS_SWEEP, O.LS_2OPT | O.LS_OROPT | O.LS_SWEEP,
                  O.LS_OROPT, O.LS_2OPT | O.LS_INIT_3OPT | O.LS_SWEEP,
                  O.LS_2OPT | O.LS_OROPT | O.LS_INIT_3OPT | O.LS_SWEEP):
        o = O.Oracle(xy, cl_size=8, ls_flags=flags)
        r = pyref.Ref(xy, cl_size=8, ls_flags=flags)
        rng = np.random.default_rng(flags)
        for trial in range(4):
            route = rng.permutation(n).astype(np.int32)
            chk = rng.choice(n, size=15, replace=False).astype(np.int32)
            out, g, _ = o.local_search(route, chk, flags)
            ref = r.local_search(route.tolist(), chk.tolist(), flags)
            assert out.tolist() == ref
