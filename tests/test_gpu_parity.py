"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tours, lengths, counters, lists and pheromone must be identical: the method's
floating-point steps are specified to the rounding (binary32 weights summed in
slot order, binary64 limits), so the benchmark spec's tolerance of 1e-6 relative on
pheromone is met with zero difference; the test asserts bit equality."""
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


def _pair(xy, threads=8, **params):
    o = O.Oracle(xy, threads=threads, **params)
    g = F.faco_build_instance(xy, **params)
    return o, g


def _cmp_setup(o, g, rows=None):
    cl, bl = o.lists()
    gcl = F.faco_debug_get(g, F.FACO_DBG_CAND_LISTS)
    gbl = F.faco_debug_get(g, F.FACO_DBG_BACKUP_LISTS)
    assert np.array_equal(gcl, cl)
    assert np.array_equal(gbl, bl)
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_HEURISTIC), o.heuristic())
    info_g = F.faco_debug_get(g, F.FACO_DBG_INFO)
    info_o = o.info()
    assert info_g[5] == info_o[5], "initial length"
    assert np.array_equal(F.faco_get_best_tour(g)[0], o.best()[0])
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_INIT_COUNTERS), o.init_counters())
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_LIMITS)[:2], o.limits()[:2])
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_PHEROMONE), o.pheromone())
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_SOURCE), o.source()[0])


def _cmp_iter(o, g, it):
    gr = F.faco_debug_get(g, F.FACO_DBG_ANT_ROUTES)
    orr = o.ant_routes()
    if not np.array_equal(gr, orr):
        bad = [a for a in range(orr.shape[0]) if not np.array_equal(gr[a], orr[a])]
        pos = np.nonzero(gr[bad[0]] != orr[bad[0]])[0][:5]
        raise AssertionError(f"iteration {it}: ant routes differ for ants {bad[:8]}, "
                             f"first positions {pos.tolist()}")
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_ANT_LENGTHS), o.ant_lengths()), it
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_COUNTERS), o.ant_counters()), it
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_INFO), o.info()), it
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_LIMITS), o.limits()), it
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_SOURCE), o.source()[0]), it
    tg, to = F.faco_debug_get(g, F.FACO_DBG_PHEROMONE), o.pheromone()
    assert np.array_equal(tg, to), (it, float(np.max(np.abs(tg - to) / to)))
    bt, bl = F.faco_get_best_tour(g)
    ot, ol = o.best()
    assert bl == ol and np.array_equal(bt, ot), it
    assert F.faco_debug_get(g, F.FACO_DBG_FAULT)[0] == 0, it


SMALL = [
    (4, "uniform", 1, dict(n_ants=3, min_new_edges=1, cl_size=16)),
    (5, "uniform", 2, dict(n_ants=4, min_new_edges=0, rho=0.2)),
    (7, "uniform", 3, dict(n_ants=5, min_new_edges=2, cl_size=3, bl_size=1)),
    (12, "uniform", 4, dict(n_ants=6, min_new_edges=2, ls_flags=1)),
    (33, "cluster16", 5, dict(n_ants=4, min_new_edges=5, cl_size=7, bl_size=5,
                              ls_flags=6, oropt_max_seg=2)),
    (64, "uniform", 6, dict(n_ants=8, min_new_edges=10**6, cl_size=5, bl_size=2)),
    (65, "uniform", 7, dict(n_ants=8, min_new_edges=3, cl_size=6, bl_size=0)),
    (130, "cluster16", 8, dict(n_ants=8, min_new_edges=4, ls_flags=0)),
    (257, "uniform", 9, dict(n_ants=7, min_new_edges=6, rho=0.9, p_source_gbest=0.5)),
    # calc_num_new_edges() drawn per ant from a range
    (300, "cluster16", 10, dict(n_ants=9, min_new_edges=2, min_new_edges_max=25)),
    # initial solution with 3-opt (2-opt + Or-opt + 3-opt), and without Or-opt
    (400, "uniform", 11, dict(n_ants=6, min_new_edges=8, ls_flags=15)),
    (150, "cluster16", 12, dict(n_ants=5, min_new_edges=4, cl_size=6, ls_flags=13)),
    (9, "uniform", 13, dict(n_ants=4, min_new_edges=2, ls_flags=15)),
]


@pytest.mark.parametrize("n,kind,seed,params", SMALL)
def test_small_instances_every_iteration(n, kind, seed, params):
    say(f"[gpu] small n={n} kind={kind} params={params}")
    xy = I.make_points(kind, n, seed)
    o, g = _pair(xy, threads=1, **params)
    _cmp_setup(o, g)
    for it in range(1, 9):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    g.close()


def test_uniform1k_every_iteration():
    w = I.WORKLOADS["uniform1k"]
    say(f"[gpu] uniform1k n={w.n} params={w.params()}")
    xy = w.points()
    o, g = _pair(xy, **w.params())
    _cmp_setup(o, g)
    for it in range(1, 31):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    # batched enqueue of several iterations gives the same state
    o.run(10)
    F.faco_run_iterations(g, 10)
    _cmp_iter(o, g, 40)
    g.close()


def test_gmm20k_first_iterations():
    w = I.WORKLOADS["gmm20k"]
    say(f"[gpu] gmm20k n={w.n} params={w.params()}")
    xy = w.points()
    o, g = _pair(xy, **w.params())
    _cmp_setup(o, g)
    for it in range(1, 4):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    g.close()


def test_build_errors():
    xy = I.uniform(50, 1)
    dup = xy.copy()
    dup[9] = dup[2]
    with pytest.raises(F.FacoError) as e:
        F.faco_build_instance(dup)
    assert e.value.code == F.FACO_EDUP
    with pytest.raises(F.FacoError) as e:
        F.faco_build_instance(xy, rho=1.5)
    assert e.value.code == F.FACO_EINVAL


def test_full_coordinate_range():
    """Coordinates up to 2^26 - 1 (squared lengths up to 2^53): the cost
    function's extreme range, including near-collinear and far pairs."""
    rng = np.random.default_rng(77)
    pts = rng.integers(0, (1 << 26), size=(1500, 2))
    pts[:20, 0] = (1 << 26) - 1 - np.arange(20)       # a column at the far edge
    pts[20:40] = np.stack([np.arange(20) * 3, np.zeros(20, np.int64)], 1)  # tight row
    xy = np.unique(pts, axis=0).astype(np.int32)
    xy = xy[rng.permutation(len(xy))]
    params = dict(n_ants=8, min_new_edges=6, rho=0.5)
    say(f"[gpu] full coordinate range n={len(xy)}")
    o, g = _pair(xy, **params)
    _cmp_setup(o, g)
    for it in range(1, 6):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    g.close()


@pytest.mark.parametrize("spacing", [1, 7])
def test_integer_grid(spacing):
    """A 32 x 32 integer grid: squared lengths hit r^2 + r and r^2 - r + 1
    (the nint boundaries, e.g. sqrt(20) -> 4, sqrt(13) -> 4, sqrt(5) -> 2) and
    distances tie massively (lists break ties by city id)."""
    g1 = np.arange(32, dtype=np.int32) * spacing + 5
    xy = np.stack(np.meshgrid(g1, g1, indexing="ij"), -1).reshape(-1, 2).astype(np.int32)
    xy = xy[np.random.default_rng(spacing).permutation(len(xy))].copy()
    params = dict(n_ants=6, min_new_edges=10, cl_size=10, bl_size=20)
    say(f"[gpu] integer grid spacing={spacing}")
    o, g = _pair(xy, **params)
    _cmp_setup(o, g)
    for it in range(1, 5):
        o.run(1)
        F.faco_run_iterations(g, 1)
        _cmp_iter(o, g, it)
    g.close()


def test_build_on_recycled_device_blocks():
    """Destroyed instances leave their device blocks to the library, and the
    next builds of similar size take them back with their old contents: an
    instance built on such blocks still matches the oracle bit for bit."""
    say("[gpu] recycled blocks: build, run, destroy n=3000, then n=2950 and n=3050")
    first = F.faco_build_instance(I.make_points("uniform", 3000, 81), n_ants=6, min_new_edges=8)
    F.faco_run_iterations(first, 4)
    F.faco_get_best_tour(first)
    first.close()
    for n, seed in ((2950, 82), (3050, 83)):
        xy = I.make_points("cluster16", n, seed)
        g = F.faco_build_instance(xy, n_ants=6, min_new_edges=8)
        o = O.Oracle(xy, threads=8, n_ants=6, min_new_edges=8)
        _cmp_setup(o, g)
        for it in range(1, 4):
            o.run(1)
            F.faco_run_iterations(g, 1)
            _cmp_iter(o, g, it)
        g.close()
        o.close()
