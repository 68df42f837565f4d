"""Every configured workload over its whole iteration budget, against the CPU
oracle element by element.

* uniform1k (1000 cities, 16 ants, m 8, retention 0.02): all 200 iterations,
  every array every iteration.
* gmm20k (20 000 clustered cities, 32 ants, m 16): all 500 iterations;
  lengths, counters, state, limits, source and faults every iteration; ant
  routes and pheromone every 10th and at the end.
* stipple100k (100 000 stipple cities, 64 ants, m 32): all 1000 iterations;
  the same per-iteration set; ant routes and pheromone every 10th and at
  the end; the device recomputes and checks every tour length in every
  iteration (verification on).
* batch256 (256 uneven instances, 200-5000 cities, k 12, 16 ants, m 8): one
  faco_run_batch call of all 300 iterations; every instance's final ant
  routes, lengths, counters, pheromone, source, state and global best against
  its own oracle run.
* served: the first eight requests of the Poisson stipple stream (1 341 to
  128 396 cities) and its 192 728-city request, 32 ants, m 16, 200
  iterations, through the continuous-batching server under an HBM budget
  that forces queueing; each result against the oracle.

The oracle runs on the host while the GPU works; a progress line is printed
as the runs advance."""
import concurrent.futures as cf
import os
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2203_02228_amd import faco as F
from paper_2203_02228_amd import instances as I
from tests.test_gpu_parity import _cmp_iter, _cmp_setup

pytestmark = pytest.mark.gpu

HOST_THREADS = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _no_fault(g, where):
    f = F.faco_debug_get(g, F.FACO_DBG_FAULT)
    assert f[0] == 0, f"{where}: device fault {f.tolist()}"
    return f


def _cmp_light(o, g, it):
    """Per-iteration state that every later iteration depends on."""
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_ANT_LENGTHS), o.ant_lengths()), it
    gc, oc = F.faco_debug_get(g, F.FACO_DBG_COUNTERS), o.ant_counters()
    if not np.array_equal(gc, oc):
        bad = np.nonzero((gc != oc).any(1))[0]
        raise AssertionError(f"iteration {it}: counters differ for ants {bad[:8].tolist()}: "
                             f"{gc[bad[0]].tolist()} vs {oc[bad[0]].tolist()}")
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_INFO), o.info()), it
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_LIMITS), o.limits()), it
    assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_SOURCE), o.source()[0]), it
    _no_fault(g, f"iteration {it}")


def _cmp_heavy(o, g, it):
    gr, orr = F.faco_debug_get(g, F.FACO_DBG_ANT_ROUTES), o.ant_routes()
    if not np.array_equal(gr, orr):
        bad = [a for a in range(orr.shape[0]) if not np.array_equal(gr[a], orr[a])]
        raise AssertionError(f"iteration {it}: ant routes differ for ants {bad[:8]}")
    tg, to = F.faco_debug_get(g, F.FACO_DBG_PHEROMONE), o.pheromone()
    assert np.array_equal(tg, to), (it, float(np.max(np.abs(tg - to) / to)))
    bt, bl = F.faco_get_best_tour(g)
    ot, ol = o.best()
    assert bl == ol and np.array_equal(bt, ot), it


def _full_run(name, heavy_every, verify):
    w = I.WORKLOADS[name]
    t0 = time.time()
    xy = w.points()
    say(f"[gpu] {name}: n={w.n} params={w.params()} iterations={w.iterations} "
        f"(points {time.time() - t0:.1f} s)")
    o = O.Oracle(xy, threads=HOST_THREADS, **w.params())
    g = F.faco_build_instance(xy, **w.params())
    F.faco_set_verify(g, verify)
    _cmp_setup(o, g)
    t0 = time.time()
    for it in range(1, w.iterations + 1):
        F.faco_run_iterations(g, 1)   # enqueued; runs while the oracle works
        o.run(1)
        _cmp_light(o, g, it)
        if it % heavy_every == 0 or it == w.iterations:
            _cmp_heavy(o, g, it)
        if it % 50 == 0:
            say(f"[gpu] {name}: {it}/{w.iterations} iterations identical "
                f"({time.time() - t0:.0f} s), best {o.best()[1]}")
    f = _no_fault(g, name)
    if verify:
        assert f[3] == w.iterations * (w.n_ants + 1), f.tolist()
    rec = F.faco_debug_get(g, F.FACO_DBG_RECOMPUTED_LENGTHS)
    assert np.array_equal(rec[:-1], o.ant_lengths()) and rec[-1] == o.best()[1]
    g.close()
    o.close()


@pytest.mark.timeout(300)
def test_uniform1k_all_200_iterations():
    w = I.WORKLOADS["uniform1k"]
    xy = w.points()
    say(f"[gpu] uniform1k: every array, every iteration, {w.iterations} iterations")
    o = O.Oracle(xy, threads=1, **w.params())
    g = F.faco_build_instance(xy, **w.params())
    _cmp_setup(o, g)
    for it in range(1, w.iterations + 1):
        F.faco_run_iterations(g, 1)
        o.run(1)
        _cmp_iter(o, g, it)
        _no_fault(g, f"iteration {it}")
    g.close()


@pytest.mark.timeout(400)
def test_gmm20k_all_500_iterations():
    _full_run("gmm20k", heavy_every=10, verify=False)


@pytest.mark.timeout(600)
def test_stipple100k_all_1000_iterations():
    _full_run("stipple100k", heavy_every=10, verify=True)


def _oracle_final(xy, params, iterations, threads):
    o = O.Oracle(xy, threads=threads, **params)
    o.run(iterations)
    out = dict(routes=o.ant_routes(), lengths=o.ant_lengths(), counters=o.ant_counters(),
               tau=o.pheromone(), source=o.source()[0], info=o.info(), limits=o.limits(),
               best=o.best())
    o.close()
    return out


@pytest.mark.timeout(600)
def test_batch256_all_300_iterations():
    ws = I.batch_instances(count=256)
    iters = ws[0].iterations
    say(f"[gpu] batch256: {len(ws)} instances n in [{min(w.n for w in ws)}, "
        f"{max(w.n for w in ws)}], {iters} iterations in one faco_run_batch call")
    pts = [w.points() for w in ws]
    t0 = time.time()
    hs = [F.faco_build_instance(p, **w.params()) for p, w in zip(pts, ws)]
    for h in hs:
        F.faco_set_verify(h, True)
    F.faco_run_batch(hs, iters)
    # the oracles run meanwhile, one instance per host thread
    done = 0
    with cf.ThreadPoolExecutor(HOST_THREADS) as ex:
        futs = {ex.submit(_oracle_final, p, w.params(), iters, 1): i
                for i, (p, w) in enumerate(zip(pts, ws))}
        for fut in cf.as_completed(futs):
            i = futs[fut]
            ref, g, w = fut.result(), hs[i], ws[i]
            assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_ANT_ROUTES), ref["routes"]), w.name
            assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_ANT_LENGTHS), ref["lengths"]), w.name
            assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_COUNTERS), ref["counters"]), w.name
            assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_PHEROMONE), ref["tau"]), w.name
            assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_SOURCE), ref["source"]), w.name
            assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_INFO), ref["info"]), w.name
            assert np.array_equal(F.faco_debug_get(g, F.FACO_DBG_LIMITS), ref["limits"]), w.name
            bt, bl = F.faco_get_best_tour(g)
            assert bl == ref["best"][1] and np.array_equal(bt, ref["best"][0]), w.name
            f = _no_fault(g, w.name)
            assert f[3] == iters * (w.n_ants + 1), (w.name, f.tolist())
            g.close()
            done += 1
            if done % 32 == 0:
                say(f"[gpu] batch256: {done}/{len(ws)} instances identical "
                    f"({time.time() - t0:.0f} s)")
    assert done == len(ws)


@pytest.mark.timeout(600)
def test_served_stream_against_oracle():
    import torch
    from paper_2203_02228_amd import serve as S
    torch.cuda.set_device(0)
    stream = I.served_requests(count=256)
    picked = list(range(8)) + [67]
    reqs = [stream[i][1] for i in picked]
    say(f"[gpu] served: requests {picked} sizes {[w.n for w in reqs]}")
    t0 = time.time()
    pts = [w.points() for w in reqs]
    say(f"[gpu] served: points generated ({time.time() - t0:.0f} s)")
    fps = sorted(F.faco_footprint_bytes(w.n, F.make_params(**w.params())) for w in reqs)
    budget = fps[-1] + fps[-2]    # the two largest fit together, not three
    srv = S.Server(hbm_budget_bytes=budget, chunk=10, builders=2)
    futs = []
    for i, (w, p) in enumerate(zip(reqs, pts)):
        futs.append(srv.submit(picked[i], p, w.params(), w.iterations))
        time.sleep(0.05)
    # the oracle runs of the same requests, meanwhile
    per = max(1, HOST_THREADS // 4)
    with cf.ThreadPoolExecutor(4) as ex:
        refs = [ex.submit(_oracle_final, p, w.params(), w.iterations, per)
                for w, p in zip(reqs, pts)]
        for k, (w, fut, ref) in enumerate(zip(reqs, futs, refs)):
            tour, length = fut.result(timeout=600)
            r = ref.result()
            assert length == r["best"][1] and np.array_equal(tour, r["best"][0]), w.name
            say(f"[gpu] served: request {picked[k]} n={w.n} identical to the oracle "
                f"({time.time() - t0:.0f} s)")
    srv.close()
    assert srv.used == 0 and not srv.errors, srv.errors
