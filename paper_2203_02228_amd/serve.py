"""Continuous-batching solve server over the C ABI.

Requests (points + parameters + an iteration budget) arrive at any time.  A
request is admitted when its device footprint (faco_footprint_bytes: points,
candidate/backup lists, pheromone, tours) fits in the HBM budget next to the
solves already resident; it is then built on a builder stream, moved to the
stream of its size class and joins the running batch of that class at the
next batch call.  Each size class has a
worker with its own stream that advances all of its resident solves together
(faco_run_batch, one launch per phase) in chunks of iterations, retires the
ones that reached their budget and admits newly built ones between chunks.
State stays on the device from build to retirement.  The method's arithmetic
is unchanged: a solve returns exactly what a lone faco_run_iterations run of
the same request returns.

The builder and class streams only overlap on the GPU if each has a hardware
queue of its own: HIP maps a process's streams onto GPU_MAX_HW_QUEUES queues
(4 unless set, read when HIP initialises), and streams that share a queue run
in submission order, so a class would wait behind another stream's builds.
Start a serving process with at least builders + classes + 1 queues.
"""
import collections
import concurrent.futures as cf
import os
import threading
import time
import warnings
from dataclasses import dataclass, field

import numpy as np

from . import faco as F

# upper bounds (exclusive) of the size classes, each with its own worker
DEFAULT_CLASSES = (4_000, 16_000, 64_000, 1 << 30)


@dataclass
class Request:
    rid: int
    xy: np.ndarray
    params: dict
    iterations: int
    arrival: float = 0.0          # host clock when submitted
    admitted: float = 0.0
    built: float = 0.0
    finished: float = 0.0
    footprint: int = 0
    handle: object = None
    done_iters: int = 0
    result: tuple = None
    future: cf.Future = field(default_factory=cf.Future)


class Server:
    def __init__(self, hbm_budget_bytes=8 << 30, chunk=10, classes=DEFAULT_CLASSES,
                 builders=3, ants_per_block=1):
        import torch  # streams
        self._torch = torch
        self.budget = int(hbm_budget_bytes)
        self.chunk = int(chunk)
        self.classes = tuple(classes)
        self.used = 0
        self.lock = threading.Condition()
        self.waiting = collections.deque()     # not yet admitted
        self.ready = [collections.deque() for _ in self.classes]  # built, not yet batched
        self.closed = False
        self.completed = []
        self.errors = []
        self.tuned = {}
        # per size class: batch calls, iterations, resident solves summed over
        # calls, the most resident at once, and host time inside batch calls
        self.class_stats = [dict(calls=0, iterations=0, active_sum=0, max_active=0, busy_s=0.0)
                            for _ in self.classes]
        F.faco_set_batch_ants_per_block(ants_per_block)
        need = builders + len(self.classes) + 1
        have = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
        if have < need:
            warnings.warn(f"GPU_MAX_HW_QUEUES={have} < {need}: builder and class streams "
                          "share hardware queues, and solves wait behind other builds")
        self.build_streams = [torch.cuda.Stream() for _ in range(builders)]
        self.run_streams = [torch.cuda.Stream() for _ in self.classes]
        self.build_q = collections.deque()
        self.threads = []
        for b in range(builders):
            t = threading.Thread(target=self._builder, args=(b,), daemon=True)
            t.start()
            self.threads.append(t)
        for c in range(len(self.classes)):
            t = threading.Thread(target=self._worker, args=(c,), daemon=True)
            t.start()
            self.threads.append(t)

    # ------------------------------------------------------------- public
    def submit(self, rid, xy, params, iterations):
        p = F.make_params(**params)
        fp = F.faco_footprint_bytes(len(xy), p)
        if fp == 0:
            raise F.FacoError(F.FACO_EINVAL, "invalid request")
        r = Request(rid, np.ascontiguousarray(xy, np.int32), dict(params), int(iterations),
                    arrival=time.perf_counter(), footprint=fp)
        with self.lock:
            if fp > self.budget:
                r.future.set_exception(F.FacoError(F.FACO_ENOMEM,
                                                   "request can never fit the HBM budget"))
                return r.future
            self.waiting.append(r)
            self._admit_locked()
            self.lock.notify_all()
        return r.future

    def tune(self, samples, trial_iterations=3):
        """Autotune the batch configuration of each size class on sample
        requests [(xy, params)] built on the side (the library's autotuner
        times every configuration on twins and stores the fastest for the
        class; later batches of the class use it).  Returns {class: config}."""
        by_class = {}
        for xy, params in samples:
            by_class.setdefault(self._class_of(len(xy)), []).append((xy, params))
        out = {}
        for c, items in sorted(by_class.items()):
            stream = self.run_streams[c]
            hs = [F.faco_build_instance(xy, stream=stream, **p) for xy, p in items]
            try:
                out[c] = F.faco_autotune_batch(hs, trial_iterations, stream=stream)
            finally:
                for h in hs:
                    h.close()
        self.tuned = out
        return out

    def close(self, wait=True):
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        if wait:
            for t in self.threads:
                t.join()

    def drain(self):
        """Block until every submitted request has finished."""
        with self.lock:
            while self.waiting or self.build_q or any(self.ready) or self._busy():
                self.lock.wait(0.05)

    # ------------------------------------------------------------ internals
    def _busy(self):
        return self.used > 0

    def _class_of(self, n):
        for c, hi in enumerate(self.classes):
            if n < hi:
                return c
        return len(self.classes) - 1

    def _admit_locked(self):
        # FIFO admission by footprint
        while self.waiting and self.used + self.waiting[0].footprint <= self.budget:
            r = self.waiting.popleft()
            self.used += r.footprint
            r.admitted = time.perf_counter()
            self.build_q.append(r)
        self.lock.notify_all()

    def _release(self, r):
        with self.lock:
            self.used -= r.footprint
            self._admit_locked()

    def _builder(self, b):
        stream = self.build_streams[b]
        while True:
            with self.lock:
                while not self.build_q and not self.closed:
                    self.lock.wait()
                if not self.build_q and self.closed:
                    return
                r = self.build_q.popleft()
            try:
                r.handle = F.faco_build_instance(r.xy, stream=stream, **r.params)
                # the solve now lives on its class's stream: its batches and
                # reads must not wait for the next builds on this stream
                F.faco_set_stream(r.handle, self.run_streams[self._class_of(len(r.xy))])
                r.built = time.perf_counter()
                with self.lock:
                    self.ready[self._class_of(len(r.xy))].append(r)
                    self.lock.notify_all()
            except Exception as e:  # report and free the slot
                self._fail(r, e)

    def _fail(self, r, exc):
        """Resolve r's future with exc, free its device state and footprint."""
        if not r.future.done():
            r.future.set_exception(exc)
        self.errors.append((r.rid, repr(exc)))
        h, r.handle = r.handle, None
        if h is not None:
            try:
                h.close()
            except Exception as e:  # the slot is released regardless
                self.errors.append((r.rid, "close: " + repr(e)))
        self._release(r)

    def _retire(self, r):
        """Read back a finished solve, free it and resolve its future."""
        try:
            tour, length = F.faco_get_best_tour(r.handle)
            r.finished = time.perf_counter()
            r.result = (tour, length)
            h, r.handle = r.handle, None
            h.close()
        except Exception as e:
            self._fail(r, e)
            return
        self.completed.append(r)
        r.future.set_result((tour, length))
        self._release(r)

    def _worker(self, c):
        stream = self.run_streams[c]
        active = []
        while True:
            with self.lock:
                while not active and not self.ready[c] and not self.closed:
                    self.lock.wait()
                if not active and not self.ready[c] and self.closed:
                    return
                while self.ready[c]:
                    active.append(self.ready[c].popleft())
            try:
                steps = min(self.chunk, min(r.iterations - r.done_iters for r in active))
                t0 = time.perf_counter()
                F.faco_run_batch([r.handle for r in active], steps, stream=stream)
                stream.synchronize()
                st = self.class_stats[c]
                st["calls"] += 1
                st["iterations"] += steps
                st["active_sum"] += len(active)
                st["max_active"] = max(st["max_active"], len(active))
                st["busy_s"] += time.perf_counter() - t0
            except Exception as e:
                # every resident solve of the class fails with the batch
                for r in active:
                    self._fail(r, e)
                self.errors.append(("batch", repr(e)))
                active = []
                continue
            keep = []
            for r in active:
                r.done_iters += steps
                if r.done_iters >= r.iterations:
                    self._retire(r)
                else:
                    keep.append(r)
            active = keep


def latency_stats(reqs):
    lat = np.array([r.finished - r.arrival for r in reqs])
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}
