"""ctypes binding of the CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module.  It never imports the product package's GPU
library, and the product package never imports it.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc_faco.so")

LS_2OPT, LS_OROPT, LS_SWEEP, LS_INIT_3OPT = 1, 2, 4, 8
CNT_NAMES = ["aco_steps", "copied", "backup", "fallback", "new_edges",
             "ls_pops", "moves_2opt", "moves_oropt", "moved_elems", "sweeps",
             "checklist0", "ls_gain", "moves_3opt"]
NCNT = len(CNT_NAMES)


class OrcParams(ctypes.Structure):
    _fields_ = [("cl_size", ctypes.c_int32), ("bl_size", ctypes.c_int32),
                ("n_ants", ctypes.c_int32), ("min_new_edges", ctypes.c_int32),
                ("rho", ctypes.c_float), ("_pad0", ctypes.c_float),
                ("p_best", ctypes.c_double), ("p_source_gbest", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("ls_flags", ctypes.c_uint32),
                ("oropt_max_seg", ctypes.c_int32), ("min_new_edges_max", ctypes.c_int32),
                ("_pad1", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        i32p, i64p, f32p, u64p = (P(ctypes.c_int32), P(ctypes.c_int64),
                                  P(ctypes.c_float), P(ctypes.c_uint64))
        vp = ctypes.c_void_p
        L.orc_build.restype = vp
        L.orc_build.argtypes = [i32p, ctypes.c_int32, P(OrcParams), ctypes.c_int32]
        L.orc_free.argtypes = [vp]
        L.orc_run.argtypes = [vp, ctypes.c_int32]
        L.orc_best.restype = ctypes.c_int64
        L.orc_best.argtypes = [vp, i32p]
        L.orc_source.restype = ctypes.c_int64
        L.orc_source.argtypes = [vp, i32p]
        L.orc_ant_routes.argtypes = [vp, i32p]
        L.orc_ant_lengths.argtypes = [vp, i64p]
        L.orc_ant_counters.argtypes = [vp, i64p]
        L.orc_init_counters.argtypes = [vp, i64p]
        L.orc_pheromone.argtypes = [vp, f32p]
        L.orc_heuristic.argtypes = [vp, f32p]
        L.orc_lists.argtypes = [vp, i32p, i32p]
        L.orc_limits.argtypes = [vp, f32p]
        L.orc_info.argtypes = [vp, i64p]
        L.orc_set_source.argtypes = [vp, i32p]
        L.orc_set_pheromone.argtypes = [vp, f32p]
        L.orc_construct.restype = ctypes.c_int64
        L.orc_construct.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64, i32p,
                                    i32p, i32p, i64p]
        L.orc_local_search.restype = ctypes.c_int64
        L.orc_local_search.argtypes = [vp, i32p, i32p, ctypes.c_int32,
                                       ctypes.c_uint32, i64p]
        L.orc_nearest_neighbour.restype = ctypes.c_int64
        L.orc_nearest_neighbour.argtypes = [vp, i32p]
        L.orc_min_new_edges.restype = ctypes.c_int32
        L.orc_min_new_edges.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_best_move_gain.restype = ctypes.c_int64
        L.orc_best_move_gain.argtypes = [vp, i32p, ctypes.c_int32, ctypes.c_uint32]
        L.orc_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.orc_nint_sqrt.restype = ctypes.c_int32
        L.orc_nint_sqrt.argtypes = [ctypes.c_int64]
        L.orc_dist.restype = ctypes.c_int32
        L.orc_dist.argtypes = [i32p, ctypes.c_int32, ctypes.c_int32]
        L.orc_tour_length.restype = ctypes.c_int64
        L.orc_tour_length.argtypes = [i32p, ctypes.c_int32, i32p]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox4x64_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, ctypes.c_uint64), _p(k, ctypes.c_uint64),
                            _p(out, ctypes.c_uint64))
    return out


def dist(xy, i, j):
    xy = np.ascontiguousarray(xy, dtype=np.int32)
    return int(lib().orc_dist(_p(xy, ctypes.c_int32), int(i), int(j)))


def nint_sqrt(d2):
    return int(lib().orc_nint_sqrt(int(d2)))


def tour_length(xy, route):
    xy = np.ascontiguousarray(xy, dtype=np.int32)
    r = np.ascontiguousarray(route, dtype=np.int32)
    return int(lib().orc_tour_length(_p(xy, ctypes.c_int32), len(r),
                                     _p(r, ctypes.c_int32)))


def make_params(cl_size=16, bl_size=64, n_ants=16, min_new_edges=8, rho=0.5,
                p_best=0.05, p_source_gbest=0.01, seed=1,
                ls_flags=LS_2OPT | LS_OROPT | LS_SWEEP, oropt_max_seg=3,
                min_new_edges_max=0):
    return OrcParams(cl_size, bl_size, n_ants, min_new_edges, rho, 0.0, p_best,
                     p_source_gbest, seed, ls_flags, oropt_max_seg, min_new_edges_max, 0)


class Oracle:
    """One FACO instance in the CPU oracle."""

    def __init__(self, xy, threads=1, **params):
        self.xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
        self.n = self.xy.shape[0]
        self.params = make_params(**params)
        self.h = lib().orc_build(_p(self.xy, ctypes.c_int32), self.n,
                                 ctypes.byref(self.params), int(threads))
        if not self.h:
            raise ValueError("oracle rejected the instance")
        info = self.info()
        self.k, self.bl = int(info[1]), int(info[2])
        self.A = self.params.n_ants

    def close(self):
        if self.h:
            lib().orc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, iterations):
        lib().orc_run(self.h, int(iterations))

    def info(self):
        out = np.zeros(8, dtype=np.int64)
        lib().orc_info(self.h, _p(out, ctypes.c_int64))
        return out

    def best(self):
        t = np.zeros(self.n, dtype=np.int32)
        L = lib().orc_best(self.h, _p(t, ctypes.c_int32))
        return t, int(L)

    def source(self):
        t = np.zeros(self.n, dtype=np.int32)
        L = lib().orc_source(self.h, _p(t, ctypes.c_int32))
        return t, int(L)

    def ant_routes(self):
        r = np.zeros((self.A, self.n), dtype=np.int32)
        lib().orc_ant_routes(self.h, _p(r, ctypes.c_int32))
        return r

    def ant_lengths(self):
        r = np.zeros(self.A, dtype=np.int64)
        lib().orc_ant_lengths(self.h, _p(r, ctypes.c_int64))
        return r

    def ant_counters(self):
        r = np.zeros((self.A, NCNT), dtype=np.int64)
        lib().orc_ant_counters(self.h, _p(r, ctypes.c_int64))
        return r

    def init_counters(self):
        r = np.zeros(NCNT, dtype=np.int64)
        lib().orc_init_counters(self.h, _p(r, ctypes.c_int64))
        return r

    def pheromone(self):
        r = np.zeros((self.n, self.k), dtype=np.float32)
        lib().orc_pheromone(self.h, _p(r, ctypes.c_float))
        return r

    def heuristic(self):
        r = np.zeros((self.n, self.k), dtype=np.float32)
        lib().orc_heuristic(self.h, _p(r, ctypes.c_float))
        return r

    def lists(self):
        cl = np.zeros((self.n, self.k), dtype=np.int32)
        bl = np.zeros((self.n, max(self.bl, 1)), dtype=np.int32)
        lib().orc_lists(self.h, _p(cl, ctypes.c_int32), _p(bl, ctypes.c_int32))
        return cl, bl[:, :self.bl]

    def limits(self):
        r = np.zeros(3, dtype=np.float32)
        lib().orc_limits(self.h, _p(r, ctypes.c_float))
        return r

    def set_source(self, tour):
        t = np.ascontiguousarray(tour, dtype=np.int32)
        lib().orc_set_source(self.h, _p(t, ctypes.c_int32))

    def set_pheromone(self, tau):
        t = np.ascontiguousarray(tau, dtype=np.float32)
        assert t.shape == (self.n, self.k)
        lib().orc_set_pheromone(self.h, _p(t, ctypes.c_float))

    def construct(self, t, ant):
        route = np.zeros(self.n, dtype=np.int32)
        chk = np.zeros(self.n, dtype=np.int32)
        nchk = ctypes.c_int32(0)
        cnt = np.zeros(NCNT, dtype=np.int64)
        L = lib().orc_construct(self.h, int(t), int(ant), _p(route, ctypes.c_int32),
                                _p(chk, ctypes.c_int32), ctypes.byref(nchk),
                                _p(cnt, ctypes.c_int64))
        return route, chk[:nchk.value].copy(), int(L), cnt

    def local_search(self, route, checklist, flags=None):
        r = np.ascontiguousarray(route, dtype=np.int32).copy()
        c = np.ascontiguousarray(checklist, dtype=np.int32)
        cnt = np.zeros(NCNT, dtype=np.int64)
        fl = self.params.ls_flags if flags is None else flags
        g = lib().orc_local_search(self.h, _p(r, ctypes.c_int32), _p(c, ctypes.c_int32),
                                   len(c), int(fl), _p(cnt, ctypes.c_int64))
        return r, int(g), cnt

    def nearest_neighbour(self):
        r = np.zeros(self.n, dtype=np.int32)
        L = lib().orc_nearest_neighbour(self.h, _p(r, ctypes.c_int32))
        return r, int(L)

    def min_new_edges(self, t, ant):
        """calc_num_new_edges() of ant `ant` at iteration t."""
        return int(lib().orc_min_new_edges(self.h, int(t), int(ant)))

    def best_move_gain(self, route, a, flags=None):
        r = np.ascontiguousarray(route, dtype=np.int32)
        fl = self.params.ls_flags if flags is None else flags
        return int(lib().orc_best_move_gain(self.h, _p(r, ctypes.c_int32), int(a), int(fl)))
