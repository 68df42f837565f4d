"""Thin Python binding of the C ABI in include/faco.h (argument marshalling
only; every step of the method runs in the HIP library).

The library is ``libfaco_hip.so`` beside this file, built by ``build.py``.
There is no fallback: if the library is missing or cannot be loaded, every
call raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfaco_hip.so")

FACO_OK, FACO_EINVAL, FACO_EDUP, FACO_ENOMEM, FACO_EDEVICE = 0, -1, -2, -3, -4
FACO_LS_2OPT, FACO_LS_OROPT, FACO_LS_SWEEP, FACO_LS_INIT_3OPT = 1, 2, 4, 8
(FACO_DBG_ANT_ROUTES, FACO_DBG_ANT_LENGTHS, FACO_DBG_PHEROMONE, FACO_DBG_SOURCE,
 FACO_DBG_LIMITS, FACO_DBG_COUNTERS, FACO_DBG_CAND_LISTS, FACO_DBG_BACKUP_LISTS,
 FACO_DBG_HEURISTIC, FACO_DBG_INFO, FACO_DBG_INIT_COUNTERS,
 FACO_DBG_COUNTER_TOTALS, FACO_DBG_PHASE_TICKS, FACO_DBG_TEAM_WAVES, FACO_DBG_FAULT,
 FACO_DBG_RECOMPUTED_LENGTHS, FACO_DBG_TOUR, FACO_DBG_INIT_TICKS) = range(18)
FACO_NTICKS = 32  # tick and count slots per ant (FACO_DBG_PHASE_TICKS)
FACO_FAULT_LS_STALL, FACO_FAULT_LENGTH, FACO_FAULT_PERMUTATION = 1, 2, 4
CNT_NAMES = ["aco_steps", "copied", "backup", "fallback", "new_edges",
             "ls_pops", "moves_2opt", "moves_oropt", "moved_elems", "sweeps",
             "checklist0", "ls_gain", "moves_3opt"]
FACO_NCNT = len(CNT_NAMES)

EXPORTED = ["faco_build_instance", "faco_run_iterations", "faco_get_best_tour",
            "faco_destroy_instance", "faco_last_error", "faco_run_batch",
            "faco_debug_get", "faco_footprint_bytes", "faco_set_timing",
            "faco_phase_times", "faco_set_batch_ants_per_block", "faco_set_team_waves",
            "faco_set_queue_lds_capacity", "faco_set_verify", "faco_run_batch_noalloc",
            "faco_set_batch_config", "faco_get_batch_config", "faco_autotune_batch",
            "faco_set_tour_segments", "faco_set_stream"]


class faco_params(ctypes.Structure):
    _fields_ = [("cl_size", ctypes.c_int32), ("bl_size", ctypes.c_int32),
                ("n_ants", ctypes.c_int32), ("min_new_edges", ctypes.c_int32),
                ("rho", ctypes.c_float), ("reserved0", ctypes.c_float),
                ("p_best", ctypes.c_double), ("p_source_gbest", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("ls_flags", ctypes.c_uint32),
                ("oropt_max_seg", ctypes.c_int32), ("min_new_edges_max", ctypes.c_int32),
                ("reserved1", ctypes.c_int32)]


class faco_batch_config(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("team_waves", ctypes.c_int32),
                ("ants_per_block", ctypes.c_int32), ("queue_lds_capacity", ctypes.c_int32),
                ("big_percent", ctypes.c_int32), ("big_team_waves", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class FacoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"FACO error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libfaco_hip.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FacoError(FACO_EDEVICE, f"{LIB_PATH} is not built (run build())")
        # PyTorch brings its own HIP runtime; loading it first makes the
        # library bind to that same runtime, so torch streams and events and
        # the library's launches share one runtime in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER
        L.faco_build_instance.restype = ctypes.c_int
        L.faco_build_instance.argtypes = [P(ctypes.c_int32), ctypes.c_int32, P(faco_params),
                                          vp, P(vp)]
        L.faco_run_iterations.restype = ctypes.c_int
        L.faco_run_iterations.argtypes = [vp, ctypes.c_int32]
        L.faco_get_best_tour.restype = ctypes.c_int
        L.faco_get_best_tour.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int64)]
        L.faco_destroy_instance.restype = None
        L.faco_destroy_instance.argtypes = [vp]
        L.faco_set_stream.restype = ctypes.c_int
        L.faco_set_stream.argtypes = [vp, vp]
        L.faco_last_error.restype = ctypes.c_char_p
        L.faco_last_error.argtypes = [vp]
        L.faco_run_batch.restype = ctypes.c_int
        L.faco_run_batch.argtypes = [P(vp), ctypes.c_int32, ctypes.c_int32, vp]
        L.faco_set_batch_config.restype = ctypes.c_int
        L.faco_set_batch_config.argtypes = [P(faco_batch_config)]
        L.faco_get_batch_config.restype = ctypes.c_int
        L.faco_get_batch_config.argtypes = [P(faco_batch_config)]
        L.faco_autotune_batch.restype = ctypes.c_int
        L.faco_autotune_batch.argtypes = [P(vp), ctypes.c_int32, ctypes.c_int32, vp,
                                          P(faco_batch_config)]
        L.faco_run_batch_noalloc.restype = ctypes.c_int
        L.faco_run_batch_noalloc.argtypes = [P(vp), ctypes.c_int32, ctypes.c_int32, vp]
        L.faco_debug_get.restype = ctypes.c_int
        L.faco_debug_get.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_size_t]
        L.faco_footprint_bytes.restype = ctypes.c_uint64
        L.faco_footprint_bytes.argtypes = [ctypes.c_int32, P(faco_params)]
        L.faco_set_timing.restype = ctypes.c_int
        L.faco_set_timing.argtypes = [vp, ctypes.c_int32]
        L.faco_set_batch_ants_per_block.restype = ctypes.c_int
        L.faco_set_batch_ants_per_block.argtypes = [ctypes.c_int32]
        L.faco_set_team_waves.restype = ctypes.c_int
        L.faco_set_team_waves.argtypes = [ctypes.c_int32]
        L.faco_set_queue_lds_capacity.restype = ctypes.c_int
        L.faco_set_queue_lds_capacity.argtypes = [ctypes.c_int32]
        L.faco_set_tour_segments.restype = ctypes.c_int
        L.faco_set_tour_segments.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.faco_set_verify.restype = ctypes.c_int
        L.faco_set_verify.argtypes = [vp, ctypes.c_int32]
        L.faco_phase_times.restype = ctypes.c_int
        L.faco_phase_times.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
        _lib = L
    return _lib


def make_params(cl_size=16, bl_size=64, n_ants=16, min_new_edges=8, rho=0.5,
                p_best=0.05, p_source_gbest=0.01, seed=1,
                ls_flags=FACO_LS_2OPT | FACO_LS_OROPT | FACO_LS_SWEEP,
                oropt_max_seg=3, min_new_edges_max=0):
    return faco_params(cl_size, bl_size, n_ants, min_new_edges, rho, 0.0, p_best,
                       p_source_gbest, seed, ls_flags, oropt_max_seg, min_new_edges_max, 0)


def _check(rc, h=None):
    if rc != FACO_OK:
        msg = lib().faco_last_error(h)
        raise FacoError(rc, msg.decode() if msg else "")


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class Instance:
    """Handle returned by faco_build_instance."""

    def __init__(self, h, n, params):
        self.h = h
        self.n = n
        self.params = params
        info = faco_debug_get(self, FACO_DBG_INFO)
        self.k, self.bl = int(info[1]), int(info[2])
        self.A = params.n_ants

    def close(self):
        if self.h:
            faco_destroy_instance(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def faco_build_instance(xy, params=None, stream=None, **kw):
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    p = params if params is not None else make_params(**kw)
    out = ctypes.c_void_p()
    rc = lib().faco_build_instance(xy.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   xy.shape[0], ctypes.byref(p), _stream_handle(stream),
                                   ctypes.byref(out))
    _check(rc)
    return Instance(out.value, xy.shape[0], p)


def faco_run_iterations(inst, iterations):
    _check(lib().faco_run_iterations(inst.h, int(iterations)), inst.h)


def faco_get_best_tour(inst):
    tour = np.zeros(inst.n, dtype=np.int32)
    L = ctypes.c_int64()
    _check(lib().faco_get_best_tour(inst.h, tour.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    ctypes.byref(L)), inst.h)
    return tour, int(L.value)


def faco_destroy_instance(inst):
    if inst.h:
        lib().faco_destroy_instance(inst.h)
        inst.h = None


def faco_set_stream(inst, stream):
    """Later calls on the handle run on `stream`, after its queued work."""
    if inst.h is None:
        raise FacoError(FACO_EINVAL, "handle is closed")
    _check(lib().faco_set_stream(inst.h, _stream_handle(stream)), inst.h)


def faco_run_batch(insts, iterations, stream=None):
    arr = (ctypes.c_void_p * len(insts))(*[i.h for i in insts])
    rc = lib().faco_run_batch(arr, len(insts), int(iterations), _stream_handle(stream))
    _check(rc)


def faco_run_batch_noalloc(insts, iterations, stream=None):
    """faco_run_batch without device allocation (fixed tables; every handle
    built on `stream`)."""
    arr = (ctypes.c_void_p * len(insts))(*[i.h for i in insts])
    rc = lib().faco_run_batch_noalloc(arr, len(insts), int(iterations), _stream_handle(stream))
    _check(rc)


def faco_set_batch_config(persistent=0, team_waves=0, ants_per_block=1,
                          queue_lds_capacity=0, big_percent=0, big_team_waves=0):
    c = faco_batch_config(persistent, team_waves, ants_per_block, queue_lds_capacity,
                          big_percent, big_team_waves)
    _check(lib().faco_set_batch_config(ctypes.byref(c)))


def faco_get_batch_config():
    c = faco_batch_config()
    _check(lib().faco_get_batch_config(ctypes.byref(c)))
    return c.as_dict()


def faco_autotune_batch(insts, trial_iterations=5, stream=None):
    """Time the candidate batch configurations on twins of `insts`, store
    the fastest for their size class and return it (a dict)."""
    arr = (ctypes.c_void_p * len(insts))(*[i.h for i in insts])
    c = faco_batch_config()
    rc = lib().faco_autotune_batch(arr, len(insts), int(trial_iterations),
                                   _stream_handle(stream), ctypes.byref(c))
    _check(rc)
    return c.as_dict()


def faco_set_batch_ants_per_block(apb):
    _check(lib().faco_set_batch_ants_per_block(int(apb)))


def faco_set_queue_lds_capacity(cap):
    """LDS capacity of each ant's work queue for instances built afterwards
    (0 = default)."""
    _check(lib().faco_set_queue_lds_capacity(int(cap)))


def faco_set_tour_segments(mode, length_log2=0, max_records=0):
    """Tour representation of the local search for instances built afterwards:
    mode 0 by size, 1 flat arrays, 2 segment lists; segment length
    2**length_log2 (0: by size); record limit (0: 2048)."""
    _check(lib().faco_set_tour_segments(int(mode), int(length_log2), int(max_records)))


def faco_set_team_waves(tw):
    """Waves per ant for instances built afterwards (0 = by size; 1, 4, 8)."""
    _check(lib().faco_set_team_waves(int(tw)))


def faco_footprint_bytes(n, params=None, **kw):
    p = params if params is not None else make_params(**kw)
    return int(lib().faco_footprint_bytes(int(n), ctypes.byref(p)))


def faco_set_timing(inst, enable=True, reserve_iterations=0):
    """Phase timing on/off; reserve_iterations > 1 creates that many
    iterations' events up front."""
    v = (max(2, int(reserve_iterations)) if reserve_iterations else 1) if enable else 0
    _check(lib().faco_set_timing(inst.h, v), inst.h)


def faco_set_verify(inst, enable=True):
    """Recompute and check every tour length in each later iteration."""
    _check(lib().faco_set_verify(inst.h, 1 if enable else 0), inst.h)


def faco_phase_times(inst):
    ms = (ctypes.c_double * 4)()
    cnt = (ctypes.c_int64 * 4)()
    _check(lib().faco_phase_times(inst.h, ms, cnt), inst.h)
    return list(ms), list(cnt)


def faco_debug_get(inst, what):
    n, A = inst.n, inst.params.n_ants
    k = getattr(inst, "k", None)
    bl = getattr(inst, "bl", None)
    shapes = {
        FACO_DBG_ANT_ROUTES: (np.int32, (A, n)),
        FACO_DBG_ANT_LENGTHS: (np.int64, (A,)),
        FACO_DBG_PHEROMONE: (np.float32, (n, k)),
        FACO_DBG_SOURCE: (np.int32, (n,)),
        FACO_DBG_LIMITS: (np.float32, (3,)),
        FACO_DBG_COUNTERS: (np.int64, (A, FACO_NCNT)),
        FACO_DBG_CAND_LISTS: (np.int32, (n, k)),
        FACO_DBG_BACKUP_LISTS: (np.int32, (n, bl)),
        FACO_DBG_HEURISTIC: (np.float32, (n, k)),
        FACO_DBG_INFO: (np.int64, (8,)),
        FACO_DBG_INIT_COUNTERS: (np.int64, (FACO_NCNT,)),
        FACO_DBG_COUNTER_TOTALS: (np.int64, (A, FACO_NCNT)),
        FACO_DBG_PHASE_TICKS: (np.int64, (A, FACO_NTICKS)),
        FACO_DBG_TEAM_WAVES: (np.int32, (1,)),
        FACO_DBG_FAULT: (np.int64, (4,)),
        FACO_DBG_RECOMPUTED_LENGTHS: (np.int64, (A + 1,)),
        FACO_DBG_TOUR: (np.int64, (3,)),
        FACO_DBG_INIT_TICKS: (np.int64, (FACO_NTICKS,)),
    }
    dt, shape = shapes[what]
    out = np.zeros(shape, dtype=dt)
    _check(lib().faco_debug_get(inst.h, int(what), out.ctypes.data_as(ctypes.c_void_p),
                                out.nbytes), inst.h)
    return out
