"""ctypes binding of libmf4d.so (declared in include/mf4d.h).

Argument marshalling only: every step of the grower runs in the HIP library.
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int64, c_size_t, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmf4d.so")

MF4D_OK = 0
MF4D_ERR_ARG = -1
MF4D_ERR_RANGE = -2
MF4D_ERR_OOM = -3
MF4D_ERR_HIP = -4
MF4D_ERR_STATE = -5
MF4D_ERR_NOT_CONVERGED = -6
MF4D_ERR_UNSUPPORTED = -7
MF4D_HOST = 0
MF4D_DEVICE = 1
MF4D_ADMIT_TILES = 0
MF4D_ADMIT_ALL = 1
MF4D_TRAJ_BOTH = 0
MF4D_TRAJ_FORWARD = 1
MF4D_SCHED_PERSISTENT = 0
MF4D_SCHED_LAUNCH = 1
MF4D_SCHED_JACOBI = 2
MF4D_SCHEDULER_PLAIN = 0
MF4D_SCHEDULER_LEARNED = 1
MF4D_SCHEDULER_HEURISTIC = 2

ERROR_NAMES = {
    MF4D_ERR_ARG: "ARG", MF4D_ERR_RANGE: "RANGE", MF4D_ERR_OOM: "OOM", MF4D_ERR_HIP: "HIP",
    MF4D_ERR_STATE: "STATE", MF4D_ERR_NOT_CONVERGED: "NOT_CONVERGED",
    MF4D_ERR_UNSUPPORTED: "UNSUPPORTED",
}


# Library objects (contexts, networks) still open.  They are closed by an exit
# handler, before the interpreter shuts down: a HIP call made from a finaliser
# while the runtime itself is being torn down can crash the process after its
# work is done.
_open_handles = weakref.WeakSet()


def track(obj) -> None:
    """Register an object with a close() method to be closed at exit."""
    _open_handles.add(obj)


def finalizing() -> bool:
    return sys.is_finalizing()


@atexit.register
def _close_open_handles() -> None:
    for obj in list(_open_handles):
        try:
            obj.close()
        except Exception:
            pass


class Stats(ctypes.Structure):
    _fields_ = [
        ("rounds", c_int64),
        ("tile_visits", c_int64),
        ("particle_visits", c_int64),
        ("members_field", c_int64),
        ("members_particle", c_int64),
        ("seeds_dropped", c_int64),
        ("active_tiles", c_int64),
        ("ms_admit_field", c_double),
        ("ms_admit", c_double),
        ("ms_rounds", c_double),
        ("ms_total", c_double),
        ("tiles_tested", c_int64),
        ("tiles_deferred_read", c_int64),
        ("ms_sweep", c_double),
        ("ms_pull", c_double),
        ("ms_close", c_double),
        ("coupled_steps", c_int64),
        ("priority_visits", c_int64),
        ("verify_rounds", c_int64),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); mirrors include/mf4d.h
SIGNATURES = {
    "mf4d_version": (c_char_p, []),
    "mf4d_last_error": (c_char_p, []),
    "mf4d_device_bytes": (c_int64, []),
    "mf4d_create": (c_int, [POINTER(c_void_p), c_int, c_void_p]),
    "mf4d_destroy": (None, [c_void_p]),
    "mf4d_set_tile": (c_int, [c_void_p, c_int]),
    "mf4d_set_phase_timing": (c_int, [c_void_p, c_int]),
    "mf4d_load_field": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "mf4d_load_particles": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_int, c_int]),
    "mf4d_load_particles_rate": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_int, c_int, c_int]),
    "mf4d_set_criteria": (c_int, [c_void_p, c_float, c_float, c_float, c_float]),
    "mf4d_set_seeds": (c_int, [c_void_p, c_void_p, c_int64, c_int]),
    "mf4d_set_schedule": (c_int, [c_void_p, c_int]),
    "mf4d_set_admit_mode": (c_int, [c_void_p, c_int]),
    "mf4d_set_max_rounds": (c_int, [c_void_p, c_int64]),
    "mf4d_set_trajectory_mode": (c_int, [c_void_p, c_int]),
    "mf4d_grow": (c_int, [c_void_p, POINTER(Stats)]),
    "mf4d_grow_resume": (c_int, [c_void_p, POINTER(Stats)]),
    "mf4d_grow_read": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, POINTER(Stats)]),
    "mf4d_set_read_async": (c_int, [c_void_p, c_int]),
    "mf4d_read_wait": (c_int, [c_void_p]),
    "mf4d_grow_submit": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t]),
    "mf4d_grow_finish": (c_int, [c_void_p, POINTER(Stats)]),
    "mf4d_read_field_mask": (c_int, [c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_read_particle_mask": (c_int, [c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_read_particle_segments": (c_int, [c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_grow_seed_ids": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_int, c_void_p]),
    "mf4d_last_stats": (c_int, [c_void_p, POINTER(Stats)]),
    "mf4d_slic_set_params": (c_int, [c_void_p, c_void_p, c_float, c_float, c_float, c_float, c_double, c_int]),
    "mf4d_slic_run": (c_int, [c_void_p, c_void_p]),
    "mf4d_slic_read_labels": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_int]),
    "mf4d_slic_read_centres": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_slic_merge": (c_int, [c_void_p, c_double, c_void_p]),
    "mf4d_slic_read_features": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_slic_read_segments": (c_int, [c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_set_queries": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int64, c_int]),
    "mf4d_grow_batched": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_int,
                                  POINTER(Stats)]),
    "mf4d_set_batched_tile": (c_int, [c_void_p, c_int, c_int, c_int, c_int]),
    "mf4d_net_num_params": (c_int, []),
    "mf4d_net_create": (c_int, [POINTER(c_void_p), c_int, c_void_p]),
    "mf4d_net_destroy": (None, [c_void_p]),
    "mf4d_net_last_error": (c_char_p, []),
    "mf4d_net_set_params": (c_int, [c_void_p, c_void_p, c_int]),
    "mf4d_net_get_params": (c_int, [c_void_p, c_void_p, c_int]),
    "mf4d_net_forward": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_int]),
    "mf4d_net_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_float,
                              c_void_p, POINTER(c_float), c_int]),
    "mf4d_net_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                                    c_float, c_float, POINTER(c_float)]),
    "mf4d_brick_dims": (c_int, [c_void_p, POINTER(c_int)]),
    "mf4d_features": (c_int, [c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_brick_labels": (c_int, [c_void_p, c_void_p, c_size_t, c_int]),
    "mf4d_set_predictor": (c_int, [c_void_p, c_void_p, c_float]),
    "mf4d_set_scheduler": (c_int, [c_void_p, c_int, c_void_p, c_size_t]),
    "mf4d_reset_labels": (c_int, [c_void_p]),
    "mf4d_read_batched": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_size_t, c_int]),
    "mf4d_nn_forward": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_int]),
    "mf4d_nn_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_float,
                                 c_void_p, c_void_p, c_void_p, c_int]),
    "mf4d_nn_adam_step": (c_int, [c_void_p, c_void_p, c_float, c_int]),
    "mf4d_nn_forward_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_int]),
}


class LibraryMissing(RuntimeError):
    pass


class MF4DError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"mf4d error {code} ({ERROR_NAMES.get(code, '?')}): {message}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Open libmf4d.so and declare every exported function.  Raises
    LibraryMissing when the library has not been built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} is not built; run paper_1903_12294_amd.build.build_library() first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(rc: int, lib=None) -> int:
    if rc != MF4D_OK:
        lib = lib or load_library()
        raise MF4DError(rc, (lib.mf4d_last_error() or b"").decode())
    return rc
