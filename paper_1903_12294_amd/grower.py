"""Thin Python wrapper of the mf4d C ABI: one object per library context.

Arrays are numpy arrays (host memory, MF4D_HOST) or torch tensors on the GPU
(device memory, MF4D_DEVICE).  Torch supplies device memory and the stream;
the library does all of the work.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import MF4D_DEVICE, MF4D_HOST, MF4DError, Stats  # noqa: F401


def _torch():
    import torch
    return torch


def _is_device_tensor(a) -> bool:
    return hasattr(a, "is_cuda") and a.is_cuda


def _arg(a, dtype):
    """(pointer, where, keep-alive) for a numpy array or a device tensor."""
    if _is_device_tensor(a):
        torch = _torch()
        want = {np.float32: torch.float32, np.int32: torch.int32, np.uint32: torch.int32,
                np.uint8: torch.uint8}[dtype]
        if a.dtype != want and not (dtype is np.uint32 and a.dtype in (torch.int32,)):
            raise TypeError(f"tensor dtype {a.dtype}, expected {want}")
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), MF4D_DEVICE, a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(ctypes.c_void_p), MF4D_HOST, arr


class Grower:
    """A library context on one GPU, ordering its work on one HIP stream."""

    def __init__(self, device: int = 0, stream=None, tile_t: int | None = None,
                 schedule: str | None = None, admit: str | None = None):
        self.lib = _lib.load_library()
        if stream is None:
            torch = _torch()
            stream = torch.cuda.current_stream(device).cuda_stream
        self.ctx = ctypes.c_void_p()
        self._check(self.lib.mf4d_create(ctypes.byref(self.ctx), device, ctypes.c_void_p(stream)))
        _lib.track(self)
        self.device = device
        self.dims = None
        self.T = None
        self.Tp = None  # particle steps (the field's T unless loaded at another rate)
        self.P = 0
        if tile_t is not None:
            self._check(self.lib.mf4d_set_tile(self.ctx, tile_t))
        if schedule is not None:
            self.set_schedule(schedule)
        if admit is not None:
            self.set_admit_mode(admit)

    def _check(self, rc):
        return _lib.check(rc, self.lib)

    def close(self):
        if self.ctx:
            self.lib.mf4d_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        # at interpreter shutdown the exit handler has closed every context;
        # make no HIP call from a finaliser then
        if _lib.finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- inputs -----------------------------------------------------------
    def load_field(self, field):
        T, Z, Y, X = field.shape
        p, where, keep = _arg(field, np.float32)
        self._check(self.lib.mf4d_load_field(self.ctx, p, X, Y, Z, T, where))
        self.dims, self.T, self.P, self.Tp = (X, Y, Z), T, 0, T
        del keep

    def load_particles(self, xyz, attr, rate: int = 1):
        """xyz [Tp][P][3], attr [Tp][P]; rate = particle steps per field step
        (step tau couples with field step tau // rate; Tp == T when rate is
        1)."""
        T, P = attr.shape[0], attr.shape[1]
        if tuple(xyz.shape) != (T, P, 3):
            raise ValueError("xyz must be [T][P][3] matching attr [T][P]")
        px, wx, kx = _arg(xyz, np.float32)
        pa, wa, ka = _arg(attr, np.float32)
        if wx != wa:
            raise ValueError("xyz and attr must both live on the host or both on the device")
        if rate == 1:
            self._check(self.lib.mf4d_load_particles(self.ctx, px, pa, P, T, wx))
        else:
            self._check(self.lib.mf4d_load_particles_rate(self.ctx, px, pa, P, T, int(rate), wx))
        self.P = P
        self.Tp = T if P else self.T
        del kx, ka

    def set_criteria(self, f_lo, f_hi=np.inf, a_lo=-np.inf, a_hi=np.inf):
        self._check(self.lib.mf4d_set_criteria(self.ctx, float(np.float32(f_lo)),
                                               float(np.float32(f_hi)), float(np.float32(a_lo)),
                                               float(np.float32(a_hi))))

    def set_seeds(self, seeds):
        n = int(seeds.shape[0]) if len(seeds.shape) else 0
        p, where, keep = _arg(seeds, np.int32)
        self._check(self.lib.mf4d_set_seeds(self.ctx, p, n, where))
        del keep

    def set_schedule(self, mode):
        """"persistent" (one cooperative kernel), "launch" (launches per round)
        or "jacobi" (debugging: synchronous sweeps, one edge per sweep)."""
        m = {"persistent": _lib.MF4D_SCHED_PERSISTENT, "launch": _lib.MF4D_SCHED_LAUNCH,
             "jacobi": _lib.MF4D_SCHED_JACOBI}[mode]
        self._check(self.lib.mf4d_set_schedule(self.ctx, m))

    def set_admit_mode(self, mode):
        """"tiles" (only tiles whose value range meets the band) or "all"."""
        m = {"tiles": _lib.MF4D_ADMIT_TILES, "all": _lib.MF4D_ADMIT_ALL}[mode]
        self._check(self.lib.mf4d_set_admit_mode(self.ctx, m))

    def set_trajectory_mode(self, mode):
        """"both" (membership spreads both ways along a trajectory) or
        "forward" (causal: from t to t + 1 only)."""
        m = {"both": _lib.MF4D_TRAJ_BOTH, "forward": _lib.MF4D_TRAJ_FORWARD}[mode]
        self._check(self.lib.mf4d_set_trajectory_mode(self.ctx, m))

    def set_phase_timing(self, on: bool):
        """Device times of each launched round's kernels in the stats (costs a
        few microseconds per event; off by default)."""
        self._check(self.lib.mf4d_set_phase_timing(self.ctx, 1 if on else 0))

    def set_max_rounds(self, cap: int):
        self._check(self.lib.mf4d_set_max_rounds(self.ctx, int(cap)))

    # -- growth -----------------------------------------------------------
    def grow(self) -> dict:
        st = Stats()
        self._check(self.lib.mf4d_grow(self.ctx, ctypes.byref(st)))
        return st.as_dict()

    def grow_read(self, field_out=None, particle_out=None, stats: bool = True):
        """grow() and the read-out of both masks in one call, the read-outs
        queued on the device behind the rounds: field_out (int32 device
        tensor of field_words() words) and particle_out (uint8 device tensor
        of T*P bytes), either None to skip.  Statistics as grow() (None with
        stats=False; stats() still returns them)."""
        for a in (field_out, particle_out):
            if a is not None and not _is_device_tensor(a):
                raise ValueError("grow_read writes device tensors only")
        fp = ctypes.c_void_p(field_out.data_ptr()) if field_out is not None else None
        pp = ctypes.c_void_p(particle_out.data_ptr()) if particle_out is not None else None
        st = Stats() if stats else None
        self._check(self.lib.mf4d_grow_read(self.ctx, fp, field_out.numel() if field_out is not None else 0,
                                            pp, particle_out.numel() if particle_out is not None else 0,
                                            ctypes.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def grow_submit(self, field_out=None, particle_out=None):
        """Queue grow_read's work and return without waiting for the device;
        grow_finish() returns its statistics.  The output tensors must stay
        untouched until then."""
        for a in (field_out, particle_out):
            if a is not None and not _is_device_tensor(a):
                raise ValueError("grow_submit writes device tensors only")
        fp = ctypes.c_void_p(field_out.data_ptr()) if field_out is not None else None
        pp = ctypes.c_void_p(particle_out.data_ptr()) if particle_out is not None else None
        self._check(self.lib.mf4d_grow_submit(self.ctx, fp, field_out.numel() if field_out is not None else 0,
                                              pp, particle_out.numel() if particle_out is not None else 0))

    def grow_finish(self) -> dict:
        """Complete the submitted grow (more rounds if it needs them) and
        return its statistics, as grow_read would."""
        st = Stats()
        self._check(self.lib.mf4d_grow_finish(self.ctx, ctypes.byref(st)))
        return st.as_dict()

    def set_read_async(self, on: bool):
        """grow_read leaves its read-outs deferred: the next grow_read
        issues them beside its own rounds (two label sets); read_wait() or
        any other call issues what is deferred and orders the context stream
        after them."""
        self._check(self.lib.mf4d_set_read_async(self.ctx, 1 if on else 0))

    def read_wait(self):
        """Issue deferred read-outs and order the context stream after them."""
        self._check(self.lib.mf4d_read_wait(self.ctx))

    def grow_resume(self) -> dict:
        st = Stats()
        self._check(self.lib.mf4d_grow_resume(self.ctx, ctypes.byref(st)))
        return st.as_dict()

    def stats(self) -> dict:
        st = Stats()
        self._check(self.lib.mf4d_last_stats(self.ctx, ctypes.byref(st)))
        return st.as_dict()

    # -- outputs ----------------------------------------------------------
    def field_words(self) -> int:
        X, Y, Z = self.dims
        return (X * Y * Z * self.T + 31) // 32

    def read_field_mask(self, out=None):
        """uint32 canonical bit words.  `out` may be a device tensor (int32)."""
        n = self.field_words()
        if out is None:
            out = np.zeros(n, np.uint32)
        if _is_device_tensor(out):
            if out.numel() < n:
                raise ValueError("out too small")
            self._check(self.lib.mf4d_read_field_mask(self.ctx, ctypes.c_void_p(out.data_ptr()),
                                                      out.numel(), MF4D_DEVICE))
        else:
            self._check(self.lib.mf4d_read_field_mask(
                self.ctx, out.ctypes.data_as(ctypes.c_void_p), out.size, MF4D_HOST))
        return out

    def read_particle_mask(self, out=None):
        """uint8 [T][P].  `out` may be a device tensor (uint8)."""
        n = self.Tp * self.P
        if out is None:
            out = np.zeros((self.Tp, self.P), np.uint8)
        if _is_device_tensor(out):
            self._check(self.lib.mf4d_read_particle_mask(
                self.ctx, ctypes.c_void_p(out.data_ptr()), out.numel(), MF4D_DEVICE))
        else:
            self._check(self.lib.mf4d_read_particle_mask(
                self.ctx, out.ctypes.data_as(ctypes.c_void_p), n, MF4D_HOST))
        return out

    def read_particle_segments(self, out=None):
        """Trajectory segments of the grown feature (Section 3.4): uint8
        [T][P], members with a member neighbour step.  `out` may be a device
        tensor (uint8)."""
        n = self.Tp * self.P
        if out is None:
            out = np.zeros((self.Tp, self.P), np.uint8)
        if _is_device_tensor(out):
            self._check(self.lib.mf4d_read_particle_segments(
                self.ctx, ctypes.c_void_p(out.data_ptr()), out.numel(), MF4D_DEVICE))
        else:
            self._check(self.lib.mf4d_read_particle_segments(
                self.ctx, out.ctypes.data_as(ctypes.c_void_p), n, MF4D_HOST))
        return out

    def grow_seed_ids(self, field_out=None, particle_out=None):
        """Per-seed component ids: (field int32 [T][Z][Y][X], particle int32
        [T][P], number of grows run); each grown node carries the lowest seed
        index whose own region holds it, others -1.  Outputs may be device
        tensors (int32) or numpy arrays; the context holds no grown labels
        afterwards."""
        X, Y, Z = self.dims
        T, P = self.T, self.P
        if field_out is None:
            field_out = np.zeros((T, Z, Y, X), np.int32)
        if particle_out is None:
            particle_out = np.zeros((self.Tp, P), np.int32)
        dev = _is_device_tensor(field_out)
        if dev != _is_device_tensor(particle_out):
            raise ValueError("both outputs on the device or both on the host")

        def ptr(a):
            return ctypes.c_void_p(a.data_ptr()) if dev else a.ctypes.data_as(ctypes.c_void_p)
        n_f = field_out.numel() if dev else field_out.size
        n_p = particle_out.numel() if dev else particle_out.size
        grows = ctypes.c_int64(0)
        self._check(self.lib.mf4d_grow_seed_ids(self.ctx, ptr(field_out), n_f,
                                                ptr(particle_out) if n_p else None, n_p,
                                                MF4D_DEVICE if dev else MF4D_HOST, ctypes.byref(grows)))
        return field_out, particle_out, int(grows.value)

    # -- 4D SLIC clustering (Section 3.2) ------------------------------------
    def slic_set_params(self, k, w_d: float, w_f: float, w_p: float, c_f: float, eps: float,
                        max_iter: int):
        """k = (kx, ky, kz, kt) centres per axis; distance weights and the
        time-to-space factor of Sections 3.2.1 and 3.2.3; relative-change
        threshold and iteration cap of Section 3.2.2."""
        k4 = (ctypes.c_int * 4)(*[int(v) for v in k])
        self._check(self.lib.mf4d_slic_set_params(self.ctx, k4, float(w_d), float(w_f), float(w_p),
                                                  float(c_f), float(eps), int(max_iter)))
        self.slic_K = int(k[0]) * int(k[1]) * int(k[2]) * int(k[3])

    def slic_run(self) -> int:
        """Cluster the loaded samples; returns the number of assignment passes."""
        it = ctypes.c_int(0)
        self._check(self.lib.mf4d_slic_run(self.ctx, ctypes.byref(it)))
        return int(it.value)

    def slic_read_labels(self, field_out=None, point_out=None):
        """(field int32 [T][Z][Y][X], point int32 [T][P]); outputs may be
        device tensors (int32) or numpy arrays."""
        X, Y, Z = self.dims
        T, P = self.T, self.P
        if field_out is None:
            field_out = np.zeros((T, Z, Y, X), np.int32)
        if point_out is None:
            point_out = np.zeros((self.Tp, P), np.int32)
        dev = _is_device_tensor(field_out)
        if dev != _is_device_tensor(point_out):
            raise ValueError("both outputs on the device or both on the host")

        def ptr(a):
            return ctypes.c_void_p(a.data_ptr()) if dev else a.ctypes.data_as(ctypes.c_void_p)
        n_f = field_out.numel() if dev else field_out.size
        n_p = point_out.numel() if dev else point_out.size
        self._check(self.lib.mf4d_slic_read_labels(self.ctx, ptr(field_out), n_f,
                                                   ptr(point_out) if n_p else None, n_p,
                                                   MF4D_DEVICE if dev else MF4D_HOST))
        return field_out, point_out

    def slic_read_centres(self):
        """(centres fp64 [K][6] as x, y, z, t, p_c, f_c; counts int64 [K][2])."""
        K = self.slic_K
        cen = np.zeros((K, 6), np.float64)
        cnt = np.zeros((K, 2), np.int64)
        self._check(self.lib.mf4d_slic_read_centres(self.ctx, cen.ctypes.data_as(ctypes.c_void_p),
                                                    cnt.ctypes.data_as(ctypes.c_void_p), K, MF4D_HOST))
        return cen, cnt

    def slic_merge(self, eps_m: float) -> int:
        """Merge the last run's centres into features (Section 3.3); returns
        the number of features."""
        n = ctypes.c_int(0)
        self._check(self.lib.mf4d_slic_merge(self.ctx, float(eps_m), ctypes.byref(n)))
        return int(n.value)

    def slic_read_features(self):
        """(feature id of each centre int32 [K], per feature id fp64 [K][14]:
        n_f, n_p, mean f, mean p, std f, std p, x/y/z/t min and max)."""
        K = self.slic_K
        feat = np.zeros(K, np.int32)
        st = np.zeros((K, 14), np.float64)
        self._check(self.lib.mf4d_slic_read_features(self.ctx, feat.ctypes.data_as(ctypes.c_void_p),
                                                     st.ctypes.data_as(ctypes.c_void_p), K, MF4D_HOST))
        return feat, st

    def slic_read_segments(self, out=None):
        """Trajectory segments of the merged features (Section 3.4): int32
        [T][P], the feature id where the particle keeps it at a neighbouring
        step, else -1.  `out` may be a device tensor (int32)."""
        n = self.Tp * self.P
        if out is None:
            out = np.zeros((self.Tp, self.P), np.int32)
        if _is_device_tensor(out):
            self._check(self.lib.mf4d_slic_read_segments(
                self.ctx, ctypes.c_void_p(out.data_ptr()), out.numel(), MF4D_DEVICE))
        else:
            self._check(self.lib.mf4d_slic_read_segments(
                self.ctx, out.ctypes.data_as(ctypes.c_void_p), n, MF4D_HOST))
        return out

    # -- batched queries ----------------------------------------------------
    def set_queries(self, crit, seeds):
        """crit fp32 [Q][4] = (f_lo, f_hi, a_lo, a_hi); seeds int32 [S][5] = (x, y, z, t, q)."""
        crit = np.ascontiguousarray(crit, np.float32)
        seeds = np.ascontiguousarray(seeds, np.int32).reshape(-1, 5)
        self._check(self.lib.mf4d_set_queries(self.ctx, crit.shape[0],
                                              crit.ctypes.data_as(ctypes.c_void_p),
                                              seeds.ctypes.data_as(ctypes.c_void_p),
                                              seeds.shape[0], MF4D_HOST))
        self.Q = crit.shape[0]

    def set_batched_tile(self, bx: int, by: int, bz: int, bt: int):
        self._check(self.lib.mf4d_set_batched_tile(self.ctx, bx, by, bz, bt))

    def grow_batched(self, fplanes=None, pplanes=None) -> tuple:
        """Grow all queries.  Outputs are device tensors (int32, grown in place)
        or, when None, numpy arrays: fplanes [V][8], pplanes [T][P][8] uint32."""
        X, Y, Z = self.dims
        V = X * Y * Z * self.T
        st = Stats()
        if fplanes is None:
            fplanes = np.zeros((V, 8), np.uint32)
            pplanes = np.zeros((self.Tp, self.P, 8), np.uint32)
            self._check(self.lib.mf4d_grow_batched(
                self.ctx, fplanes.ctypes.data_as(ctypes.c_void_p), fplanes.size,
                pplanes.ctypes.data_as(ctypes.c_void_p) if self.P else None, pplanes.size,
                MF4D_HOST, ctypes.byref(st)))
        else:
            pp = ctypes.c_void_p(pplanes.data_ptr()) if pplanes is not None else None
            self._check(self.lib.mf4d_grow_batched(
                self.ctx, ctypes.c_void_p(fplanes.data_ptr()), fplanes.numel(), pp,
                0 if pplanes is None else pplanes.numel(), MF4D_DEVICE, ctypes.byref(st)))
        return fplanes, pplanes, st.as_dict()

    def grow_batched_owned(self) -> dict:
        """Grow all queries into planes the context owns (read them with
        read_batched)."""
        st = Stats()
        self._check(self.lib.mf4d_grow_batched(self.ctx, None, 0, None, 0, MF4D_DEVICE, ctypes.byref(st)))
        return st.as_dict()

    def read_batched(self, fplanes=None, pplanes=None) -> tuple:
        """The planes of the last grow_batched_owned: into device tensors
        (int32) or, when None, new numpy arrays [V][8] and [T][P][8] uint32."""
        X, Y, Z = self.dims
        V = X * Y * Z * self.T
        if fplanes is None:
            fplanes = np.zeros((V, 8), np.uint32)
            pplanes = np.zeros((self.Tp, self.P, 8), np.uint32)
            self._check(self.lib.mf4d_read_batched(
                self.ctx, fplanes.ctypes.data_as(ctypes.c_void_p), fplanes.size,
                pplanes.ctypes.data_as(ctypes.c_void_p) if self.P else None, pplanes.size, MF4D_HOST))
        else:
            pp = ctypes.c_void_p(pplanes.data_ptr()) if pplanes is not None else None
            self._check(self.lib.mf4d_read_batched(
                self.ctx, ctypes.c_void_p(fplanes.data_ptr()), fplanes.numel(), pp,
                0 if pplanes is None else pplanes.numel(), MF4D_DEVICE))
        return fplanes, pplanes

    def reset_labels(self):
        """Discard the grown feature (reads fail until the next grow)."""
        self._check(self.lib.mf4d_reset_labels(self.ctx))

    def set_scheduler(self, kind: str, params=None, logit_threshold: float = 0.0):
        """'plain'; 'heuristic' (candidate tiles visited first in descending
        order of their greatest field value, then a verification round); or
        'learned' with the predictor's fp32 parameters (the context keeps its
        own copy of the network): tiles scoring at least the threshold
        visited first in descending score, the others' admissibility deferred,
        then a verification round."""
        if kind in ("plain", "heuristic"):
            k = _lib.MF4D_SCHEDULER_PLAIN if kind == "plain" else _lib.MF4D_SCHEDULER_HEURISTIC
            self._check(self.lib.mf4d_set_scheduler(self.ctx, k, None, 0))
            return
        if kind != "learned":
            raise ValueError(f"unknown scheduler {kind!r}")
        buf = np.concatenate([np.asarray(params, np.float32).ravel(),
                              np.array([logit_threshold], np.float32)])
        self._check(self.lib.mf4d_set_scheduler(self.ctx, _lib.MF4D_SCHEDULER_LEARNED,
                                                buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))
