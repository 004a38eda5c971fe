"""ctypes wrapper of the C breadth-first oracle (grow_bfs.c).

TEST INFRASTRUCTURE ONLY (see the package docstring)."""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grow_bfs.c")
_LIB = os.path.join(_HERE, "liboracle_bfs.so")
_lib = None

ERRORS = {0: "ok", -1: "bad argument", -2: "seed out of range", -3: "out of memory"}


def build_oracle(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the C oracle with gcc (always recompiles)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, src, "-lm"],
                   check=True)
    os.replace(tmp, out)
    return out


def load(path: str = _LIB):
    global _lib
    if _lib is not None and path == _LIB:
        return _lib
    if not os.path.exists(path):
        build_oracle(out=path)
    lib = ctypes.CDLL(path)
    f = lib.oracle_grow
    f.restype = ctypes.c_int
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    flt = ctypes.c_float
    f.argtypes = [P, i64, i64, i64, i64, P, P, i64, flt, flt, flt, flt, P, i64, P, P, P]
    g = lib.oracle_grow_rate
    g.restype = ctypes.c_int
    g.argtypes = [P, i64, i64, i64, i64, P, P, i64, i64, i64, flt, flt, flt, flt, P, i64, ctypes.c_int,
                  P, P, P]
    if path == _LIB:
        _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def oracle_grow(field: np.ndarray, xyz: np.ndarray | None, attr: np.ndarray | None,
                crit, seeds: np.ndarray, lib=None, forward_only: bool = False, rate: int = 1):
    """Grow from seeds.  field fp32 [T][Z][Y][X]; xyz fp32 [Tp][P][3];
    attr fp32 [Tp][P]; crit = (f_lo, f_hi, a_lo, a_hi); seeds int32 [S][4].
    forward_only: trajectory edges lead from t to t + 1 only (causal).
    rate: particle steps per field step (particle step tau couples with field
    step tau // rate); Tp <= rate * T, and Tp == T when rate is 1.
    Returns (field mask uint32 words, particle mask uint8 [Tp][P], stats dict)."""
    lib = lib or load()
    field = np.ascontiguousarray(field, np.float32)
    T, Z, Y, X = field.shape
    Tp = T if xyz is None else xyz.shape[0]
    if xyz is None or xyz.shape[1] == 0:
        P = 0
        xyz = attr = None
        pmask = np.zeros((Tp, 0), np.uint8)
    else:
        xyz = np.ascontiguousarray(xyz, np.float32)
        attr = np.ascontiguousarray(attr, np.float32)
        P = xyz.shape[1]
        assert xyz.shape == (Tp, P, 3) and attr.shape == (Tp, P)
        pmask = np.zeros((Tp, P), np.uint8)
    seeds = np.ascontiguousarray(np.asarray(seeds, np.int32).reshape(-1, 4))
    V = X * Y * Z * T
    fmask = np.zeros((V + 31) // 32, np.uint32)
    stats = np.zeros(5, np.int64)
    c = [float(np.float32(v)) for v in crit]
    rc = lib.oracle_grow_rate(_ptr(field), X, Y, Z, T, _ptr(xyz), _ptr(attr), P, Tp, int(rate),
                              c[0], c[1], c[2], c[3], _ptr(seeds), len(seeds), int(bool(forward_only)),
                              _ptr(fmask), _ptr(pmask) if P else None, _ptr(stats))
    if rc != 0:
        raise OracleError(rc, ERRORS.get(rc, str(rc)))
    st = dict(members_field=int(stats[0]), members_particle=int(stats[1]),
              seeds_dropped=int(stats[2]), depth=int(stats[3]), seeds_kept=int(stats[4]))
    return fmask, pmask, st


def oracle_grow_queries(field, xyz, attr, crit_q: np.ndarray, qseeds: np.ndarray,
                        queries=None, threads: int | None = None, forward_only: bool = False,
                        rate: int = 1):
    """One independent oracle grow per query (thread pool over queries).
    crit_q fp32 [Q][4]; qseeds int32 [S][5] = (x, y, z, t, q).
    Returns {q: (fmask, pmask, stats)} for the requested queries."""
    Q = len(crit_q)
    qs = range(Q) if queries is None else queries
    lib = load()

    def one(q):
        s = qseeds[qseeds[:, 4] == q][:, :4]
        return q, oracle_grow(field, xyz, attr, crit_q[q], s, lib=lib, forward_only=forward_only, rate=rate)

    with ThreadPoolExecutor(threads or max(1, min(16, os.cpu_count() or 1))) as ex:
        return dict(ex.map(one, qs))


def oracle_seed_ids(field, xyz, attr, crit, seeds, forward_only: bool = False, rate: int = 1):
    """Per-seed component ids: every node gets the index of the lowest seed
    whose own grown region (a grow from that seed alone) holds it, -1 where no
    seed reaches.  Returns (field ids int32 [T][Z][Y][X], particle ids int32
    [T][P]).  One oracle grow per seed, in index order."""
    field = np.ascontiguousarray(field, np.float32)
    T, Z, Y, X = field.shape
    P = 0 if xyz is None else xyz.shape[1]
    Tp = T if xyz is None else xyz.shape[0]
    fid = np.full(field.size, -1, np.int32)
    pid = np.full((Tp, P), -1, np.int32)
    seeds = np.asarray(seeds, np.int32).reshape(-1, 4)
    for i, s in enumerate(seeds):
        fm, pm, _ = oracle_grow(field, xyz, attr, crit, s[None], forward_only=forward_only, rate=rate)
        bits = np.unpackbits(fm.view(np.uint8), bitorder="little")[:field.size].astype(bool)
        fid[bits & (fid < 0)] = i
        if P:
            pid[(pm != 0) & (pid < 0)] = i
    return fid.reshape(T, Z, Y, X), pid


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code
