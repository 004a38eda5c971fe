"""Autotuner: picks the tile shape and round schedule of the single-query
grower, and the tile shape of the batched grower, by timing real grows on the
caller's data.  Every candidate must produce the same masks (compared by
SHA-256 of the read-out); a disagreement raises.  Results are cached as JSON
keyed by the problem shape, the device name and the library version.

Only orchestration lives here: every grow runs in libmf4d.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import _lib
from .grower import Grower

PLAIN_SPACE = [dict(tile_t=bt, schedule=s, admit=a)
               for bt in (4, 8, 16) for s in ("persistent", "launch") for a in ("tiles", "all")]
BATCHED_SPACE = [(8, 4, 4, 4), (8, 8, 8, 1), (16, 4, 4, 2), (4, 4, 4, 8), (8, 8, 4, 2),
                 (16, 8, 4, 1), (32, 4, 4, 1), (4, 8, 4, 4)]


def _torch():
    import torch
    return torch


def cache_path() -> str:
    return os.environ.get("MF4D_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mf4d", "tune.json"))


def _key(kind: str, inst: dict, Q: int = 0) -> str:
    torch = _torch()
    X, Y, Z = inst["dims"]
    ver = _lib.load_library().mf4d_version().decode()
    dev = torch.cuda.get_device_name(0)
    return f"{kind}:{X}x{Y}x{Z}x{inst['T']}:P{inst['P']}:Q{Q}:{dev}:{ver}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(key: str, value: dict):
    data = _load_cache()
    data[key] = value
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _time(fn, repeats: int) -> float:
    torch = _torch()
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)) * 1e3


def _load(g: Grower, inst: dict):
    torch = _torch()
    dev = torch.device("cuda:0")
    g.load_field(torch.from_numpy(inst["field"]).to(dev))
    if inst["P"]:
        g.load_particles(torch.from_numpy(inst["xyz"]).to(dev), torch.from_numpy(inst["attr"]).to(dev))


def tune_plain(inst: dict, repeats: int = 5, space=None, use_cache: bool = True, log=None) -> dict:
    """Best {tile_t, schedule, admit} for growing this instance; every
    candidate is checked to give identical masks."""
    key = _key("plain", inst)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit
    torch = _torch()
    space = space or PLAIN_SPACE
    X, Y, Z = inst["dims"]
    V = X * Y * Z * inst["T"]
    fm = torch.empty((V + 31) // 32, dtype=torch.int32, device="cuda:0")
    pm = torch.empty((inst["T"], max(inst["P"], 1)), dtype=torch.uint8, device="cuda:0")
    rows, ref = [], None
    for bt in sorted({c["tile_t"] for c in space}):
        g = Grower(device=0, tile_t=bt)
        try:
            _load(g, inst)
            g.set_criteria(*inst["crit"])
            g.set_seeds(inst["seeds"])
            for c in [c for c in space if c["tile_t"] == bt]:
                g.set_schedule(c["schedule"])
                g.set_admit_mode(c["admit"])

                def step():
                    g.grow()
                    g.read_field_mask(fm)
                    if inst["P"]:
                        g.read_particle_mask(pm)

                ms = _time(step, repeats)
                dig = _digest(fm.cpu().numpy(), pm.cpu().numpy() if inst["P"] else b"")
                if ref is None:
                    ref = dig
                elif dig != ref:
                    raise RuntimeError(f"autotune: candidate {c} changed the masks")
                rows.append(dict(c, ms=ms))
                if log:
                    log(f"plain {c}: {ms:.3f} ms")
        finally:
            g.close()
    best = min(rows, key=lambda r: r["ms"])
    out = dict(best=best, table=rows, digest=ref)
    _store_cache(key, out)
    return out


def tune_batched(inst: dict, crit, qseeds, repeats: int = 3, space=None, use_cache: bool = True,
                 log=None) -> dict:
    """Best batched tile (bx, by, bz, bt) for these queries; identical planes
    across candidates."""
    key = _key("batched", inst, Q=len(crit))
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit
    torch = _torch()
    space = space or BATCHED_SPACE
    X, Y, Z = inst["dims"]
    V = X * Y * Z * inst["T"]
    fp = torch.empty((V, 8), dtype=torch.int32, device="cuda:0")
    pp = torch.empty((inst["T"], inst["P"], 8), dtype=torch.int32, device="cuda:0") if inst["P"] else None
    rows, ref = [], None
    g = Grower(device=0)
    try:
        _load(g, inst)
        g.set_queries(crit, qseeds)
        for shape in space:
            g.set_batched_tile(*shape)
            ms = _time(lambda: g.grow_batched(fp, pp), repeats)
            dig = _digest(fp.cpu().numpy(), pp.cpu().numpy() if pp is not None else b"")
            if ref is None:
                ref = dig
            elif dig != ref:
                raise RuntimeError(f"autotune: batched tile {shape} changed the planes")
            rows.append(dict(tile=list(shape), ms=ms))
            if log:
                log(f"batched tile {shape}: {ms:.3f} ms")
    finally:
        g.close()
    best = min(rows, key=lambda r: r["ms"])
    out = dict(best=best, table=rows, digest=ref)
    _store_cache(key, out)
    return out
