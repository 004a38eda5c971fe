"""Loader for the hand-derived fixtures under tests/golden/."""
import glob
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _f(v):
    if isinstance(v, str):
        s = v.strip().lower()
        if s.startswith(("0x", "-0x")):
            return float.fromhex(s)
        return float(s)
    return float(v)


def _arr(x, shape):
    flat = np.array([_f(v) for v in np.asarray(x, dtype=object).ravel()], np.float64)
    return flat.astype(np.float32).reshape(shape)


def load(path):
    with open(path) as fh:
        d = json.load(fh)
    X, Y, Z = d["dims"]
    T, P = d["T"], d["P"]
    field = _arr(d["field"], (T, Z, Y, X))
    if P:
        xyz = _arr(d["xyz"], (T, P, 3))
        attr = _arr(d["attr"], (T, P))
    else:
        xyz = np.zeros((T, 0, 3), np.float32)
        attr = np.zeros((T, 0), np.float32)
    crit = np.array([_f(v) for v in d["crit"]], np.float32)
    seeds = np.asarray(d["seeds"], np.int32).reshape(-1, 4)
    e = d["expect"]
    Mf = np.zeros((T, Z, Y, X), bool)
    for x, y, z, t in e["field"]:
        Mf[t, z, y, x] = True
    Mp = np.zeros((T, P), bool)
    for i, t in e["particle"]:
        Mp[t, i] = True
    return dict(name=d["name"], cite=d["cite"], field=field, xyz=xyz, attr=attr, crit=crit,
                seeds=seeds, Mf=Mf, Mp=Mp, dropped=e["dropped"], depth=e["depth"])


def all_cases():
    return [load(p) for p in sorted(glob.glob(os.path.join(GOLDEN, "*.json")))]


def unpack_field(words, shape):
    n = int(np.prod(shape))
    bits = np.unpackbits(np.asarray(words, np.uint32).view(np.uint8), bitorder="little")
    return bits[:n].astype(bool).reshape(shape)
