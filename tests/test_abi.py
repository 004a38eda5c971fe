"""The C ABI library: it loads and exports every function include/mf4d.h
declares (no compute calls; this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1903_12294_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(mf4d_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_is_built():
    assert os.path.exists(_lib.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 15
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert _declared() == set(_lib.SIGNATURES)


def test_version_and_error_without_gpu():
    lib = _lib.load_library()
    assert lib.mf4d_version().startswith(b"mf4d")
    # NULL context arguments are rejected before any device call
    assert lib.mf4d_set_max_rounds(None, 1) == _lib.MF4D_ERR_ARG
    assert b"NULL" in lib.mf4d_last_error()
    assert lib.mf4d_grow(None, None) == _lib.MF4D_ERR_ARG


def test_missing_library_raises(tmp_path):
    with pytest.raises(_lib.LibraryMissing):
        _lib.load_library(str(tmp_path / "nope.so"))


def test_every_package_module_imports():
    import importlib
    import pkgutil

    import paper_1903_12294_amd as pkg
    for m in pkgutil.iter_modules(pkg.__path__):
        if m.name.startswith("lib"):  # the HIP shared library, not a Python module
            continue
        importlib.import_module(f"{pkg.__name__}.{m.name}")


# The boundary's calls by the names the design of the library gives them:
# context, inputs, criteria, seeds, queries, scheduler, round cap, reset, grow,
# read-outs, and the network's forward / backward / optimizer step.
BOUNDARY_CALLS = [
    "mf4d_create", "mf4d_destroy", "mf4d_last_error", "mf4d_load_field", "mf4d_load_particles",
    "mf4d_set_criteria", "mf4d_set_seeds", "mf4d_set_queries", "mf4d_set_scheduler",
    "mf4d_set_max_rounds", "mf4d_reset_labels", "mf4d_grow", "mf4d_read_field_mask",
    "mf4d_read_particle_mask", "mf4d_read_batched", "mf4d_nn_forward", "mf4d_nn_backward",
    "mf4d_nn_adam_step",
]


def test_boundary_calls_declared_and_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    declared = _declared()
    for name in BOUNDARY_CALLS:
        assert name in declared, name
        assert hasattr(lib, name), name


def test_every_declared_call_cites_or_explains():
    """Each declaration in the header is preceded by a comment block."""
    src = open(os.path.join(ROOT, "include", "mf4d.h")).read()
    body = src[src.index("extern \"C\" {"):]
    for name in sorted(_declared()):
        i = body.index(name + "(")
        before = body[:i].rstrip()
        # the nearest preceding comment block ends within a few lines
        end = before.rfind("*/")
        assert end >= 0 and before[end:].count("\n") <= 6, name


def test_new_calls_reject_null_without_gpu():
    lib = _lib.load_library()
    assert lib.mf4d_reset_labels(None) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_set_scheduler(None, 0, None, 0) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_read_batched(None, None, 0, None, 0, 0) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_nn_adam_step(None, None, ctypes.c_float(1e-3), 1) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_grow_read(None, None, 0, None, 0, None) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_set_read_async(None, 1) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_read_wait(None) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_grow_submit(None, None, 0, None, 0) == _lib.MF4D_ERR_ARG
    assert lib.mf4d_grow_finish(None, None) == _lib.MF4D_ERR_ARG
