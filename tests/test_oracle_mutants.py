"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of the C oracle with one plausible slip (a dropped
edge, a wrong sign, a strict comparison, truncation instead of floor, a
periodic wrap, a skipped criterion).  It is compiled to a temporary library
and run against the hand-derived fixtures and the brute-force cross-checks;
every mutant must fail at least one of them.  The mistakes live only in the
temporary copies, on the CPU.  Some mistakes index out of bounds (an index
past the grid edge), so each mutant runs the battery in a child process; a
crash there also counts as the mistake being caught.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import bfs, components_grow, oracle_grow, reach_grow, sweep_grow
from tests import golden_io
from tests.test_oracle_pins import _random_instance

SRC = os.path.join(os.path.dirname(bfs.__file__), "grow_bfs.c")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHILD = ("import sys; from oracle import bfs; from tests.test_oracle_mutants import _battery; "
         "r = _battery(bfs.load(sys.argv[1])); print('CAUGHT ' + r if r else 'SURVIVED')")

MUTANTS = {
    "drop_plus_t_edge": ("if (t + 1 < (uint64_t)T) nb[k++] = v + XYZ;", ""),
    "drop_minus_y_edge": ("if (y > 0) nb[k++] = v - X;", ""),
    "wrong_sign_minus_z": ("if (z > 0) nb[k++] = v - XY;", "if (z > 0) nb[k++] = v + XY;"),
    "strict_lower_bound": ("return lo <= v && v <= hi;", "return lo < v && v <= hi;"),
    "strict_upper_bound": ("return lo <= v && v <= hi;", "return lo <= v && v < hi;"),
    "truncate_not_floor": ("float cx = floorf(p[0]),", "float cx = (float)(int)p[0],"),
    "periodic_x": ("if (x > 0) nb[k++] = v - 1;", "nb[k++] = x > 0 ? v - 1 : v + X - 1;"),
    "skip_particle_criterion": ("if (in_band(attr[q], a_lo, a_hi) && test_and_set(visP, q))",
                                "if (test_and_set(visP, q))"),
    "skip_field_check_on_bin": ("if (bin[q] != NO_VOXEL && in_band(field[bin[q]], f_lo, f_hi) &&",
                                "if (bin[q] != NO_VOXEL &&"),
    "drop_trajectory_back": ("if (!forward_only && t > 0 && in_band(attr[q - P], a_lo, a_hi) &&",
                             "if (0 &&"),
    "forward_only_ignored": ("if (!forward_only && t > 0 && in_band(attr[q - P], a_lo, a_hi) &&",
                             "if (t > 0 && in_band(attr[q - P], a_lo, a_hi) &&"),
    "forward_only_reversed": ("if (t + 1 < (uint64_t)Tp && in_band(attr[q + P], a_lo, a_hi) &&",
                              "if (!forward_only && t + 1 < (uint64_t)Tp && in_band(attr[q + P], a_lo, a_hi) &&"),
    "seed_unchecked": ("if (!in_band(field[v], f_lo, f_hi)) { dropped++; continue; }", ""),
    "upper_bin_inclusive": ("if (!(cx >= 0.0f && cx < (float)X)) return -1;",
                            "if (!(cx >= 0.0f && cx <= (float)X)) return -1;"),
    "transposed_xy_index": ("return ((int64_t)cz * Y + (int64_t)cy) * X + (int64_t)cx;",
                            "return ((int64_t)cz * Y + (int64_t)cx) * X + (int64_t)cy;"),
    "depth_counts_every_layer": ("if (fifo.tail > layer_end) depth++;", "depth++;"),
}


def _battery(lib):
    """Returns the name of the first pin that fails, or None."""
    for case in golden_io.all_cases():
        try:
            fm, pm, st_ = oracle_grow(case["field"], case["xyz"], case["attr"], case["crit"],
                                      case["seeds"], lib=lib)
        except Exception:
            return "golden:" + case["name"]
        if not (np.array_equal(golden_io.unpack_field(fm, case["field"].shape), case["Mf"])
                and np.array_equal(pm.astype(bool), case["Mp"])
                and st_["seeds_dropped"] == case["dropped"] and st_["depth"] == case["depth"]):
            return "golden:" + case["name"]
    rng = np.random.default_rng(12345)
    for _ in range(60):
        X, Y, Z, T = (int(v) for v in rng.integers(1, 6, 4))
        inst = _random_instance(rng, X, Y, Z, T, int(rng.integers(0, 30)), 3)
        fm, pm, st_ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                                  inst["seeds"], lib=lib)
        sf, sp_, sweeps, _ = sweep_grow(inst["field"], inst["xyz"], inst["attr"],
                                        inst["crit"], inst["seeds"])
        cf, cp = components_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                                 inst["seeds"])
        Mf = golden_io.unpack_field(fm, inst["field"].shape)
        if not (np.array_equal(Mf, sf) and np.array_equal(pm.astype(bool), sp_)
                and np.array_equal(Mf, cf) and sweeps == st_["depth"] + 1):
            return "random"
    # forward-only coupling against the directed sweeps and scipy reachability
    for _ in range(40):
        X, Y, Z, T = (int(v) for v in rng.integers(1, 6, 4))
        inst = _random_instance(rng, X, Y, Z, T, int(rng.integers(1, 30)), 3)
        args = (inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"])
        fm, pm, st_ = oracle_grow(*args, lib=lib, forward_only=True)
        sf, sp_, sweeps, _ = sweep_grow(*args, forward_only=True)
        rf, rp = reach_grow(*args, forward_only=True)
        Mf = golden_io.unpack_field(fm, inst["field"].shape)
        if not (np.array_equal(Mf, sf) and np.array_equal(pm.astype(bool), sp_)
                and np.array_equal(Mf, rf) and np.array_equal(sp_, rp) and sweeps == st_["depth"] + 1):
            return "random-forward"
    return None


def test_unmutated_passes_battery(oracle_lib):
    assert _battery(oracle_lib) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / f"lib{name}.so")
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, str(path), "-lm"],
                   check=True)
    res = subprocess.run([sys.executable, "-c", CHILD, so], cwd=ROOT, capture_output=True,
                         text=True, timeout=600)
    out = res.stdout.strip().splitlines()
    crashed = res.returncode < 0
    assert crashed or (res.returncode == 0 and out and out[-1].startswith("CAUGHT")), (
        f"mutant {name} survived every pin: rc={res.returncode} {res.stdout[-300:]} {res.stderr[-300:]}")
