"""Benchmark: voxel-timesteps segmented per second to the fixed point on one GPU.

One step = one pass of the whole hot path over resident inputs: admissibility
of every field and particle sample, seeding, rounds of tile sweeps and
particle coupling until nothing changes, and the read-out of the uint32 field
mask and the uint8 particle-step mask into device buffers.

Prints one JSON line (stdout).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def field_kernel_bytes(V: int) -> int:
    """Algorithmic bytes of one field-admissibility launch: read every fp32
    sample once, write one bit per voxel-step."""
    return 4 * V + V // 8


def grow_model_bytes(V: int, Q: int) -> int:
    """Algorithmic bytes of one eager grow: read field (4 B) and particle values
    (4 B) once, write admissibility bits, write both output masks."""
    return 4 * V + 4 * Q + V // 8 + Q // 8 + V // 8 + Q


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3])
    ap.add_argument("--tile-t", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the grower runs on a single MI355X; see DESIGN.md for how it would shard)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_12294_amd import Grower, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = synth.CONFIGS[args.config]
    t0 = time.time()
    inst = synth.make_config(args.config)
    log(f"[bench] generated {cfg['name']} in {time.time() - t0:.1f}s")
    X, Y, Z = inst["dims"]
    T, P = inst["T"], inst["P"]
    V, Q = X * Y * Z * T, P * T

    g = Grower(device=0, tile_t=args.tile_t)
    t0 = time.time()
    f_d = torch.from_numpy(inst["field"]).to(dev)
    g.load_field(f_d)
    del f_d
    xyz_d = torch.from_numpy(inst["xyz"]).to(dev)
    at_d = torch.from_numpy(inst["attr"]).to(dev)
    g.load_particles(xyz_d, at_d)
    del xyz_d, at_d
    g.set_criteria(*inst["crit"])
    g.set_seeds(inst["seeds"])
    torch.cuda.synchronize()
    log(f"[bench] loaded and binned in {time.time() - t0:.1f}s")

    fmask = torch.empty((V + 31) // 32, dtype=torch.int32, device=dev)
    pmask = torch.empty((T, P), dtype=torch.uint8, device=dev)

    def step():
        st = g.grow()
        g.read_field_mask(fmask)
        g.read_particle_mask(pmask)
        return st

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    w0 = time.perf_counter()
    for i in range(args.steps):
        stats.append(step())
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1) / args.steps
    ms = max(ms, wall * 1e3 / args.steps)
    last = g.stats()
    log(f"[bench] {args.steps} steps, {ms:.3f} ms/step, rounds {last['rounds']}, "
        f"tile visits {last['tile_visits']}, members {last['members_field']} / "
        f"{last['members_particle']}")

    ms_field = float(np.mean([s["ms_admit_field"] for s in stats]))
    fbytes = field_kernel_bytes(V)
    achieved = fbytes / (ms_field * 1e-3) / 1e9
    traffic = None
    roofline = {"bound": "hbm", "kernel": "k_admit_field", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": fbytes,
                "ms_per_launch": round(ms_field, 4)}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        from oracle import oracle_grow
        t0 = time.perf_counter()
        ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                                    inst["seeds"])
        tc = time.perf_counter() - t0
        cpu = {"value": round(V / tc, 1), "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"full {cfg['name']} workload, single-thread C breadth-first oracle "
                         f"({tc:.1f}s incl. binning and index build)",
               "host_cores_available": os.cpu_count()}
        gm = fmask.cpu().numpy().view(np.uint32)
        pm = pmask.cpu().numpy()
        parity = bool(np.array_equal(gm, ofm) and np.array_equal(pm, opm))
        log(f"[bench] oracle {tc:.1f}s, parity {parity}")

    mb = grow_model_bytes(V, Q)
    out = {
        "metric": "voxel-timesteps segmented/s to fixed point",
        "value": round(V / (ms * 1e-3), 1),
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: field {X}x{Y}x{Z}x{T} fp32, {P} particles x {T} "
                               f"steps, {len(inst['seeds'])} seeds, thresholds "
                               f"{float(inst['crit'][0])}/{float(inst['crit'][2])}",
                   "voxel_steps": V, "particle_steps": Q,
                   "tile": f"32x8x8x{args.tile_t or 8}"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {
            "rounds": last["rounds"], "tile_visits": last["tile_visits"],
            "particle_visits": last["particle_visits"], "active_tiles": last["active_tiles"],
            "members_field": last["members_field"], "members_particle": last["members_particle"],
            "ms_admit": round(float(np.mean([s["ms_admit"] for s in stats])), 4),
            "ms_rounds": round(float(np.mean([s["ms_rounds"] for s in stats])), 4),
            "ms_grow": round(float(np.mean([s["ms_total"] for s in stats])), 4),
            "model_bytes_per_step": mb,
            "model_GBps": round(mb / (ms * 1e-3) / 1e9, 1),
            "parity_vs_oracle": parity,
        },
    }
    print(json.dumps(out), flush=True)
    g.close()


if __name__ == "__main__":
    main()
