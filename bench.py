"""Benchmark: voxel-timesteps segmented per second to the fixed point on one GPU.

One step = one pass of the whole hot path over resident inputs: admissibility
of the field and particle samples, seeding, rounds of tile sweeps and
particle coupling until nothing changes, and the read-out of the uint32 field
mask and the uint8 particle-step mask into device buffers.  The workload is
the 256^3 x 64 field with 4,194,304 particles (64 crossing blobs, 32 seeds,
thresholds 0.25 / 0.25); the single-query configuration (tile depth, round
schedule, admissibility mode) is the autotuner's pick, every candidate
checked to give identical masks.

Beside the headline the bench reports, on the same GPU:
  city_2d  - a planar 2D + t city-like workload with particles at 4 steps
             per field step: grow (masks compared with the oracle) and
             clustering;
  rate4_3d - the 128^3 x 32 workload with particles saved 4 times per field
             step: grow, masks compared with the oracle;
  forward_only - the same grow with causal trajectory coupling (t -> t+1
             only), its masks compared with the directed oracle;
  seed_ids - per-seed component ids of the same grow (lowest seed index
             per node), labelled nodes compared with the oracle's union grow;
  segments - the trajectory segments of the grown feature (runs of >= 2
             member steps), timed as a read-out pass, sampled particles
             compared with the oracle's rule on the oracle's mask;
  eager    - admissibility of every sample each step (the dense HBM pass);
  learned  - the brick-activity predictor choosing the tiles tested up front,
             trained (committed weights) and untrained, masks compared;
  batched  - 256 queries as bit-planes on the 128^3 x 32 workload versus 256
             single-query grows, sampled planes compared.
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
# HBM bytes per launch read from the FETCH_SIZE / WRITE_SIZE counters (scaled by a
# 1 GiB copy), per (kernel, library version); a kernel changed since then has none.
# Source: profiles/grow_256x256x256x64_bt16_launch_hbm_counters.md (0.7.7).
MEASURED_TRAFFIC = {
    ("k_round_pull", "mf4d 0.7.7 (gfx950)"): 45795399,
    ("k_round_sweep<16>", "mf4d 0.7.7 (gfx950)"): 14023401,
}
PREDICTOR = os.path.join(ROOT, "paper_1903_12294_amd", "predictor.npy")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tile_voxels(bt: int) -> int:
    return 32 * 8 * 8 * bt


def visit_bytes(bt: int) -> int:
    """Algorithmic bytes of one tile visit (a tile of 32x8x8xBT voxel-steps):
    its label and admissibility bits (256*BT B each), the face halos it needs
    (x: 2 x 8*BT B, y and z: 4 x 32*BT B, t: 2 x 256 B) and the label bits
    written back (256*BT B)."""
    return 912 * bt + 512


def kernel_table(V: int, Q: int, bt: int, st: dict, r: dict, admit_all: bool, launch: bool,
                 T: int) -> dict:
    """Per kernel (or kernel group): algorithmic bytes per launch, measured
    device time per launch (HIP events on the library's stream), launches per
    step.  The unit counts come from the grow's statistics."""
    tv = tile_voxels(bt)
    rounds = max(st["rounds"], 1)
    tested = V if admit_all else st["tiles_tested"] * tv
    rows = {}
    rows["k_admit_field" if admit_all else "k_admit_tiles"] = (
        int(tested * 4 + tested // 4), r["ms_admit_field"], 1)
    rows["read-out (k_read_field_tiles + k_read_particles16)"] = (
        int(V // 8 + Q + st["active_tiles"] * tv // 8 + Q // 8), r["ms_read"], 1)
    sweep_b = int(st["tile_visits"] / rounds * visit_bytes(bt))
    pull_b = int(8 * st["coupled_steps"])
    if launch:
        rows[f"k_round_sweep<{bt}>"] = (sweep_b, r["ms_sweep"] / rounds, rounds)
        rows["k_round_pull"] = (pull_b, r["ms_pull"] / rounds, rounds)
        if T > 64:  # up to 64 steps the close is part of the pull kernel
            rows["k_round_close"] = (int(st["particle_visits"] / rounds * 16), r["ms_close"] / rounds, rounds)
    else:
        rows[f"k_rounds<{bt}>"] = (sweep_b * rounds + pull_b * rounds, r["ms_rounds"], 1)
    out = {}
    for k, (b, ms, n) in rows.items():
        gbs = b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out[k] = {"bytes_per_launch": b, "ms_per_launch": round(ms, 4), "launches_per_step": n,
                  "ms_per_step": round(ms * n, 4), "achieved_GBps": round(gbs, 1),
                  "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


class Timer:
    """HIP events on torch's current stream, which the library also uses."""

    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def start(self):
        self.a.record()

    def stop(self) -> float:
        self.b.record()
        self.b.synchronize()
        return self.a.elapsed_time(self.b)


def run_steps(g, fmask, pmask, steps: int, warmup: int, torch, instrumented: bool = False,
              read_async: bool = False):
    """Warm up, then time `steps` steps; per step: grow, field read, particle
    read.  Uninstrumented (the headline): one grow_read call per step, two
    events around the whole loop and nothing else.  Instrumented: grow and
    the two read calls apart, the library records its phase events and each
    step's read-out is bracketed by events (both cost device time)."""
    g.set_phase_timing(instrumented)
    # asynchronous read-outs: a step's read-outs overlap the next step's grow
    # (two label sets); the timed region ends after all of them
    g.set_read_async(read_async and not instrumented)

    def step():
        # the grow with both read-outs queued behind its rounds (one call);
        # its statistics are read after the timed steps
        g.grow_read(fmask, pmask, stats=False)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    rd = Timer(torch)
    stats, reads = [], []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    w0 = time.perf_counter()
    for _ in range(steps):
        if instrumented:
            st = g.grow()
            rd.start()
            g.read_field_mask(fmask)
            if pmask is not None:
                g.read_particle_mask(pmask)
            reads.append(rd.stop())
            stats.append(st)
        else:
            step()
    g.read_wait()
    ev1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) * 1e3 / steps
    ms = max(ev0.elapsed_time(ev1) / steps, wall)
    last = g.stats()
    g.set_phase_timing(False)
    g.set_read_async(False)
    mean = lambda k: float(np.mean([s[k] for s in stats])) if stats else 0.0
    return dict(ms=ms, ms_admit_field=mean("ms_admit_field"), ms_admit=mean("ms_admit"),
                ms_rounds=mean("ms_rounds"), ms_grow=mean("ms_total"),
                ms_sweep=mean("ms_sweep"), ms_pull=mean("ms_pull"), ms_close=mean("ms_close"),
                ms_read=float(np.mean(reads)) if reads else 0.0, stats=last)


def run_in_flight(gs, bufs, steps: int, warmup: int, torch):
    """Two grows in flight: contexts gs[0] and gs[1] (each loaded with the
    same data, each on its own stream) take the steps in turn; step i is
    submitted on context i % 2 once the host has finished that context's
    step i - 2, so step i - 1 runs on the device meanwhile.  Wall time over
    the timed steps, bracketed by device synchronisations."""
    pending = [False, False]
    stats = []

    def run(n):
        for i in range(n):
            k = i & 1
            if pending[k]:
                stats.append(gs[k].grow_finish())
            gs[k].grow_submit(*bufs[k])
            pending[k] = True
        for k in (0, 1):
            if pending[k]:
                stats.append(gs[k].grow_finish())
                pending[k] = False

    run(warmup)
    torch.cuda.synchronize()
    stats.clear()
    w0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - w0) * 1e3 / steps
    return dict(ms=ms, rounds=[s["rounds"] for s in stats])


SLIC_K = (16, 16, 16, 4)     # centres per axis (x, y, z, t): 16,384 centres
SLIC_W = (1.0, 8.0, 8.0)     # w_d, w_f, w_p
SLIC_CF = 2.0                # time-to-space factor
SLIC_ITERS = 5
SLIC_EPS_M = 0.05            # merging threshold (relative difference of both means)


def time_call(fn, torch, reps: int = 5) -> float:
    """Least wall time of fn over reps calls, each bracketed by device
    synchronisation, in ms."""
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) * 1e3
        best = t if best is None else min(best, t)
    return best


def bench_slic(torch, log, inst, name, k=SLIC_K, cpu_leg=True):
    """4D SLIC clustering (Section 3.2) of a workload (the headline one: 1.07e9
    field and 2.7e8 point samples): time per iteration (runs of 1 and 1 +
    SLIC_ITERS iterations with eps = 0, the difference), HBM bytes of an
    iteration against peak, parity at full size on 20,000 sampled labels (the
    oracle assigns them from the GPU's centres of the iteration before), the
    merge and the segment read-out, and (cpu_leg) the oracle's own speed on
    the 32^3 x 8 workload.  Particles load at the instance's rate."""
    from oracle import segments as oseg
    from oracle import slic as oslic
    from paper_1903_12294_amd import Grower, synth
    dev = torch.device("cuda:0")
    X, Y, Z = inst["dims"]
    T, P = inst["T"], inst["P"]
    rate = inst.get("rate", 1)
    Tp = inst["xyz"].shape[0]
    V, Qs = X * Y * Z * T, Tp * P
    g = Grower(device=0)
    try:
        g.load_field(torch.from_numpy(inst["field"]).to(dev))
        g.load_particles(torch.from_numpy(inst["xyz"]).to(dev), torch.from_numpy(inst["attr"]).to(dev),
                         rate=rate)

        def run(m):
            g.slic_set_params(k, *SLIC_W, SLIC_CF, 0.0, m)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it = g.slic_run()
            torch.cuda.synchronize()
            return it, time.perf_counter() - t0

        run(1)  # builds the point samples' visiting order (once per particle load)
        t1 = min(run(1)[1] for _ in range(2))
        tn, itn = None, None
        for _ in range(2):
            itn, t = run(1 + SLIC_ITERS)
            tn = t if tn is None else min(tn, t)
        ms_iter = (tn - t1) / SLIC_ITERS * 1e3
        # sampled parity at full size
        m = 3
        rng = np.random.default_rng(11)
        fi = np.sort(rng.integers(0, V, 10000))
        pi = np.sort(rng.integers(0, Qs, 10000))
        fl = torch.empty((T, Z, Y, X), dtype=torch.int32, device=dev)
        pl = torch.empty((Tp, P), dtype=torch.int32, device=dev)
        fi_d, pi_d = torch.from_numpy(fi).to(dev), torch.from_numpy(pi).to(dev)
        g.slic_set_params(k, *SLIC_W, SLIC_CF, 0.0, m - 1)
        g.slic_run()
        cen_prev, _ = g.slic_read_centres()
        g.slic_read_labels(fl, pl)
        prev = np.concatenate([fl.view(-1)[fi_d].cpu().numpy(), pl.view(-1)[pi_d].cpu().numpy()])
        g.slic_set_params(k, *SLIC_W, SLIC_CF, 0.0, m)
        it_m = g.slic_run()
        g.slic_read_labels(fl, pl)
        got = np.concatenate([fl.view(-1)[fi_d].cpu().numpy(), pl.view(-1)[pi_d].cpu().numpy()])
        tt_f = fi // (X * Y * Z)
        r = fi % (X * Y * Z)
        z, r = r // (X * Y), r % (X * Y)
        y, x = r // X, r % X
        tp, pp = pi // P, pi % P
        pos = np.concatenate([np.stack([x + 0.5, y + 0.5, z + 0.5], 1).astype(np.float32),
                              inst["xyz"][tp, pp].astype(np.float32)])
        # point times tau / rate in field steps (fp32), field times t
        tt = np.concatenate([tt_f.astype(np.float32), (tp.astype(np.float32) / np.float32(rate)).astype(np.float32)])
        val = np.concatenate([inst["field"].reshape(-1)[fi], inst["attr"][tp, pp]]).astype(np.float32)
        typ = np.concatenate([np.zeros(len(fi), np.int64), np.ones(len(pi), np.int64)])
        C = oslic.grid_interval((X, Y, Z, T), k)
        want = oslic.assign(pos, tt, val, typ, prev.astype(np.int64), cen_prev, C, k, SLIC_W, SLIC_CF)
        parity = bool(it_m == m and np.array_equal(want, got))
        # merging into features (Section 3.3) at full size; the oracle merges
        # the same centres
        cen_m, cnt_m = g.slic_read_centres()
        g.slic_merge(SLIC_EPS_M)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_feat = g.slic_merge(SLIC_EPS_M)
        ms_merge = (time.perf_counter() - t0) * 1e3
        feat, fst = g.slic_read_features()
        merge_parity = bool(np.array_equal(feat, oslic.merge_centres(cen_m, cnt_m, SLIC_EPS_M)))
        big = int(fst[:, 0:2].sum(1).max())
        # trajectory segments of the merged features (Section 3.4); the
        # oracle's rule applied to the same particles' labels and features
        sseg = torch.empty((Tp, P), dtype=torch.int32, device=dev)
        ms_sseg = time_call(lambda: g.slic_read_segments(sseg), torch)
        sel = np.sort(np.random.default_rng(13).choice(P, min(P, 4096), replace=False))
        sel_d = torch.from_numpy(sel).to(dev)
        got_s = sseg[:, sel_d].cpu().numpy()
        want_s = oseg.feature_segments(oseg.point_features(pl[:, sel_d].cpu().numpy(), feat))
        seg_parity = bool(np.array_equal(got_s, want_s))
        seg_kept = int((sseg >= 0).sum().item())
        del sseg
    finally:
        g.close()
    if cpu_leg:
        # the oracle on the small workload, for a CPU reference
        small = synth.make_config(1)
        sX, sY, sZ = small["dims"]
        sN = sX * sY * sZ * small["T"] + small["T"] * small["P"]
        t0 = time.perf_counter()
        oslic.slic(small["field"], small["xyz"], small["attr"], (4, 4, 4, 2), SLIC_W, SLIC_CF, 0.0, 3)
        tc = time.perf_counter() - t0
    N = V + Qs
    # HBM bytes of an iteration: field value, label read and write (12 B); point
    # position and time (16 B), value, label read and write (28 B)
    b = 12 * V + 28 * Qs
    gbs = b / (ms_iter * 1e-3) / 1e9
    log(f"[bench] slic {ms_iter:.2f} ms/iteration, {N / (ms_iter * 1e-3):.3e} samples/s, parity {parity}; "
        f"merge {ms_merge:.2f} ms, {n_feat} features, parity {merge_parity}; "
        f"segments {ms_sseg:.3f} ms, parity {seg_parity}")
    out = {"workload": f"{name}: {V} field + {Qs} point samples, k = {k} "
                       f"({k[0] * k[1] * k[2] * k[3]} centres), w_d/w_f/w_p = {SLIC_W}, "
                       f"c_f = {SLIC_CF}",
            "ms_per_iteration": round(ms_iter, 3), "value": round(N / (ms_iter * 1e-3), 1),
            "unit": "samples/s per iteration",
            # bound by VALU issue in the candidate loop: the field pass's
            # wave instructions (SQ_INSTS_VALU + SALU + branch + LDS) per second
            # against 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64
            # instruction, from the counter run in
            # profiles/slic_256x256x256x64_k16x16x16x4_kernel_trace.md (not
            # measurable without the profiler)
            "roofline": {"bound": "alu (distance evaluation)", "hbm_bytes_per_iteration": b,
                         "achieved_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                         "issue_peak_wave_instr_per_s": 6.144e11, "issue_frac_profiled": 0.73},
            "parity_sampled": parity, "parity_samples": int(len(got)),
            "merge": {"eps_m": SLIC_EPS_M, "ms": round(ms_merge, 3), "features": n_feat,
                      "largest_feature_samples": big, "parity_feature_ids": merge_parity},
            "segments": {"ms": round(ms_sseg, 3), "kept_point_samples": seg_kept,
                         "hbm_bytes": 20 * Qs, "achieved_GBps": round(20 * Qs / (ms_sseg * 1e-3) / 1e9, 1),
                         "parity_sampled_particles": seg_parity, "particles_checked": int(len(sel))},
            }
    if cpu_leg:
        out["cpu_oracle"] = {"value": round(sN * 4 / tc, 1), "unit": "samples/s per iteration", "cores": 1,
                             "sample": f"the 32^3 x 8 workload ({sN} samples), initial pass and 3 iterations, "
                                       f"numpy ({tc:.1f}s)"}
    return out


def bench_batched(args, torch, log):
    """256 queries on the 128^3 x 32 workload: one batched grow (tile shape from
    the autotuner) versus one single-query grow per query."""
    from paper_1903_12294_amd import Grower, autotune, synth
    dev = torch.device("cuda:0")
    inst = synth.make_config(2)
    crit, qseeds = synth.make_queries(inst, Q=256, seed=4)
    X, Y, Z = inst["dims"]
    T, P = inst["T"], inst["P"]
    V = X * Y * Z * T
    if args.batched_tile:
        tune = {"best": {"tile": list(args.batched_tile)}, "table": None}
    elif args.no_tune:
        tune = {"best": {"tile": [8, 4, 4, 4]}, "table": None}
    else:
        tune = autotune.tune_batched(inst, crit, qseeds, repeats=1, use_cache=False)
    shape = tuple(tune["best"]["tile"])
    log(f"[bench] batched tile {shape}" + (f" from {len(tune['table'])} candidates" if tune["table"] else ""))
    # the single-query grows it is compared with run their rounds as launches
    # (faster than the persistent kernel at this size)
    g = Grower(device=0, schedule="launch")
    try:
        g.load_field(torch.from_numpy(inst["field"]).to(dev))
        g.load_particles(torch.from_numpy(inst["xyz"]).to(dev), torch.from_numpy(inst["attr"]).to(dev))
        g.set_queries(crit, qseeds)
        g.set_batched_tile(*shape)
        fp = torch.empty((V, 8), dtype=torch.int32, device=dev)
        pp = torch.empty((T, P, 8), dtype=torch.int32, device=dev)
        g.grow_batched(fp, pp)
        tm = Timer(torch)
        times = []
        for _ in range(args.batched_reps):
            tm.start()
            _, _, bst = g.grow_batched(fp, pp)
            times.append(tm.stop())
        ms_b = float(np.median(times))
        # plain: one grow + read per query
        fm = torch.empty((V + 31) // 32, dtype=torch.int32, device=dev)
        pm = torch.empty((T, P), dtype=torch.uint8, device=dev)
        per_q = [qseeds[qseeds[:, 4] == q][:, :4] for q in range(len(crit))]

        def plain(q):
            g.set_criteria(*crit[q])
            g.set_seeds(per_q[q])
            g.grow()
            g.read_field_mask(fm)
            g.read_particle_mask(pm)

        for q in range(3):
            plain(q)
        tm.start()
        for q in range(len(crit)):
            plain(q)
        ms_p = tm.stop()
        bit = torch.arange(32, dtype=torch.int32, device=dev)
        ok = True
        for q in range(0, len(crit), len(crit) // 8):
            plain(q)
            plane_f = ((fp[:, q >> 5] >> (q & 31)) & 1).bool()
            plain_f = ((fm.view(-1, 1) >> bit) & 1).bool().flatten()[:V]
            plane_p = ((pp[..., q >> 5] >> (q & 31)) & 1).bool()
            ok = ok and bool(torch.equal(plane_f, plain_f)) and bool(torch.equal(plane_p, pm.bool()))
        cpu = None
        if not args.no_cpu_baseline:
            # the oracle on a bounded sample of the queries, one single-thread
            # grow per query on every host core; its planes checked too
            from oracle import oracle_grow_queries
            nq = 64
            threads = max(1, min(16, os.cpu_count() or 1))
            t0 = time.perf_counter()
            res = oracle_grow_queries(inst["field"], inst["xyz"], inst["attr"], crit[:nq],
                                      qseeds[qseeds[:, 4] < nq], threads=threads)
            tc = time.perf_counter() - t0
            for q in range(nq):
                ofm, opm, _ = res[q]
                plane_f = ((fp[:, q >> 5] >> (q & 31)) & 1).to(torch.uint8).cpu().numpy().astype(bool)
                want_f = np.unpackbits(ofm.view(np.uint8), bitorder="little")[:V].astype(bool)
                plane_p = ((pp[..., q >> 5] >> (q & 31)) & 1).to(torch.uint8).cpu().numpy()
                ok = ok and bool(np.array_equal(plane_f, want_f)) and bool(np.array_equal(plane_p, opm))
            cpu = {"value": round(nq * V / tc, 1), "unit": "query-voxel-steps/s", "cores": threads,
                   "kind": "oracle",
                   "sample": f"{nq} of the 256 queries, one single-thread C breadth-first grow each, "
                             f"on {threads} host threads ({tc:.1f}s); their planes compared too"}
    finally:
        g.close()
    return {"workload": "128^3x32 field, 262144 particles x 32 steps, 256 queries "
                        "(1-16 seeds each, thresholds U[0.15, 0.6])",
            "tile": list(shape), "ms_batched": round(ms_b, 3), "ms_plain_256": round(ms_p, 3),
            "speedup": round(ms_p / ms_b, 2),
            "value": round(256 * V / (ms_b * 1e-3), 1), "unit": "query-voxel-steps/s",
            "rounds": bst["rounds"], "tile_visits": bst["tile_visits"], "sampled_planes_equal": ok,
            "cpu_baseline": cpu, "autotune": tune["table"]}


def bench_grow_form(args, torch, log, inst, name, slic_k=None):
    """A grow workload beside the headline: the grow under both round
    schedules, masks compared with the oracle at the instance's particle rate
    (unless --no-cpu-baseline), and (slic_k) the clustering."""
    from paper_1903_12294_amd import Grower
    dev = torch.device("cuda:0")
    X, Y, Z = inst["dims"]
    T, P, r = inst["T"], inst["P"], inst.get("rate", 1)
    Tp = inst["xyz"].shape[0]
    V = X * Y * Z * T
    fmask = torch.empty((V + 31) // 32, dtype=torch.int32, device=dev)
    pmask = torch.empty((Tp, P), dtype=torch.uint8, device=dev)
    res = {}
    for sched in ("persistent", "launch"):
        g = Grower(device=0, schedule=sched)
        try:
            g.load_field(torch.from_numpy(inst["field"]).to(dev))
            g.load_particles(torch.from_numpy(inst["xyz"]).to(dev), torch.from_numpy(inst["attr"]).to(dev),
                             rate=r)
            g.set_criteria(*inst["crit"])
            g.set_seeds(inst["seeds"])
            rs = run_steps(g, fmask, pmask, args.steps, args.warmup, torch)
            res[sched] = (rs, fmask.cpu().numpy().view(np.uint32).copy(), pmask.cpu().numpy().copy())
        finally:
            g.close()
    best = min(res, key=lambda k: res[k][0]["ms"])
    st = res[best][0]["stats"]
    out = {"workload": f"{name}: field {X}x{Y}x{Z}x{T} fp32, {P} particles x {Tp} steps ({r} per field "
                       f"step), {len(inst['seeds'])} seeds, thresholds {float(inst['crit'][0])}"
                       f"/{float(inst['crit'][2])}",
           "ms_per_step": {s: round(v[0]["ms"], 4) for s, v in res.items()}, "schedule": best,
           "value": round(V / (res[best][0]["ms"] * 1e-3), 1), "unit": "voxel-steps/s",
           "rounds": st["rounds"], "members_field": st["members_field"],
           "members_particle": st["members_particle"]}
    if not args.no_cpu_baseline:
        from oracle import oracle_grow
        t0 = time.perf_counter()
        ofm, opm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"], rate=r)
        out["oracle_s"] = round(time.perf_counter() - t0, 2)
        out["parity_vs_oracle"] = bool(all(np.array_equal(f, ofm) and np.array_equal(p, opm)
                                           for _, f, p in res.values()))
    log(f"[bench] {name} {out['ms_per_step']} ms/step, parity {out.get('parity_vs_oracle')}")
    del fmask, pmask
    torch.cuda.empty_cache()
    if slic_k is not None:
        out["slic"] = bench_slic(torch, log, inst, name, k=slic_k, cpu_leg=False)
    return out


def bench_city(args, torch, log):
    """The planar 2D + t city-like workload (1024 x 1024 x 1 cells x 48 field
    steps, 28,672 particles at 4 steps per field step): grow and clustering
    with 32 x 32 x 1 x 4 centres."""
    from paper_1903_12294_amd import synth
    t0 = time.time()
    inst = synth.make_city()
    log(f"[bench] generated {synth.CITY['name']} in {time.time() - t0:.1f}s")
    return bench_grow_form(args, torch, log, inst, synth.CITY["name"], slic_k=(32, 32, 1, 4))


def bench_rate3d(args, torch, log):
    """The 128^3 x 32 workload with its 262,144 particles saved 4 times per
    field step (128 steps, two label words each), as the paper's combustion
    particles are saved more often than the field: the grow."""
    from paper_1903_12294_amd import synth
    c = synth.CONFIGS[2]
    t0 = time.time()
    inst = synth.make_instance(c["X"], c["Y"], c["Z"], c["T"], c["P"], n_blobs=c["n_blobs"], seed=c["seed"],
                               n_seeds=c["n_seeds"], tau_f=c["tau"], tau_p=c["tau"], crossing=c["crossing"],
                               rate=4)
    name = "single-128^3x32-r4"
    log(f"[bench] generated {name} in {time.time() - t0:.1f}s")
    return bench_grow_form(args, torch, log, inst, name)


def bench_learned(g, args, torch, fmask, pmask, ref_f, ref_p):
    """Score-ordered scheduling on the loaded workload (lazy admissibility):
    the plain grow, the heuristic priority (candidate tiles in descending
    order of their greatest field value), and the learned scheduler with the
    trained (committed weights) and an untrained network: time per step,
    rounds (the verification round and any after it included), tile visits
    of the rounds and of the priority pass, tiles tested up front; masks
    compared with the plain grow's (ref_f, ref_p)."""
    from paper_1903_12294_amd.learned import init_params
    g.set_scheduler("plain")
    base = run_steps(g, fmask, pmask, args.steps, 2, torch)
    bst = base["stats"]
    lf = {"plain": {"ms_per_step": round(base["ms"], 4), "rounds": bst["rounds"],
                    "tile_visits": bst["tile_visits"], "tiles_tested": bst["tiles_tested"]}}
    variants = [("heuristic", None, None), ("untrained", init_params(0), 0.0)]
    if os.path.exists(PREDICTOR):
        meta = json.load(open(os.path.splitext(PREDICTOR)[0] + ".json"))
        variants.insert(1, ("trained", np.load(PREDICTOR), float(meta["logit_threshold"])))
    for name, params, thr in variants:
        if params is None:
            g.set_scheduler("heuristic")
        else:
            g.set_scheduler("learned", params, thr)
        rl = run_steps(g, fmask, pmask, args.steps, 2, torch)
        st = rl["stats"]
        lf[name] = {"ms_per_step": round(rl["ms"], 4), "speedup_vs_plain": round(base["ms"] / rl["ms"], 3),
                    "rounds": st["rounds"], "verify_rounds": st["verify_rounds"],
                    "tile_visits": st["tile_visits"], "priority_visits": st["priority_visits"],
                    "tiles_tested": st["tiles_tested"], "tiles_deferred_read": st["tiles_deferred_read"],
                    "masks_equal": bool(torch.equal(fmask, ref_f) and torch.equal(pmask, ref_p))}
        if thr is not None:
            lf[name]["logit_threshold"] = thr
    g.set_scheduler("plain")
    return lf


def bench_adjacent(g, inst, fmask, pmask, args, torch, forms):
    """Adjacent outputs of the grower on the headline workload, on the same
    context: the trajectory segment read-out, the grow with forward-only
    coupling, and the per-seed component ids.  Fills `forms`; returns what the
    oracle checks afterwards."""
    dev = torch.device("cuda:0")
    X, Y, Z = inst["dims"]
    T, P = inst["T"], inst["P"]
    V = X * Y * Z * T
    # trajectory segments of the grown feature (Section 3.4): a read-out pass
    seg = torch.empty((T, P), dtype=torch.uint8, device=dev)
    ms_seg = time_call(lambda: g.read_particle_segments(seg), torch)
    seg_sel = np.sort(np.random.default_rng(12).choice(P, min(P, 4096), replace=False))
    seg_cols = seg[:, torch.from_numpy(seg_sel).to(dev)].cpu().numpy()
    seg_kept = int(seg.sum(dtype=torch.int64).item())
    del seg
    # label words, candidate flags, output bytes
    seg_bytes = 8 * max(1, (T + 63) // 64) * P + P + T * P
    forms_seg = {"ms": round(ms_seg, 4), "kept_particle_steps": seg_kept, "hbm_bytes": seg_bytes,
                 "achieved_GBps": round(seg_bytes / (ms_seg * 1e-3) / 1e9, 1),
                 "frac": round(seg_bytes / (ms_seg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    forms["segments"] = forms_seg
    # forward-only (causal) trajectory coupling: the same workload and
    # configuration, a different fixed point
    g.set_trajectory_mode("forward")
    rf = run_steps(g, fmask, pmask, args.steps, 2, torch)
    fwd_f, fwd_p = fmask.clone(), pmask.clone()
    forms["forward_only"] = {"ms_per_step": round(rf["ms"], 4), "value": round(V / (rf["ms"] * 1e-3), 1),
                             "rounds": rf["stats"]["rounds"],
                             "members_field": rf["stats"]["members_field"],
                             "members_particle": rf["stats"]["members_particle"]}
    g.set_trajectory_mode("both")
    # per-seed component ids: one grow per seed outside the earlier seeds'
    # regions, folded into int32 ids
    fid = torch.empty((T, Z, Y, X), dtype=torch.int32, device=dev)
    pid = torch.empty((T, P), dtype=torch.int32, device=dev)
    g.grow_seed_ids(fid, pid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, n_grows = g.grow_seed_ids(fid, pid)
    ms_ids = (time.perf_counter() - t0) * 1e3
    sd = np.asarray(inst["seeds"], np.int64).reshape(-1, 4)
    sd_d = torch.from_numpy(((sd[:, 3] * Z + sd[:, 2]) * Y + sd[:, 1]) * X + sd[:, 0]).to(dev)
    seed_id = fid.view(-1)[sd_d].cpu().numpy()
    # labelled field nodes as canonical bit words, to compare with the masks
    lab = np.packbits(fid.view(-1).cpu().numpy() >= 0, bitorder="little")
    ids_words = np.zeros((V + 31) // 32, np.uint32)
    ids_words.view(np.uint8)[:len(lab)] = lab
    del lab
    ids_pl = (pid >= 0).cpu().numpy()
    forms["seed_ids"] = {"ms": round(ms_ids, 3), "seeds": int(len(sd)), "grows": n_grows,
                         "ids_in_use": int(torch.unique(fid[fid >= 0]).numel()),
                         "seed_ids": [int(v) for v in seed_id]}
    del fid, pid
    return dict(seg_sel=seg_sel, seg_cols=seg_cols, fwd_f=fwd_f, fwd_p=fwd_p, ids_words=ids_words,
                ids_pl=ids_pl, sd=sd)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 30 timed steps: the last step's read-outs, which no later grow hides,
    # weigh 1/30 of one read-out per step
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3])
    ap.add_argument("--no-tune", action="store_true", help="default configuration, no autotuning")
    ap.add_argument("--schedule", choices=["persistent", "launch"], help="fix the schedule (no tuning)")
    ap.add_argument("--admit", choices=["tiles", "all"], help="fix the admissibility mode (no tuning)")
    ap.add_argument("--tile-t", type=int, choices=[4, 8, 16], help="fix the tile depth (no tuning)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="the headline grow only (no other form)")
    ap.add_argument("--in-flight", type=int, choices=[1, 2], default=1,
                    help="grows in flight: 2 = two contexts on two streams take the steps in turn")
    ap.add_argument("--sync-reads", action="store_true",
                    help="headline steps with stream-ordered read-outs (default: asynchronous, "
                         "each step's read-outs beside the next step's rounds)")
    ap.add_argument("--slic-only", action="store_true",
                    help="only the clustering form (for profiling its kernels); prints its JSON object")
    ap.add_argument("--city-only", action="store_true",
                    help="only the planar city-like form (for profiling); prints its JSON object")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched form (for profiling its kernels); prints its JSON object")
    ap.add_argument("--learned-only", action="store_true",
                    help="only the learned-scheduling form at the chosen config (for profiling); "
                         "prints its JSON object")
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--batched-tile", type=int, nargs=4, metavar=("BX", "BY", "BZ", "BT"),
                    help="fix the batched tile shape (no tuning)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run three 1 GiB device copies (a plain copy kernel of known size, "
                         "the scale for hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the grower runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_12294_amd import Grower, autotune, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.city_only:
        print(json.dumps(bench_city(args, torch, log)), flush=True)
        return
    if args.batched_only:
        print(json.dumps(bench_batched(args, torch, log)), flush=True)
        return
    cfg = synth.CONFIGS[args.config]
    t0 = time.time()
    inst = synth.make_config(args.config)
    log(f"[bench] generated {cfg['name']} in {time.time() - t0:.1f}s")
    if args.slic_only:
        print(json.dumps(bench_slic(torch, log, inst, cfg["name"])), flush=True)
        return
    X, Y, Z = inst["dims"]
    T, P = inst["T"], inst["P"]
    V, Q = X * Y * Z * T, P * T

    choice = dict(tile_t=8, schedule="persistent", admit="tiles")
    fixed = {k: v for k, v in (("tile_t", args.tile_t), ("schedule", args.schedule),
                               ("admit", args.admit)) if v is not None}
    choice.update(fixed)
    tune = None
    if not args.no_tune and not fixed:
        t0 = time.time()
        tune = autotune.tune_plain(inst, repeats=3, use_cache=False)
        choice = {k: tune["best"][k] for k in ("tile_t", "schedule", "admit")}
        log(f"[bench] autotuned {choice} over {len(tune['table'])} candidates "
            f"(identical masks) in {time.time() - t0:.1f}s")

    g = Grower(device=0, tile_t=choice["tile_t"])
    t0 = time.time()
    g.load_field(torch.from_numpy(inst["field"]).to(dev))
    g.load_particles(torch.from_numpy(inst["xyz"]).to(dev), torch.from_numpy(inst["attr"]).to(dev))
    g.set_criteria(*inst["crit"])
    g.set_seeds(inst["seeds"])
    g.set_schedule(choice["schedule"])
    g.set_admit_mode(choice["admit"])
    torch.cuda.synchronize()
    log(f"[bench] loaded and binned in {time.time() - t0:.1f}s")

    fmask = torch.empty((V + 31) // 32, dtype=torch.int32, device=dev)
    pmask = torch.empty((T, P), dtype=torch.uint8, device=dev)
    r0 = run_steps(g, fmask, pmask, args.steps, args.warmup, torch, read_async=not args.sync_reads)
    ms_one = r0["ms"]
    ms = ms_one
    flight = None
    if args.in_flight == 2:
        # a second context on its own stream, loaded with the same data, and
        # this one moved to a stream of its own: two grows in flight
        streams = [torch.cuda.Stream(device=dev) for _ in range(2)]
        ga = Grower(device=0, stream=streams[0].cuda_stream, tile_t=choice["tile_t"])
        gb = Grower(device=0, stream=streams[1].cuda_stream, tile_t=choice["tile_t"])
        try:
            for gx in (ga, gb):
                gx.load_field(torch.from_numpy(inst["field"]).to(dev))
                gx.load_particles(torch.from_numpy(inst["xyz"]).to(dev), torch.from_numpy(inst["attr"]).to(dev))
                gx.set_criteria(*inst["crit"])
                gx.set_seeds(inst["seeds"])
                gx.set_schedule(choice["schedule"])
                gx.set_admit_mode(choice["admit"])
            bufs = [(torch.full_like(fmask, -1), torch.full_like(pmask, 0xFF)) for _ in range(2)]
            torch.cuda.synchronize()
            rf = run_in_flight([ga, gb], bufs, args.steps, args.warmup, torch)
            torch.cuda.synchronize()
            same = all(bool(torch.equal(f, fmask) and torch.equal(p, pmask)) for f, p in bufs)
            flight = {"ms_per_step": round(rf["ms"], 4), "ms_per_step_one_in_flight": round(ms_one, 4),
                      "masks_equal": same, "rounds": sorted(set(rf["rounds"]))}
            if not same:
                raise SystemExit("[bench] two grows in flight gave other masks than one")
            ms = rf["ms"]
        finally:
            ga.close()
            gb.close()
            del bufs
            torch.cuda.empty_cache()
    # the same steps again with the library's phase events, for per-kernel times
    r = run_steps(g, fmask, pmask, args.steps, 1, torch, instrumented=True)
    # a cold step: the first grow of a fresh context (its first chunk of
    # rounds is not sized from a previous grow), stream-ordered read-outs
    g2 = Grower(device=0, tile_t=choice["tile_t"])
    try:
        g2.load_field(torch.from_numpy(inst["field"]).to(dev))
        g2.load_particles(torch.from_numpy(inst["xyz"]).to(dev), torch.from_numpy(inst["attr"]).to(dev))
        g2.set_criteria(*inst["crit"])
        g2.set_seeds(inst["seeds"])
        g2.set_schedule(choice["schedule"])
        g2.set_admit_mode(choice["admit"])
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        g2.grow_read(fmask, pmask)
        torch.cuda.synchronize()
        ms_cold = (time.perf_counter() - tc0) * 1e3
    finally:
        g2.close()
    st = r["stats"]
    log(f"[bench] {args.steps} steps, {ms:.3f} ms/step, rounds {st['rounds']}, "
        f"tile visits {st['tile_visits']}, members {st['members_field']} / {st['members_particle']}")

    admit_all = choice["admit"] == "all"
    launch = choice["schedule"] == "launch"
    phases = {"admit_field": r["ms_admit_field"], "admit_particles": r["ms_admit"] - r["ms_admit_field"],
              "rounds": r["ms_rounds"], "read_out": r["ms_read"]}
    kt = kernel_table(V, Q, choice["tile_t"], st, r, admit_all, launch, T)
    # the roofline object is the kernel with the most device time per step
    dom = max(kt, key=lambda k: kt[k]["ms_per_step"])
    from paper_1903_12294_amd import _lib
    version = _lib.load_library().mf4d_version().decode()
    # the counters were taken at 256^3 x 64 with tile depth 16 and launched rounds
    measured_here = (X, Y, Z, T) == (256, 256, 256, 64) and choice["tile_t"] == 16 and launch
    traffic = MEASURED_TRAFFIC.get((dom, version)) if measured_here else None
    # the whole step against the lazy floor: 0.43 B per voxel-step (the
    # admissible-reached nodes and their shell at ~0.5% occupancy, dominated
    # by the dense mask writes)
    floor_b = 0.43 * V
    roofline = {"bound": "hbm", "kernel": dom, "achieved": kt[dom]["achieved_GBps"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kt[dom]["frac"],
                "traffic": int(traffic) if traffic else None,
                "bytes_per_launch": kt[dom]["bytes_per_launch"],
                "ms_per_launch": kt[dom]["ms_per_launch"],
                "grow_lazy_floor_bytes": int(floor_b),
                "grow_frac": round(floor_b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ref_f = fmask.clone()
    ref_p = pmask.clone()
    if args.learned_only:
        g.set_admit_mode("tiles")
        out = bench_learned(g, args, torch, fmask, pmask, ref_f, ref_p)
        g.close()
        print(json.dumps(out), flush=True)
        return
    forms = {}
    checks = None
    if not args.no_forms:
        checks = bench_adjacent(g, inst, fmask, pmask, args, torch, forms)
    if not args.no_forms:
        # eager: every sample tested each step
        g.set_admit_mode("all")
        re0 = run_steps(g, fmask, pmask, args.steps, 2, torch)
        re_ = run_steps(g, fmask, pmask, args.steps, 1, torch, instrumented=True)
        eb = int(V * 4 + V // 4)
        ea = eb / (re_["ms_admit_field"] * 1e-3) / 1e9
        forms["eager"] = {"ms_per_step": round(re0["ms"], 4), "value": round(V / (re0["ms"] * 1e-3), 1),
                          "masks_equal": bool(torch.equal(fmask, ref_f) and torch.equal(pmask, ref_p)),
                          "k_admit_field": {"bytes_per_launch": eb, "ms_per_launch": round(re_["ms_admit_field"], 4),
                                            "achieved_GBps": round(ea, 1), "frac": round(ea / HBM_PEAK_GBS, 4)}}
        g.set_admit_mode("tiles")
        forms["learned"] = bench_learned(g, args, torch, fmask, pmask, ref_f, ref_p)
        g.set_admit_mode(choice["admit"])
    g.close()
    del g
    torch.cuda.empty_cache()

    if not args.no_forms:
        forms["batched"] = bench_batched(args, torch, log)
        forms["slic"] = bench_slic(torch, log, inst, cfg["name"])
        forms["city_2d"] = bench_city(args, torch, log)
        forms["rate4_3d"] = bench_rate3d(args, torch, log)
        torch.cuda.empty_cache()

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        from oracle import oracle_grow
        t0 = time.perf_counter()
        ofm, opm, ost = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"],
                                    inst["seeds"])
        tc = time.perf_counter() - t0
        cpu = {"value": round(V / tc, 1), "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"the full {cfg['name']} workload once, single-thread C breadth-first oracle "
                         f"({tc:.1f}s incl. binning and index build)",
               "host_cores_available": os.cpu_count()}
        parity = bool(np.array_equal(ref_f.cpu().numpy().view(np.uint32), ofm)
                      and np.array_equal(ref_p.cpu().numpy(), opm))
        if checks:
            t0 = time.perf_counter()
            ffm, fpm, _ = oracle_grow(inst["field"], inst["xyz"], inst["attr"], inst["crit"], inst["seeds"],
                                      forward_only=True)
            fo = forms["forward_only"]
            fo["oracle_s"] = round(time.perf_counter() - t0, 1)
            fo["parity_vs_oracle"] = bool(np.array_equal(checks["fwd_f"].cpu().numpy().view(np.uint32), ffm)
                                          and np.array_equal(checks["fwd_p"].cpu().numpy(), fpm))
            # per-seed ids: labelled nodes are the union grow; a seed's own
            # voxel holds an id no larger than its index
            si = forms["seed_ids"]
            adm = [bool(inst["crit"][0] <= inst["field"][t, z, y, x] <= inst["crit"][1])
                   for x, y, z, t in checks["sd"]]
            si["labelled_equal_oracle_union"] = bool(
                np.array_equal(checks["ids_words"], ofm) and np.array_equal(checks["ids_pl"], opm != 0))
            si["seed_voxels_consistent"] = bool(all(
                (0 <= s_id <= j) if a else True for j, (s_id, a) in enumerate(zip(si["seed_ids"], adm))))
            from oracle import segments as oseg
            sg = forms["segments"]
            sg["parity_sampled_particles"] = bool(
                np.array_equal(checks["seg_cols"], oseg.mask_segments(opm[:, checks["seg_sel"]])))
            sg["particles_checked"] = int(len(checks["seg_sel"]))
            log(f"[bench] forward-only parity {fo['parity_vs_oracle']}, seed ids {si['labelled_equal_oracle_union']}"
                f"/{si['seed_voxels_consistent']}, segments parity {sg['parity_sampled_particles']}")
        log(f"[bench] oracle {tc:.1f}s, parity {parity}")

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
                   "tile": f"32x8x8x{choice['tile_t']}", "schedule": choice["schedule"],
                   "admissibility": choice["admit"],
                   "in_flight": 2 if flight else 1,
                   "read_out": ("queued behind each grow's rounds (two contexts alternate)" if flight else
                                "stream-ordered" if args.sync_reads else
                                "asynchronous: each step's read-outs beside the next step's rounds")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {
            "rounds": st["rounds"], "tile_visits": st["tile_visits"],
            "particle_visits": st["particle_visits"], "active_tiles": st["active_tiles"],
            "tiles_tested": st["tiles_tested"],
            "members_field": st["members_field"], "members_particle": st["members_particle"],
            "phases_ms": {k: round(v, 4) for k, v in phases.items()},
            "kernels": kt, "coupled_steps": st["coupled_steps"],
            "ms_grow": round(r["ms_grow"], 4),
            "ms_per_step_instrumented": round(r["ms"], 4),
            "ms_first_grow_fresh_context": round(ms_cold, 4),
            "ms_per_step_one_in_flight": round(ms_one, 4),
            "two_in_flight": flight,
            "parity_vs_oracle": parity,
            "autotune": tune["table"] if tune else None,
        },
        "forms": forms,
    }
    print(json.dumps(out), flush=True)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
