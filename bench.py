"""Throughput of the full GPE + Cahn-Hilliard time step on one MI355X.

Workload: 3-D rising bubble on a 256^3 grid with no-slip walls (density and
viscosity ratio 10, Eotvos 10, Morton 1e-4, W = 2, M = 0.02, D3Q15 CH
stencils), FP32.  One step = three TVD-RK3 flow stages + four RK4 CH stages.
The state is initialised in HBM before the timed region; the timed region is
K steps enqueued back to back on the solver's stream with HIP events around
the launches of the dominant kernel, between two synchronisations (the same
K steps replayed as HIP graphs, and K more with events around every kernel,
are timed afterwards for context).

Prints one JSON line: MLUPS (cells x steps / s / 1e6), the roofline of the
dominant kernel (algorithmic bytes per launch / mean launch time from the HIP
events, against the 8 TB/s HBM peak), the step-level roofline, the CPU oracle
timed on a bounded sample of the same workload, and a short measurement of
the batched ensemble (512 independent 2-D drops, 64^2 .. 256^2).

The default line also carries the paper's own timing case (3-D drop
coalescence, 120^3, D3Q15 / 19 / 27 CH stencils, FP64 and FP32) beside the
paper's derived throughput, and a plain device-copy bandwidth measured in the
same run, so that the roofline is given against the 8 TB/s figure and against
what a copy reaches.  `--workload coalescence` prints that case alone
(D3Q15, FP64 unless --precision is given; vs_baseline = ratio to the paper's
four-node CPU figure, context only).

`--workload ensemble` measures the ensemble alone (default 5000 steps):
aggregate cell updates per second of the batch against the same cases run
one after another as plain single grids.

`--workload rt2d` times the 2-D Rayleigh-Taylor grid (256 x 1024, walls in
y, FP32 and FP64 unless --precision is given; default 2000 steps) as graph-
replayed steps; the value is the FP32 (or the given precision's) MLUPS.
The grid's fields fit in the device's last-level cache, so no HBM roofline
is given for it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS per full RK3 step (3D 256^3) vs HBM roofline; learned-coarse speedup"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


# the sources that define the stencil kernels of the step (their measured
# HBM traffic is valid only while these are unchanged)
KERNEL_SOURCES = ("gpe_device.hpp", "gpe_plane.hpp", "gpe_flow.hip", "gpe_ch.hip")


def csrc_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2011_00814_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def problem(n: int, precision: str):
    from paper_2011_00814_amd import workloads as W

    prob, _ = W.rising_bubble_3d(nx=n, ny=n, nz=n, zc=48.0, precision=precision, in_kernel_init=True)
    return prob


def measured_traffic(kernel: str, precision: str):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters, valid only while the kernel sources are unchanged."""
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = data.get(f"{kernel}:{precision}")
    if not ent or ent.get("csrc_hash") != csrc_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(n: int, precision: str, z_sample: int = 64, steps: int = 4):
    import ctypes

    import numpy as np

    from oracle import oracle as O
    from paper_2011_00814_amd import workloads as W

    prob, st = W.rising_bubble_3d(nx=n, ny=n, nz=z_sample, zc=48.0, precision="fp64")
    try:
        threads = ctypes.CDLL("libgomp.so.1").omp_get_max_threads()
    except OSError:
        threads = 1
    t0 = time.perf_counter()
    O.run(prob, st, steps)
    dt = time.perf_counter() - t0
    cells = n * n * z_sample
    return {
        "value": cells * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{steps} step(s) of the same 3-D bubble physics on a {n}x{n}x{z_sample} slab "
                  f"(bottom of the 256^3 domain, bubble included), FP64 C oracle, {dt:.1f} s",
    }


def cpu_configs() -> dict:
    """The oracle timed on all host cores and on one core for bounded samples
    of each benchmark configuration (context for the GPU figures, never a
    target): MLUPS over a few steps from the configuration's initial state."""
    import ctypes

    from oracle import oracle as O
    from paper_2011_00814_amd import workloads as W

    gomp = ctypes.CDLL("libgomp.so.1")
    nmax = int(gomp.omp_get_max_threads())
    cases = [
        ("configuration 1: static drop 64^2", W.static_drop_2d(), (200, 50)),
        ("configuration 2: Rayleigh-Taylor 256 x 1024", W.rayleigh_taylor_2d(), (20, 4)),
        ("configuration 3: rising bubble 128 x 128 x 256", W.rising_bubble_3d(precision="fp64"), (2, 1)),
        ("256^3 rising bubble, 256 x 256 x 64 slab", W.rising_bubble_3d(nx=256, ny=256, nz=64, zc=48.0,
                                                                       precision="fp64"), (2, 1)),
    ]
    rows = []
    try:
        for name, (prob, st), steps in cases:
            cells = prob["n"][0] * prob["n"][1] * prob["n"][2]
            row = {"case": name, "cells": cells}
            for threads, nsteps in ((nmax, steps[0]), (1, steps[1])):
                gomp.omp_set_num_threads(threads)
                t0 = time.perf_counter()
                O.run(prob, st, nsteps)
                dt = time.perf_counter() - t0
                key = "all_cores" if threads == nmax else "one_core"
                row[key] = {"threads": threads, "steps": nsteps, "s": round(dt, 2),
                            "mlups": round(cells * nsteps / dt / 1e6, 3)}
                print(f"cpu_configs: {name}, {threads} thread(s): {row[key]['mlups']} MLUPS",
                      file=sys.stderr, flush=True)
            rows.append(row)
    finally:
        gomp.omp_set_num_threads(nmax)
    return {"kind": "oracle", "precision": "fp64", "cores": nmax, "rows": rows}


def ensemble_bench(steps: int, warmup: int, precision: str = "fp32", baseline_steps: int = 200) -> dict:
    """The batched ensemble of 512 seeded 2-D drops: aggregate throughput of
    `steps` graph-replayed batch steps, per-case finite flags after them, and
    the time the same cases take one after another as plain single grids.
    A plain grid's step time depends only on its size (same kernels), so the
    sequential time is the sum over cases of the step time measured for that
    case's size (two cases of each size, `baseline_steps` steps each)."""
    import numpy as np
    import torch

    from paper_2011_00814_amd import gpe
    from paper_2011_00814_amd import workloads as W

    cases = W.ensemble_cases(512, seed=0, precision=precision)
    cells = [c["n"][0] * c["n"][1] for c in cases]
    ens = gpe.Ensemble(cases, device="cuda:0")

    def timed(n):
        ens.synchronize()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(ens.stream)
        ens.run(n)
        b.record(ens.stream)
        ens.synchronize()
        return a.elapsed_time(b)

    ens.run(warmup)
    default_ms = timed(min(steps, 100)) / min(steps, 100)  # 32-row tiles
    rows = ens.autotune(trial_steps=10)
    tuned_rows = {}
    for c, r in zip(cases, rows):
        tuned_rows[str(c["n"][0])] = int(r)
    ens.run(warmup)
    ms = timed(steps)
    flags = ens.finite()
    steps_done = ens.case(0).diagnostics()["step"]
    ens.close()
    # sequential plain runs, timed per size
    per_size = {}
    for N in sorted(set(c["n"][0] for c in cases)):
        sample = [c for c in cases if c["n"][0] == N][:2]
        t = []
        for c in sample:
            s = gpe.Solver(c, None, device="cuda:0")
            s.run(5)
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.run(baseline_steps)
            e1.record(s.stream)
            s.synchronize()
            t.append(e0.elapsed_time(e1) / baseline_steps)
            s.close()
        per_size[N] = sum(t) / len(t)
    seq_ms = sum(per_size[c["n"][0]] for c in cases) * steps
    dts = np.array([c["dt"] for c in cases])
    agg = sum(cells) * steps / (ms * 1e-3)
    return {
        "workload": "512 periodic 2-D elliptic drops, N uniform over {64,96,128,192,256}^2 "
                    f"({sum(cells)} cells), D2Q9, RK3 flow + RK2 CH, per-case dt, {precision}",
        "steps": steps,
        "ms_per_batch_step": round(ms / steps, 4),
        "ms_per_batch_step_32_row_tiles": round(default_ms, 4),
        "autotuned_tile_rows_by_size": tuned_rows,
        "steps_run_per_case": int(steps_done),
        "aggregate_cell_updates_per_s": round(agg, 1),
        "aggregate_mlups": round(agg / 1e6, 1),
        "sequential_ms_per_step_by_size": {str(k): round(v, 5) for k, v in per_size.items()},
        "sequential_ms_per_batch_step": round(seq_ms / steps, 4),
        "speedup_vs_sequential": round(seq_ms / ms, 2),
        "finite_cases": int(flags.sum()),
        "failed_cases": [int(i) for i in np.nonzero(flags == 0)[0]],
        "dt": {"min": float(dts.min()), "median": float(np.median(dts)), "max": float(dts.max())},
    }


def learned_bench(ntrain=200, fine_steps=20000, n_snap=40, iters=12000, neval=50, batch=32, checkpoints=32,
                  rollout=True, log=None) -> dict:
    """The learned coarse correction: training data from `ntrain` fine
    multi-mode Rayleigh-Taylor runs (256 x 1024, seeds 0..ntrain-1), training
    on the GPU (half the iterations on one-step pairs; with `rollout`, the
    rest on those and on pairs drawn from the network's own corrected coarse
    rollouts), then `neval` held-out seeds (1000..) run on the fine grid and
    on the 4x coarser grid (64 x 256, fine_steps / 4 steps) without and with
    the network; interface-position errors on the coarse grid against the
    restricted fine solution at `checkpoints` times, the horizon up to which
    every case keeps >= 95 % of its columns within one coarse cell, the
    indicator-driven fallback to the fine solver; speedup = fine time /
    (corrected coarse time + fallback time)."""
    from paper_2011_00814_amd import learned as LD

    quiet = log or (lambda *a, **k: None)  # noqa: E731
    t0 = time.perf_counter()
    data = LD.generate(list(range(ntrain)), fine_steps=fine_steps, n_snap=n_snap, log=quiet,
                       unroll=3 if rollout else 0)
    gen_s = time.perf_counter() - t0
    first = iters // 2 if rollout else iters
    net, hist, sin, sout, train_s = LD.train(data, iters=first, batch=batch, lr=1e-3, log=quiet)
    roll_s = 0.0
    if rollout:
        t1 = time.perf_counter()
        LD.rollout_pairs(net, data, sin, sout, log=quiet)
        roll_s = time.perf_counter() - t1
        net, hist2, _, _, t2 = LD.train(data, iters=iters - first, batch=batch, lr=5e-4, log=quiet, net=net,
                                        scales_=(sin, sout))
        hist, train_s = hist + hist2, train_s + t2
    del data
    held = LD.generate(list(range(1000, 1000 + min(8, neval))), fine_steps=fine_steps, n_snap=10, log=quiet)
    plain, corr = LD.one_step_gain(net, held, sin, sout)
    del held
    res = LD.evaluate(net, sin, sout, list(range(1000, 1000 + neval)), fine_steps=fine_steps, log=quiet,
                      checkpoints=checkpoints)
    res.update({
        "workload": f"multi-mode Rayleigh-Taylor, At ~ U(0.2, 0.8), Re 3000, fine 256x1024 / coarse 64x256, "
                    f"{ntrain} training runs x {fine_steps} fine steps ({n_snap} snapshot pairs each"
                    f"{', plus pairs from corrected rollouts of 1-3 steps' if rollout else ''}), "
                    f"{neval} held-out seeds; network 3x3 CNN 4-32-32-4, BF16 operands, FP32 accumulation",
        "data_generation_s": round(gen_s, 1), "rollout_pairs_s": round(roll_s, 1),
        "training_s": round(train_s, 1), "training_iters": iters,
        "loss_first_last": [round(hist[0][1], 4), round(hist[-1][1], 4)],
        "one_step_mse_plain": round(plain, 4), "one_step_mse_network": round(corr, 4),
    })
    return res


def hbm_probe(mib: int = 4096, reps: int = 10, workgroups: int = 0, warm: int = 3) -> dict:
    """HBM bandwidth of the library's streaming kernels (gpe_hbm_stream:
    read-only, write-only and copy with 16-byte accesses) on buffers far
    larger than the last-level cache, timed with events on the stream the
    kernels run on.  Bytes counted: read n, write n, copy 2n."""
    import torch

    from paper_2011_00814_amd import gpe

    nbytes = mib * (1 << 20)
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.zeros_like(a)
    sid = torch.cuda.current_stream().cuda_stream
    out = {"buffer_mib": mib, "workgroups": workgroups or "8 per CU"}
    for name, mode, moved in (("read", gpe.GPE_STREAM_READ, nbytes), ("write", gpe.GPE_STREAM_WRITE, nbytes),
                              ("copy", gpe.GPE_STREAM_COPY, 2 * nbytes)):
        for _ in range(warm):
            gpe.gpe_hbm_stream(mode, b.data_ptr(), a.data_ptr(), nbytes, workgroups, sid)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            gpe.gpe_hbm_stream(mode, b.data_ptr(), a.data_ptr(), nbytes, workgroups, sid)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{name}_gbs"] = round(moved / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(mib: int = 1024, reps: int = 20) -> float:
    """Practical HBM bandwidth of a plain device copy (read + write bytes / s)."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 8 * n / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def time_solver(prob, steps: int, warmup: int, graph_context: bool = True) -> dict:
    """Warm-up, then exactly `steps` steps enqueued back to back on the
    solver's stream (the timed region) with HIP events around the launches
    of the dominant kernel only, then (graph_context) the same number of
    steps as graph replays and as launches with events around every kernel,
    for context.  The warm-up replays the step graph once and runs its other
    steps with events around every kernel; the kernel with the longest mean
    launch there is the dominant one (the last flow stage when the warm-up
    has no such step).  The initial state is built in HBM by the library."""
    import torch

    from paper_2011_00814_amd import gpe

    s = gpe.Solver(prob, None, device="cuda:0")
    nx, ny, nz = prob["n"]
    ncell = nx * ny * nz
    d0 = s.diagnostics()
    warm = None
    if warmup >= 1:
        s.run(1)
    if warmup >= 2:
        warm = s.kernel_times(warmup - 1)
    s.synchronize()
    torch.cuda.synchronize()
    dom_q = max(range(len(warm)), key=lambda q: warm[q][1]) if warm else 2
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(s.stream)
    timed = s.kernel_times(steps, mask=1 << dom_q)
    stop.record(s.stream)
    s.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    graph_ms = None
    ktimes = None
    if graph_context:
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(s.stream)
        s.run(steps)
        g1.record(s.stream)
        s.synchronize()
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / steps
        ktimes = s.kernel_times(steps)
    d = s.diagnostics()
    s.close()
    return {
        "ncell": ncell, "ms_total": ms_total, "ms_per_step": ms_total / steps, "wall": wall,
        "mlups": ncell * steps / (ms_total / 1e3) / 1e6, "dominant": timed[dom_q], "ktimes": ktimes,
        "kernel_bytes": [r[2] for r in timed], "graph_ms_per_step": graph_ms,
        "diag": {"finite": d["finite"], "steps_run": d["step"],
                 "mass_drift": abs(d["mass"] - d0["mass"]) / d0["mass_abs0"]},
    }


# the paper's timing case: 120^3, 8 steps, four CPU nodes (hardware not
# stated), wall time per CH lattice; throughput derived as cells x steps / s
PAPER_COALESCENCE_S = {15: 19.1, 19: 19.5, 27: 19.7}


def coalescence_bench(steps: int, warmup: int, precisions=("fp64", "fp32"), lattices=(15, 19, 27)) -> dict:
    """The paper's 3-D drop-coalescence timing case (120^3 eighth domain,
    symmetry planes on all faces, Oh 0.119, N_L 40, N_t 400, CH convection
    in the advective form) per CH lattice and precision, with the paper's
    own derived throughput beside it.  With D3Q15 these parameters put the
    grid-scale CH mode beyond the RK4 stability limit (growth 1.18 per
    step from round-off), so every run is timed from the initial state over
    a bounded number of steps (the paper timed 8) and checked finite."""
    if warmup + steps > 150:
        raise ValueError("coalescence timing: at most 150 steps from the initial state")
    from paper_2011_00814_amd import workloads as W

    rows = []
    for prec in precisions:
        for lat in lattices:
            r = time_solver(W.coalescence_3d(n=120, lattice=lat, precision=prec), steps, warmup,
                            graph_context=False)
            paper = 120 ** 3 * 8 / PAPER_COALESCENCE_S[lat] / 1e6
            rows.append({"precision": prec, "lattice": f"D3Q{lat}", "mlups": round(r["mlups"], 1),
                         "ms_per_step": round(r["ms_per_step"], 4),
                         "paper_mlups_derived": round(paper, 3), "ratio_vs_paper": round(r["mlups"] / paper, 1),
                         "finite": r["diag"]["finite"], "mass_drift": r["diag"]["mass_drift"]})
    return {"workload": "3D drop coalescence 120^3 (eighth domain, symmetry planes), Oh 0.119, "
                        "r_rho 50, r_eta 58.8, N_L 40, Cn 0.1, Pe 8e3",
            "steps": steps, "rows": rows,
            "paper_context": "paper: 19.1 / 19.5 / 19.7 s for 8 steps of 120^3 (D3Q15 / 19 / 27) on four "
                             "CPU nodes, precision not stated"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the CPU oracle on every configuration, all cores and one core (about 2 min)")
    ap.add_argument("--workload", choices=("bubble3d", "ensemble", "learned", "coalescence", "rt2d"),
                    default="bubble3d")
    ap.add_argument("--learned-summary", type=int, default=1,
                    help="include a reduced learned-correction run in the default line (0: skip)")
    ap.add_argument("--ensemble-steps", type=int, default=200,
                    help="steps of the ensemble summary in the default line (0: skip)")
    ap.add_argument("--learned-reduced", action="store_true",
                    help="--workload learned at the reduced size of the default line's summary")
    ap.add_argument("--coalescence-steps", type=int, default=100,
                    help="steps of the paper's 120^3 coalescence timing case in the default line (0: skip)")
    ap.add_argument("--learned-no-rollout", action="store_true",
                    help="--workload learned: train on one-step pairs only (no pairs from corrected rollouts)")
    ap.add_argument("--learned-iters", type=int, default=0,
                    help="--workload learned: training iterations (0: the default of the workload)")
    ap.add_argument("--learned-checkpoints", type=int, default=0,
                    help="--workload learned: evaluation times (0: the default of the workload)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="print the HBM streaming probe (read / write / copy) over a sweep of work-group counts")
    ap.add_argument("--stream-calib", action="store_true",
                    help="one launch each of the streaming read / write / copy kernels on 1 GiB buffers "
                         "(calibration of HBM byte counters under a profiler)")
    ap.add_argument("--no-stream-probe", action="store_true",
                    help="leave the streaming probe out of the default line (profiled runs)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe_mb:
        # a plain device copy: calibrates the HBM byte counters (3 launches
        # under a profiler) and measures the practical copy bandwidth
        n = args.copy_probe_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "launches": 23, "ms_per_copy": round(ms, 4),
                          "copy_gbs": round(8 * n / (ms * 1e-3) / 1e9, 1)}), flush=True)
        return

    from paper_2011_00814_amd import gpe

    gpe.lib()  # fails loudly if the HIP library is not built
    if args.stream_calib:
        print(json.dumps({"stream_calib": hbm_probe(mib=1024, reps=1, warm=0), "bytes": 1 << 30}), flush=True)
        return
    if args.stream_probe:
        ncu = torch.cuda.get_device_properties(0).multi_processor_count
        for wg in (2 * ncu, 4 * ncu, 8 * ncu, 16 * ncu, 32 * ncu):
            print(json.dumps({"stream_probe": hbm_probe(workgroups=wg), "cus": ncu}), flush=True)
        return
    if args.workload == "learned":
        roll = not args.learned_no_rollout
        progress = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
        kw = dict(rollout=roll, log=progress)
        if args.learned_reduced:
            kw.update(ntrain=32, fine_steps=4000, n_snap=16, iters=800, neval=8)
        if args.learned_iters > 0:
            kw["iters"] = args.learned_iters
        if args.learned_checkpoints > 0:
            kw["checkpoints"] = args.learned_checkpoints
        r = learned_bench(**kw)
        print(json.dumps({
            "metric": "learned-coarse speedup vs the fine solver at interface-position error on the coarse grid",
            "value": r["speedup_vs_fine"], "unit": "x", "n_gpus": 1, "steps": r["coarse_steps"], "warmup": 0,
            "ms_per_step": round(r["coarse_net_ms"] / r["coarse_steps"], 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
            "config": {"workload": r["workload"]}, "learned": r}), flush=True)
        return
    if args.workload == "coalescence":
        prec = args.precision if "--precision" in sys.argv else "fp64"
        steps = args.steps if "--steps" in sys.argv else 100
        warm = args.warmup if "--warmup" in sys.argv else 2
        r = coalescence_bench(steps, warm, precisions=(prec,), lattices=(15,))
        row = r["rows"][0]
        print(json.dumps({
            "metric": "MLUPS of the full RK3 step, the paper's 3-D coalescence timing case (120^3, D3Q15)",
            "value": row["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": warm,
            "ms_per_step": row["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            # the paper's figure for this workload is from four CPU nodes:
            # context, not a target
            "vs_baseline": row["ratio_vs_paper"],
            "dtype": "f64" if prec == "fp64" else "f32", "data": "synthetic",
            "config": {"workload": r["workload"] + ", D3Q15"}, "coalescence": r}), flush=True)
        return
    if args.workload == "rt2d":
        from paper_2011_00814_amd import workloads as W

        precs = (args.precision,) if "--precision" in sys.argv else ("fp32", "fp64")
        steps = args.steps if "--steps" in sys.argv else 2000
        rows = []
        for prec in precs:
            prob, _ = W.rayleigh_taylor_2d(precision=prec, in_kernel_init=True)
            r = time_solver(prob, steps, args.warmup)
            rows.append({"precision": prec, "mlups": round(r["ncell"] / (r["graph_ms_per_step"] * 1e-3) / 1e6, 1),
                         "graph_ms_per_step": round(r["graph_ms_per_step"], 5),
                         "eager_ms_per_step": round(r["ms_per_step"], 5),
                         "kernels_us": {k[0]: round(k[1] * 1000, 1) for k in r["ktimes"]},
                         "finite": r["diag"]["finite"], "mass_drift": r["diag"]["mass_drift"]})
        print(json.dumps({
            "metric": "MLUPS of the full RK3 step, 2-D Rayleigh-Taylor 256x1024 (graph-replayed steps)",
            "value": rows[0]["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "ms_per_step": rows[0]["graph_ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" if precs[0] == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": "2-D Rayleigh-Taylor 256x1024, periodic x, no-slip walls in y, Atwood 0.5, "
                                   "Re 3000, D2Q9, RK3 flow + RK2 CH"}, "rt2d": rows}), flush=True)
        return
    if args.workload == "ensemble":
        steps = args.steps if "--steps" in sys.argv else 5000
        r = ensemble_bench(steps, args.warmup, args.precision)
        print(json.dumps({
            "metric": "aggregate cell updates/s, batched 2-D ensemble vs sequential single-grid runs",
            "value": r["aggregate_cell_updates_per_s"], "unit": "cell updates/s", "n_gpus": 1,
            "steps": steps, "warmup": args.warmup, "ms_per_step": r["ms_per_batch_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": r["workload"]}, "ensemble": r}), flush=True)
        return
    copy_gbs = copy_bandwidth()
    probe = None if args.no_stream_probe else hbm_probe()
    prob = problem(args.n, args.precision)
    ncell = args.n ** 3
    r = time_solver(prob, args.steps, args.warmup)
    ktimes, ms_per_step, mlups = r["ktimes"], r["ms_per_step"], r["mlups"]
    wall, graph_ms_per_step, d = r["wall"], r["graph_ms_per_step"], r["diag"]

    dom = r["dominant"]
    achieved = dom[2] / (dom[1] * 1e-3) / 1e9
    traffic = measured_traffic(dom[0], args.precision)
    step_bytes = sum(r["kernel_bytes"])
    step_gbs = step_bytes / (ms_per_step * 1e-3) / 1e9

    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D rising bubble {args.n}^3, no-slip walls, density/viscosity ratio 10, "
                        "Eo 10, Mo 1e-4, W 2, M 0.02, D3Q15 CH stencils, RK3 flow + RK4 CH",
            "grid": [args.n] * 3,
            "precision": args.precision,
            "wall_s": round(wall, 3),
            "graph_replay_ms_per_step": round(graph_ms_per_step, 4),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom[0],
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "copy_gbs_measured": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
            "stream_probe": probe,
            "frac_of_stream_copy": round(achieved / probe["copy_gbs"], 4) if probe else None,
            "algorithmic_bytes_per_launch": dom[2],
            "launch_ms": round(dom[1], 5),
        },
        "step_roofline": {
            "algorithmic_bytes_per_step": step_bytes,
            "bytes_per_cell_step": step_bytes / ncell,
            "achieved": round(step_gbs, 1),
            "frac": round(step_gbs / HBM_PEAK_GBS, 4),
            "frac_of_copy": round(step_gbs / copy_gbs, 4),
            "frac_of_stream_copy": round(step_gbs / probe["copy_gbs"], 4) if probe else None,
            "roofline_mlups": round(HBM_PEAK_GBS * 1e9 / (step_bytes / ncell) / 1e6, 1),
        },
        # every kernel, from the steps after the timed region with events around each launch
        "kernels": [{"name": r[0], "ms": round(r[1], 5), "bytes": r[2],
                     "gbs": round(r[2] / (r[1] * 1e-3) / 1e9, 1)} for r in ktimes],
        "diag": d,
    }
    if args.coalescence_steps > 0:
        line["coalescence"] = coalescence_bench(args.coalescence_steps, 2)
    if args.ensemble_steps > 0:
        line["ensemble"] = ensemble_bench(args.ensemble_steps, 10, args.precision, baseline_steps=50)
    if args.learned_summary and args.precision == "fp32":
        line["learned"] = learned_bench(ntrain=32, fine_steps=4000, n_snap=16, iters=800, neval=8)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.n, args.precision)
    if args.cpu_configs:
        line["cpu_configs"] = cpu_configs()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
