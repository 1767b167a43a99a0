"""Throughput of the PSM hot path on one MI355X.

A step is one pass of the whole hot path over the lattice: geometry_map_step
(B(t) from the rotated geometry field), psm_stream_collide (fused in-place
stream + TRT/PSM collision) and body_force_torque (FP64 per-body sum).
MLUPS = cells * steps / wall time of the timed steps (inputs resident in HBM).

The dominant kernel's roofline: algorithmic bytes per cell update
(2 * Q * sizeof(storage) PDF traffic + 4 B solid fraction) times cells,
divided by its average launch time measured with HIP events on the launch
stream, against 8 TB/s.  HBM traffic per launch comes from a committed
rocprofv3 FETCH_SIZE/WRITE_SIZE record when the kernel source is unchanged
since it was taken.

The CPU baseline is the FP64 oracle timed on the host cores on a bounded
sample (a few full-size steps) of the same workload, on all threads and on
one; the same steps run on the GPU with FP32 and FP16 storage give the
accuracy fields (velocity rel. L2, torque series) against it.
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

METRIC = "MLUPS + % HBM roofline, PSM vs plain LBM, FP32/FP16 vs FP64 oracle"
LAYOUT = "blocked"  # PDF buffer layout of every field the benchmark builds (--layout)


def lay(wl):
    """The workload with the benchmark's PDF layout."""
    import dataclasses

    return dataclasses.replace(wl, layout=LAYOUT)
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ["paper_2502_20049_amd/csrc/k_stream_collide.hpp", "paper_2502_20049_amd/csrc/k_sc_launch.inc",
                  "paper_2502_20049_amd/csrc/psm_internal.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name):
    import psm_inputs as pi

    if name == "ellipsoid_channel_256":
        return lay(pi.workload_ellipsoid_channel(256, "f32", steps=2000, s=3))
    if name == "cror_768x384x384":
        return lay(pi.workload_cror(storage="f16"))
    if name == "capacity_1024":
        return lay(pi.workload_capacity())
    raise SystemExit(f"unknown workload {name}")


def bytes_per_cell(q, storage, psm=True):
    sz = {"f64": 8, "f32": 4, "f16": 2}[storage]
    return 2 * q * sz + (4 if psm else 0)


def run_steps(field, t0, n, events=None, map_events=None, fused=True):
    """Steps t0 .. t0+n-1.  fused: one psm_step per step (mapping,
    stream-collide and F/T sum in one call); else the separate calls
    geometry_map_step / psm_stream_collide / body_force_torque, with HIP
    events on the launch stream around the first two when given."""
    for i in range(n):
        t = t0 + i
        poses = field.poses(t) if field.nb else None
        if fused:
            field.step(t, ft=field.ft if field.nb else None)
            continue
        if field.nb and (field.remap_every_step or not field._mapped_once):
            if map_events is not None:
                map_events[i][0].record()
            field.map(t, poses)
            if map_events is not None:
                map_events[i][1].record()
        if events is not None:
            events[i][0].record()
        field.collide(t, poses)
        if events is not None:
            events[i][1].record()
        if field.nb:
            field.force_torque()
    return t0 + n


def time_field(field, steps, warmup, t0=0):
    """Wall time of `steps` whole steps (psm_step) after `warmup` untimed ones."""
    import torch

    t = run_steps(field, t0, warmup)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t = run_steps(field, t, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - w0, t


def time_kernels(field, steps, t0):
    """Average launch times (ms) of psm_stream_collide and geometry_map_step:
    HIP events on the launch stream around `steps` back-to-back calls of
    each (stream-collide for steps t .. t+steps-1 on the fractions of the
    last mapping, then the mapping of the same steps)."""
    import torch

    t = run_steps(field, t0, 5, fused=False)
    steps += steps & 1  # as many even as odd steps
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    e[0].record()
    for i in range(steps):
        field.collide(t + i, field.poses(t + i) if field.nb else None)
    e[1].record()
    if field.nb and field.remap_every_step:
        for i in range(steps):
            field.map(t + i, field.poses(t + i))
    e[2].record()
    torch.cuda.synchronize()
    sc_ms = e[0].elapsed_time(e[1]) / steps
    map_ms = e[1].elapsed_time(e[2]) / steps if field.nb and field.remap_every_step else 0.0
    return sc_ms, map_ms


def copy_probe(nbytes=4 << 30, reps=20):
    import torch

    from paper_2502_20049_amd import sim

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        sim.stream_copy(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sim.stream_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * nbytes / s / 1e9


def traffic_record(kname, wname):
    p = os.path.join(ROOT, "profiles", f"traffic_{kname}_{wname}.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        rec = json.load(fh)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def s_sweep(steps=200):
    """The channel workload at supersampling s = 0..3 (PSM + mapping every
    step), with every sub-sample rotated (sN) and, for s >= 1, with the block
    reading of the mapping (sN_block: centre rotated, axis-aligned block)."""
    import dataclasses

    import torch

    import psm_inputs as pi
    from paper_2502_20049_amd import sim

    out = {}
    for s, reading in ((0, 0), (1, 0), (2, 0), (3, 0), (1, 1), (2, 1), (3, 1)):
        wl = dataclasses.replace(lay(pi.workload_ellipsoid_channel(256, "f32", steps=steps, s=s)), map_reading=reading)
        f = sim.Field(wl)
        wall, t = time_field(f, steps, 20)
        sc, mp = time_kernels(f, 100, t)
        out[f"s{s}" + ("_block" if reading else "")] = {
            "mlups": round(wl.n_cells * steps / wall / 1e6, 1), "map_ms": round(mp, 5), "collide_ms": round(sc, 5)}
        del f
        torch.cuda.empty_cache()
    return out


def node_benchmark(steps=600):
    """The paper's node-level comparison (section V) on one GPU, periodic
    lattices (inflow / outflow excluded, as there): plain LBM; LBM with the
    no-slip treatment of the stationary voxelised geometry (lbm_set_obstacle);
    PSM with the geometry mapped once; PSM with the geometry rotating and
    mapped every step at s = 0, 1 and the workload's own s.  Scene B: the
    256^3 channel's ellipsoid (a small body in a large lattice); scene A: the
    256^3 box filled by an 8-blade rotor of radius 120 (118k triangles)."""
    import dataclasses

    import torch

    import psm_inputs as pi
    from paper_2502_20049_amd import sim

    def mlups(field, wl):
        wall, _ = time_field(field, steps, 20)
        return round(wl.n_cells * steps / wall / 1e6, 1)

    out = {}
    scenes = {"B_ellipsoid_channel_256": lay(pi.workload_ellipsoid_channel(256, "f32", steps=steps, s=3)),
              "A_rotor_box_256": lay(pi.workload_rotor_box(steps=steps))}
    for name, wl in scenes.items():
        wl = dataclasses.replace(wl, bc=("periodic",) * 6, u_in=(0.0, 0.0, 0.0))
        r = {}
        f = sim.Field(wl, psm=False)
        r["lbm"] = mlups(f, wl)
        solid = sim.voxelize_obstacle(wl, 0)
        r["obstacle_cells"] = int(solid.sum().item())
        r["lbm_noslip_near_cells"] = f.set_obstacle(solid)
        r["lbm_noslip_static"] = mlups(f, wl)
        del f, solid
        torch.cuda.empty_cache()
        fs = sim.Field(wl, remap_every_step=False)
        r["psm_static"] = mlups(fs, wl)
        del fs
        torch.cuda.empty_cache()
        own = wl.bodies[0].s
        for sv in sorted({0, 1, own}):
            w2 = dataclasses.replace(wl, bodies=[dataclasses.replace(b, s=sv) for b in wl.bodies])
            fr = sim.Field(w2)
            r[f"psm_rotating_s{sv}"] = mlups(fr, w2)
            del fr
            torch.cuda.empty_cache()
        r["psm_rotating_over_lbm_noslip"] = round(r[f"psm_rotating_s{own}"] / r["lbm_noslip_static"], 4)
        out[name] = r
    return out


def cumulant_cror(steps=200):
    """The counter-rotating rotor pair (768 x 384 x 384 D3Q27, s = 2) with FP16
    storage and the TRT fluid collision, the cumulant one (the paper's
    performance operator), and TRT with FP32 storage: whole-step MLUPS and the
    stream-collide launch."""
    import dataclasses

    import torch

    import psm_inputs as pi
    from paper_2502_20049_amd import sim

    out = {}
    base = lay(pi.workload_cror(storage="f16"))
    for key, coll, storage in (("trt", "trt", "f16"), ("cumulant", "cumulant", "f16"), ("trt_f32_storage", "trt", "f32")):
        wl = dataclasses.replace(base, collision=coll, storage=storage)
        f = sim.Field(wl)
        wall, t = time_field(f, steps, 10)
        sc, mp = time_kernels(f, 50, t)
        gbs = bytes_per_cell(wl.q, wl.storage) * wl.n_cells / sc / 1e6
        out[key] = {"mlups": round(wl.n_cells * steps / wall / 1e6, 1), "collide_ms": round(sc, 4),
                    "collide_gbs": round(gbs, 1), "collide_frac_of_8tbs": round(gbs / PEAK_HBM_GBS, 4),
                    "map_ms": round(mp, 4), "storage": storage}
        del f
        torch.cuda.empty_cache()
    out["case"] = base.name + ", two counter-rotating 8-blade rotors, s=2; TRT and cumulant with FP16 storage, " \
                              "TRT with FP32 storage"
    return out


def settling_sphere(steps=4000):
    """Two-way coupling on the section IV setup: a sphere (d = 20 cells, density
    ratio 1.16) released from rest near the top of a closed 135 x 135 x 216 box,
    SRT (tau = 0.575), SC2, s = 2; per step psm_coupled_step (map, stream-collide,
    F/T read back, host integrator)."""
    import torch

    import psm_inputs as pi
    from paper_2502_20049_amd import sim

    wl, rg = pi.workload_settling_sphere(steps=steps)
    wl = lay(wl)
    f = sim.Field(wl)
    states = sim.rigid_states([rg])
    vz = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(steps):
        ft = f.coupled_step(t, states)
        vz.append(states[0].V[2])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same lattice and sphere with prescribed motion (no read-back): the
    # cost of the per-step host round trip
    del f
    torch.cuda.empty_cache()
    fp = sim.Field(wl)
    wall_p, _ = time_field(fp, 500, 20)
    del fp
    torch.cuda.empty_cache()
    nu = (wl.tau - 0.5) / 3.0
    vmax = min(vz)
    k = vz.index(vmax)
    return {"case": f"{wl.name}, SRT tau {wl.tau}, SC2, s=2, {steps} coupled steps",
            "mlups": round(wl.n_cells * steps / wall / 1e6, 1), "ms_per_step": round(wall / steps * 1e3, 4),
            "prescribed_motion_ms_per_step": round(wall_p / 500 * 1e3, 4),
            "max_settling_velocity": round(vmax, 6), "at_step": k, "Re_at_max": round(abs(vmax) * 20.0 / nu, 2),
            "z_final": round(states[0].X[2], 3),
            "net_force_over_weight_last_step": round((ft[0, 2] + rg["F_ext"][2]) / abs(rg["F_ext"][2]), 5)}


def adjoint_rate(steps=800, window=200):
    """Torque-gradient sweep on the 128^3 4-blade rotor: J = mean axial torque
    over the last 200 of 800 steps, in both trajectory modes: sqrt(T)
    checkpoints (forward with checkpoints; backward = recompute + store +
    adjoint, about 472 B per cell-step) and, where the device holds it, the
    whole trajectory kept by the forward (forward + state copies; backward =
    adjoint steps only, about 250 B per cell-step).  Wall times of a second
    sweep; the two modes' J and gradients are bit-identical."""
    import numpy as np
    import torch

    import psm_inputs as pi
    from paper_2502_20049_amd import adjoint

    wl = lay(pi.workload_adjoint_rotor(steps=steps))
    w = np.zeros(steps)
    w[-window:] = 1.0 / window
    N = wl.n_cells
    out = {"case": f"{wl.name}, {steps} steps, window {window}"}
    res = {}
    for mode in ("sqrtT", "whole"):
        torch.cuda.empty_cache()
        obj = adjoint.TorqueAdjoint(wl, steps, w, store_all=None if mode == "whole" else False)
        if mode == "whole" and not obj.store_all:
            out[mode] = {"skipped": "trajectory larger than half the free device memory"}
            continue
        obj.forward()
        obj.backward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = obj.forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gB, gW, _ = obj.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res[mode] = (J, gW, gB.clone())
        bpcs = 472 if mode == "sqrtT" else 250
        rate = N * steps / (t2 - t1)
        out[mode] = {"J": J, "dJ_dOmega": gW, "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
                     "backward_mcell_steps_per_s": round(rate / 1e6, 1),
                     "backward_bytes_per_cell_step": bpcs,
                     "backward_frac_of_8TBs": round(rate * bpcs / 8e12, 3)}
        if mode == "sqrtT":
            out[mode]["checkpoint_segment"] = obj.L
        else:
            out[mode]["trajectory_GB"] = round(obj.trajectory_bytes / 1e9, 1)
        del obj, gB
    if len(res) == 2:
        a, b = res["sqrtT"], res["whole"]
        out["modes_bit_identical"] = bool(a[0] == b[0] and a[1] == b[1] and torch.equal(a[2], b[2]))
    out["sqrtT_ceiling_mcell_steps_per_s"] = round(8e12 / 472 / 1e6, 0)
    del res
    torch.cuda.empty_cache()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, min_seconds=12.0, single_core_steps=2):
    """The FP64 oracle on the host cores, full-size steps of the same workload
    (map + collide/stream + F/T) from rest, two at a time until about
    min_seconds have passed, on every thread the oracle gets (OMP_NUM_THREADS,
    else all cores), then `single_core_steps` more on one thread.  Returns
    the baseline record and the oracle state (for the accuracy check)."""
    import oracle

    oracle.build(force=False)
    run = oracle.Run(wl)
    threads = oracle.threads()
    t0 = time.perf_counter()
    nsteps = 0
    while True:
        run.advance(2)
        nsteps += 2
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    oracle.set_threads(1)
    t1 = time.perf_counter()
    one = oracle.Run(wl)
    one.advance(single_core_steps)
    dt1 = time.perf_counter() - t1
    del one
    oracle.set_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    rec = {"value": round(wl.n_cells * nsteps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{nsteps} full-size steps (map + collide/stream + F/T) of {wl.name} from rest, FP64, "
                     f"{dt:.1f} s on {threads} threads",
           "single_core": {"value": round(wl.n_cells * single_core_steps / dt1 / 1e6, 3), "unit": "MLUPS",
                           "sample": f"{single_core_steps} full-size steps on 1 thread, {dt1:.1f} s"},
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "cpus_available": affinity}
    return rec, run, nsteps


def accuracy_vs_oracle(wl, run, nsteps):
    """The oracle's steps from rest (the CPU baseline's) repeated on the GPU
    with FP32 and FP16 storage: velocity rel. L2 over all cells after the
    last step and the torque series' max error relative to max |T|."""
    import numpy as np
    import torch

    from paper_2502_20049_amd import sim

    _, uo = run.macro()
    To = np.array(run.ft)[:, 0, 3:]
    out = {"steps": nsteps, "reference": "FP64 oracle, same steps from rest"}
    for storage in ("f32", "f16"):
        f = sim.Field(wl, storage=storage)
        T = []
        for t in range(nsteps):
            f.step(t)
            T.append(f.force_torque()[0, 3:].cpu().numpy().copy())
        _, u = f.macroscopic(nsteps)
        torch.cuda.synchronize()
        u = u.cpu().numpy()
        T = np.array(T)
        out[storage] = {"u_rel_l2": float(f"{np.linalg.norm(u - uo) / np.linalg.norm(uo):.3e}"),
                        "torque_rel_max": float(f"{np.abs(T - To).max() / np.abs(To).max():.3e}")}
        del f
        torch.cuda.empty_cache()
    return out


def capacity_run(steps=20, warmup=3):
    """The 1024^3 capacity configuration (FP32 in place, two counter-rotating
    6-blade rotors of radius 300, s = 2): whole-step MLUPS and the
    stream-collide launch against the roofline."""
    import torch

    import psm_inputs as pi
    from paper_2502_20049_amd import sim

    # SoA: on 1024^3 the blocked layout measured 2-7% slower (rows per block
    # 1-16, one process), unlike the 256^3 and 768-wide lattices
    wl = pi.workload_capacity()
    t0 = time.perf_counter()
    f = sim.Field(wl)
    setup = time.perf_counter() - t0
    wall, t = time_field(f, steps, warmup)
    sc, mp = time_kernels(f, 6, t)
    bpc = bytes_per_cell(wl.q, wl.storage)
    out = {"case": f"{wl.name}, FP32 in place (SoA layout), two 6-blade rotors r=300, s=2, {steps} steps",
           "mlups": round(wl.n_cells * steps / wall / 1e6, 1), "collide_ms": round(sc, 3), "map_ms": round(mp, 3),
           "collide_gbs": round(bpc * wl.n_cells / sc / 1e6, 1),
           "collide_frac_of_8tbs": round(bpc * wl.n_cells / sc / 1e6 / PEAK_HBM_GBS, 4),
           "setup_s": round(setup, 1)}
    del f
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ellipsoid_channel_256")
    ap.add_argument("--storage", choices=["f64", "f32", "f16"], default=None,
                    help="PDF storage type (default: the workload's)")
    ap.add_argument("--layout", choices=["soa", "blocked"], default="blocked",
                    help="PDF buffer layout of every field (default: blocked)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sequential", action="store_true",
                    help="run every launch of a step on one stream (PSM_OPT_CONCURRENT = 0)")
    ap.add_argument("--no-extras", action="store_true", help="skip the variants, the copy probe and the other workloads")
    ap.add_argument("--only-psm", action="store_true", help="time the PSM path only (for profiling)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the torque-gradient sweep on the 128^3 rotor (for profiling)")
    ap.add_argument("--node-only", action="store_true",
                    help="run only the paper's node-level comparison (LBM, LBM + no-slip obstacle, PSM static, "
                         "PSM rotating)")
    ap.add_argument("--settling-only", action="store_true",
                    help="run only the two-way coupled settling sphere (section IV setup)")
    ap.add_argument("--cumulant-only", action="store_true",
                    help="run only the TRT / cumulant comparison on the counter-rotating rotor pair")
    ap.add_argument("--sweep-only", action="store_true",
                    help="run only the supersampling sweep (s = 0..3, both mapping readings) on the channel")
    ap.add_argument("--copy-only", action="store_true",
                    help="run only the device copy probe (1 GiB read + 1 GiB written per launch): the "
                         "calibration for rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    global LAYOUT
    LAYOUT = args.layout
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the PSM hot path here is single-GPU (no sharding or collectives); "
              "run with --gpus 1", file=sys.stderr)
        raise SystemExit(2)

    import torch

    from paper_2502_20049_amd import sim

    torch.cuda.set_device(0)
    if args.sequential:
        sim.CONCURRENT_DEFAULT = False
    if args.adjoint_only:
        print(json.dumps(adjoint_rate()), flush=True)
        return
    if args.node_only:
        print(json.dumps(node_benchmark()), flush=True)
        return
    if args.settling_only:
        print(json.dumps(settling_sphere()), flush=True)
        return
    if args.cumulant_only:
        print(json.dumps(cumulant_cror()), flush=True)
        return
    if args.sweep_only:
        print(json.dumps(s_sweep()), flush=True)
        return
    if args.copy_only:
        bw = copy_probe(nbytes=1 << 30, reps=5)
        print(json.dumps({"copy_probe_gbs": round(bw, 1), "bytes_read_per_launch": 1 << 30,
                          "bytes_written_per_launch": 1 << 30}), flush=True)
        return
    wl = workload(args.workload)
    if args.storage:
        wl.storage = args.storage
    storage = wl.storage
    f = sim.Field(wl)
    wall, t_end = time_field(f, args.steps, args.warmup)
    sc_ms, map_ms = time_kernels(f, min(args.steps, 300), t_end)
    N = wl.n_cells
    mlups = N * args.steps / wall / 1e6
    bpc = bytes_per_cell(wl.q, storage)
    achieved = bpc * N / (sc_ms / 1e3) / 1e9
    traffic = traffic_record("psm_stream_collide", args.workload + (f"_{storage}" if args.storage else ""))
    line = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"f32": "f32", "f16": "f32 (f16 storage)",
                                                            "f64": "f64"}[storage],
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": N, "q": wl.q, "storage": storage, "layout": wl.layout,
                   "launches": "one stream" if args.sequential else "solid and face rows on a second stream",
                   "mapping": "next step mapped during this one (psm_step_ahead)" if f.map_ahead else "psm_step",
                   "bodies": len(wl.bodies),
                   "supersampling_s": [b.s for b in wl.bodies], "bc": list(wl.bc), "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None if traffic is None else round(traffic, 0),
                     "kernel": "psm_stream_collide", "algorithmic_bytes_per_cell": bpc,
                     "avg_launch_ms": round(sc_ms, 5)},
        "kernels_ms": {"psm_stream_collide": round(sc_ms, 5), "geometry_map_step": round(map_ms, 5),
                       "note": "HIP events around back-to-back calls of each after the timed steps (which "
                               "run whole steps)"},
    }
    del f
    torch.cuda.empty_cache()
    if not args.no_extras and not args.only_psm:
        extras = {}
        fl = sim.Field(wl, psm=False)
        wall_l, tl = time_field(fl, min(args.steps, 500), 20)
        sc_l, _ = time_kernels(fl, 100, tl)
        extras["plain_lbm_same_storage"] = {"mlups": round(N * min(args.steps, 500) / wall_l / 1e6, 1),
                                            "kernel_ms": round(sc_l, 5),
                                            "gbs": round(bytes_per_cell(wl.q, storage, False) * N / sc_l / 1e6, 1)}
        del fl
        torch.cuda.empty_cache()
        fs = sim.Field(wl, remap_every_step=False)
        wall_s, _ = time_field(fs, min(args.steps, 500), 20)
        extras["psm_static_geometry"] = {"mlups": round(N * min(args.steps, 500) / wall_s / 1e6, 1)}
        del fs
        torch.cuda.empty_cache()
        for alt in [a for a in ("f16", "f32", "f64") if a != storage]:
            fa = sim.Field(wl, storage=alt)
            wall_a, ta = time_field(fa, min(args.steps, 500), 20)
            sc_a, _ = time_kernels(fa, 100, ta)
            gbs_a = bytes_per_cell(wl.q, alt) * N / sc_a / 1e6
            extras[f"psm_{alt}_storage"] = {"mlups": round(N * min(args.steps, 500) / wall_a / 1e6, 1),
                                            "kernel_ms": round(sc_a, 5), "gbs": round(gbs_a, 1),
                                            "frac_of_8tbs": round(gbs_a / PEAK_HBM_GBS, 4),
                                            "algorithmic_bytes_per_cell": bytes_per_cell(wl.q, alt)}
            del fa
            torch.cuda.empty_cache()
        bw = copy_probe()
        extras["copy_probe_gbs"] = round(bw, 1)
        extras["psm_frac_of_copy_bw"] = round(achieved / bw, 4)
        extras["supersampling_sweep"] = s_sweep()
        extras["node_benchmark"] = node_benchmark()
        extras["adjoint_rotor_128"] = adjoint_rate()
        extras["settling_sphere"] = settling_sphere()
        extras["cumulant_vs_trt_cror"] = cumulant_cror()
        extras["capacity_1024"] = capacity_run()
        line["extras"] = extras
    if not args.no_cpu_baseline:
        rec, run, nsteps = cpu_baseline(wl)
        line["cpu_baseline"] = rec
        line["accuracy_vs_fp64_oracle"] = accuracy_vs_oracle(wl, run, nsteps)
        del run
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
