#!/usr/bin/env python3
"""Benchmark of the LEE lattice Boltzmann hot path on one MI355X.

Workload (default): 3D LEE-LBM on D3Q7, 256^3 periodic cells, 8 seeded Gaussian pressure
pulses (amplitude 1e-3, sigma 12 cells, isentropic, zero velocity), tau = 1/2, 500 steps,
FP32 population storage.  A "step" is one fused pull-stream + moments + equilibrium +
relaxation pass over all cells.  The initial state is resident in HBM before timing starts.
Besides the FP32 headline the line reports every storage mode with its error against the FP64
path, the roofline of the step kernel, the FP64 CPU oracle as a baseline, and the learned
non-reflecting closure on its 2D open-box workload (reflection coefficient and step time
against the zero and sponge closures and the wider periodic run) and the step times of its 3D
open-box workload.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % peak HBM GB/s; FP16-store & learned-NRBC vs plain FP32 at stated err"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--modes", default="f32,f16,bf16,i16,e3m12,f64", help="storage modes to time and compare")
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions of the K steps (median reported)")
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="budget of the oracle CPU baseline (half on one thread, half on all cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nrbc", action="store_true", help="skip the learned-closure legs (2D and 3D)")
    ap.add_argument("--closure-only", action="store_true",
                    help="only the learned-closure leg (for rocprofv3); its result on stdout")
    ap.add_argument("--closure3d-only", action="store_true",
                    help="only the 3D learned-closure step times (for rocprofv3); its result on stdout")
    ap.add_argument("--profile-only", action="store_true", help="only the timed steps of --storage (for rocprofv3)")
    ap.add_argument("--with-copy", action="store_true",
                    help="with --profile-only: also run the plain copy kernel on one state buffer's bytes "
                         "(the reference point for counter calibration)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    """Hash of the sources of the step kernels (the device code the counters measured)."""
    h = hashlib.sha256()
    for f in ("kernels.hpp", "codec.hpp", "velsets.hpp", "temporal.hpp"):
        with open(os.path.join(ROOT, "paper_1601_08103_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_counters(storage: str, n: int, variant: str):
    """HBM bytes per launch measured with rocprofv3 counters, if they were taken on the current
    kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_step_{variant}_d3q7_{n}_{storage}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    try:
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def nrbc_leg():
    """The learned non-reflecting closure on its 2D workload (D2Q9 512^2 open box, 1536^2 periodic
    judge, 1024 steps) with the shipped weights (trained by the library's own kernels): reflection
    coefficient of the zero closure, two sponges (the wide one of the earlier comparisons and one
    that costs less per step than the network box) and the network closure on 32 held-out initial
    states, and the time per step of each box next to the judge's."""

    from paper_1601_08103_amd import lbm, nrbc

    path = os.path.join(ROOT, "paper_1601_08103_amd", "weights", "nrbc_D2Q9.npy")
    if not os.path.exists(path):
        return None
    P = np.load(path, allow_pickle=False)
    L, E, steps, seeds = 512, 1536, 1024, 32
    sponges = {"sponge": (96, 0.03), "sponge_W160": (160, 0.015)}
    info = lbm.lbm_lee_lattice_info("D2Q9")
    rng = np.random.default_rng(10_000)  # held-out states: training draws seeds below 10000
    ext = nrbc.judge_solver("D2Q9", "f32", E, 2)
    closures = ("zero", "sponge", "sponge_W160", "mlp")

    def kind(c):
        return "sponge" if c in sponges else c

    def layer(c):
        w, g = sponges.get(c, (0, 0.0))
        return w, (dict(sponge_width=w, sponge_sigma=g) if w else {})

    R = {c: [] for c in closures}
    first = None
    for _ in range(seeds):
        fields = nrbc.initial_fields("pulses", rng, info, L, 2)
        first = fields if first is None else first
        ref = nrbc.judge_reference("D2Q9", fields, L, E, steps, 8, ext=ext)  # one judge run per state
        for c in closures:
            R[c].append(nrbc.reflection_vs("D2Q9", kind(c), fields, ref, L, steps, 8, params=P, **layer(c)[1]))
        del ref
    # step times on live states: the judge holds the last run's state; each box starts from the
    # first held-out state (a sponge box from it on its inner box)
    times = {"extended_periodic": round(nrbc.time_solver(ext, 200), 5)}
    ext.close()
    for c in closures:
        W, kw = layer(c)
        times[c] = round(nrbc.time_per_step("D2Q9", (L + 2 * W,) * 2, bc=kind(c), params=P, fields=first,
                                            origin=(W, W) if W else None, **kw), 5)
    out = dict(workload=f"2D open box D2Q9 {L}^2 FP32, judge {E}^2 periodic, {steps} steps, {seeds} held-out "
                        "pulse states", weights="paper_1601_08103_amd/weights/nrbc_D2Q9.npy",
               sponges={c: dict(width=w, sigma=g) for c, (w, g) in sponges.items()},
               R_mean={c: round(float(np.mean(v)), 5) for c, v in R.items()},
               R_max={c: round(float(np.max(v)), 5) for c, v in R.items()}, ms_per_step=times)
    log("nrbc", out)
    return out


def nrbc3d_leg():
    """Step times of the 3D learned-closure workload: D3Q7 384^3 open boxes with FP16 storage, the
    zero closure and the network on all six faces (shipped weights), each started from the first
    held-out state (Gaussian pulses or a wave packet), next to the 1384^3 FP32 periodic judge that
    holds the same state in its centre.  Eager launches and graph replays.  (The reflection
    coefficients take ten seconds of judge per state and are left to `nrbc evaluate`.)"""

    import torch

    from paper_1601_08103_amd import lbm, nrbc

    path = os.path.join(ROOT, "paper_1601_08103_amd", "weights", "nrbc_D3Q7.npy")
    if not os.path.exists(path):
        return None
    P = np.load(path, allow_pickle=False)
    L, E = 384, 1384
    need = lbm.lbm_lee_state_bytes(lbm.make_desc("D3Q7", "f32", (E,) * 3))  # the judge in place, at least
    free, _ = torch.cuda.mem_get_info()
    if need > 0.9 * free:
        return dict(skipped=f"the {E}^3 FP32 judge needs {need / 2**30:.0f} GiB, {free / 2**30:.0f} GiB free")
    info = lbm.lbm_lee_lattice_info("D3Q7")
    fields = nrbc.initial_fields("mixed", np.random.default_rng(10_000), info, L, 3)
    ext = nrbc.judge_solver("D3Q7", "f32", E, 3)
    ext.reinit_region([(E - L) // 2] * 3, (L,) * 3, *fields)
    times = {"extended_periodic": round(nrbc.time_solver(ext, 24), 4)}
    graph = {"extended_periodic": round(nrbc.time_solver(ext, 24, graph=True), 4)}
    ext.close()
    del ext
    torch.cuda.empty_cache()
    for c in ("zero", "mlp"):
        for out, g in ((times, False), (graph, True)):
            out[c] = round(nrbc.time_per_step("D3Q7", (L,) * 3, bc=c, params=P, storage="f16", steps=120, graph=g,
                                              fields=fields), 4)
    res = dict(workload=f"3D open box D3Q7 {L}^3 FP16 storage, network on all six faces; judge {E}^3 FP32 "
                        "periodic; first held-out state", weights="paper_1601_08103_amd/weights/nrbc_D3Q7.npy",
               ms_per_step=times, ms_per_step_graph=graph)
    log("nrbc3d", res)
    return res


def host_cpu():
    """(nproc, CPUs this process may run on, CPU model name) of the host."""
    import platform
    import subprocess
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if not model:
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            model = platform.processor()
    return nproc, avail, model


def cpu_baseline(shape, rho, u, theta, budget_s):
    """The FP64 oracle (C stepper, OpenMP over rows) on the same workload, for a bounded number
    of steps: once on one thread and once on every CPU this process may use (capped at the 16 a
    one-GPU share of the host provides), each for about budget_s / 2 seconds."""
    from oracle import lattices as L
    from oracle import lbe

    lat = L.get("D3Q7")
    nproc, avail, model = host_cpu()
    all_threads = int(os.environ.get("LBM_ORACLE_THREADS", min(avail, 16)))
    g0 = lbe.equilibrium(lat, rho, u, theta)
    N = int(np.prod(shape))

    def leg(threads):
        g = g0
        steps = 0
        t0 = time.perf_counter()
        while True:
            g = lbe.steps(lat, g, 1, nthreads=threads)
            steps += 1
            el = time.perf_counter() - t0
            log(f"cpu baseline, {threads} thread(s): {steps} oracle steps, {el:.1f} s")
            if el >= budget_s / 2:
                break
        return steps, el

    s1, t1 = leg(1)
    sa, ta = leg(all_threads)
    return dict(value=round(N * sa / ta / 1e6, 3), unit="MLUPS", cores=all_threads, kind="oracle",
                sample=f"first {sa} steps of the same {shape[0]}^3 D3Q7 workload, FP64, push-form C stepper, "
                       f"{all_threads} OpenMP threads",
                single_thread=dict(value=round(N * s1 / t1 / 1e6, 3), unit="MLUPS", cores=1,
                                   sample=f"first {s1} steps, 1 thread"),
                nproc=nproc, cpus_available=avail, cpu_model=model)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1601_08103_amd import inputs, lbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lbm.load()
    torch.cuda.set_device(0)
    if args.closure_only:
        print(json.dumps(nrbc_leg()))
        return
    if args.closure3d_only:
        print(json.dumps(nrbc3d_leg()))
        return
    n = args.n
    shape = (n, n, n)
    N = n ** 3
    K, W = args.steps, args.warmup
    info = lbm.lbm_lee_lattice_info("D3Q7")

    log(f"building initial fields {shape}")
    p0 = inputs.gaussian_pressure(shape, inputs.pulses_3d(seed=0, n=n))
    rho, u, theta = inputs.fields_from_pressure(p0, info["rho0"], info["theta0"], info["gamma"])
    dev = torch.device("cuda")
    rho_d = torch.from_numpy(rho).to(dev)
    u_d = torch.from_numpy(u).to(dev)
    th_d = torch.from_numpy(theta).to(dev)
    stream = torch.cuda.current_stream()

    def steps_per_launch(variant):
        # the temporal-blocking variants read and write the state once per launch of 2 or 3 steps
        return {"tb2": 2, "tb3": 3}.get(variant, 1)

    reps = args.reps

    def timed_run(storage):
        """The workload's K steps, `reps` times from the initial state (HIP events on the library's
        stream around each K-step region): median time and median time per multi-step launch."""
        sim = lbm.Solver("D3Q7", storage, shape, rho_d, u_d, th_d, variant=args.variant)
        sim.step(W)
        # the multi-step variants run K // spl launches of spl steps and K % spl one-step
        # launches; the first part alone gives the time per launch of the dominant kernel
        spl = steps_per_launch(sim.variant)
        main = K - K % spl
        rep_ms, rep_launch = [], []
        for _ in range(reps):
            sim.reinit(rho_d, u_d, th_d)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev2 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            sim.step(main)
            ev1.record(stream)
            sim.step(K - main)
            ev2.record(stream)
            torch.cuda.synchronize()
            rep_ms.append(ev0.elapsed_time(ev2))
            rep_launch.append(ev0.elapsed_time(ev1) / (main // spl) if main else ev0.elapsed_time(ev2) / K)
        if not main:  # fewer steps than one multi-step launch: only one-step launches ran
            spl = 1
        ms, launch_ms = float(np.median(rep_ms)), float(np.median(rep_launch))
        log(f"{storage}: {K} steps, median of {reps}: {ms:.3f} ms ({', '.join('%.3f' % v for v in rep_ms)}); "
            f"{max(main // spl, K - main)} launches of {spl} steps, {launch_ms * 1e3:.1f} us each")
        return sim, ms, launch_ms, spl, rep_ms

    def sustained(sim, spl, launch_ms):
        """reps timed regions of at least 100 ms of whole multi-step launches each, continuing from
        the current state: median ms per step."""
        n = max(1, int(np.ceil(100.0 / launch_ms))) * spl
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sim.step(n)
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return n, out

    if args.profile_only:
        sim, ms, _, _, _ = timed_run(args.storage)
        log(f"profile-only: {N * K / (ms / 1e3) / 1e6:.1f} MLUPS, {sim.bytes_per_update} B/LU")
        if args.with_copy:
            nbytes = N * 7 * 4
            a = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
            b = torch.empty_like(a)
            for _ in range(10):
                lbm.lbm_lee_device_copy(b.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
            torch.cuda.synchronize()
            log(f"copy kernel: 10 launches of {nbytes} bytes read + {nbytes} bytes written")
        return

    modes = [m for m in args.modes.split(",") if m]
    if args.storage not in modes:
        modes.insert(0, args.storage)
    if "f64" not in modes:
        modes.append("f64")
    results = {}
    moments = {}
    for mode in modes:
        sim, ms, launch_ms, spl, rep_ms = timed_run(mode)
        m = sim.moments()
        moments[mode] = (m["p"].clone(), m["u"].clone())
        n_s, s_ms = sustained(sim, spl, launch_ms)
        log(f"{mode}: sustained, {reps} regions of {n_s} steps: {', '.join('%.2f' % v for v in s_ms)} ms")
        results[mode] = dict(ms=ms, launch_ms=launch_ms, spl=spl, bpu=sim.bytes_per_update, scale=sim.store_scale,
                             variant=sim.variant if spl > 1 or sim.variant not in ("tb2", "tb3") else "generic",
                             rep_ms=rep_ms, sustained_steps=n_s, sustained_ms=s_ms)
        sim.close()
        del sim
    p_ref, u_ref = moments["f64"]

    def rel(mode):
        p, uu = moments[mode]
        return (float(torch.linalg.vector_norm(p - p_ref) / torch.linalg.vector_norm(p_ref)),
                float(torch.linalg.vector_norm(uu - u_ref) / torch.linalg.vector_norm(u_ref)))

    storage_modes = {}
    for mode, r in results.items():
        mlups = N * K / (r["ms"] / 1e3) / 1e6
        spl = r["spl"]
        # algorithmic HBM bytes per launch (one read and one write of the moving populations)
        # over the time per launch
        gbs = N * r["bpu"] / (r["launch_ms"] / 1e3) / 1e9
        ep, eu = rel(mode)
        s_med = float(np.median(r["sustained_ms"]))
        storage_modes[mode] = dict(MLUPS=round(mlups, 1), ms_per_step=round(r["ms"] / K, 5),
                                   bytes_per_update=r["bpu"], steps_per_launch=spl, GBs=round(gbs, 1),
                                   frac_peak_hbm=round(gbs / PEAK_HBM_GBS, 4),
                                   rel_l2_p_vs_f64=ep, rel_l2_u_vs_f64=eu, store_scale=r["scale"],
                                   variant=r["variant"], rep_ms=[round(v, 4) for v in r["rep_ms"]],
                                   sustained=dict(steps_per_region=r["sustained_steps"],
                                                  region_ms=[round(v, 3) for v in r["sustained_ms"]],
                                                  MLUPS_median=round(N * r["sustained_steps"] / (s_med / 1e3) / 1e6, 1)))
        log(mode, storage_modes[mode])

    # plain copy kernel of the same size as one population buffer pair (read + write)
    nbytes = N * 7 * 4
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        lbm.lbm_lee_device_copy(b.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    copy_reps = 20
    ev0.record(stream)
    for _ in range(copy_reps):
        lbm.lbm_lee_device_copy(b.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes * copy_reps / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del a, b
    log(f"copy kernel: {copy_gbs:.1f} GB/s")

    main_mode = storage_modes[args.storage]
    ms_step = results[args.storage]["ms"] / K
    bpu = results[args.storage]["bpu"]
    variant = results[args.storage]["variant"]
    spl = results[args.storage]["spl"]
    launch_ms = results[args.storage]["launch_ms"]
    achieved = N * bpu / (launch_ms / 1e3) / 1e9
    traffic = traffic_from_counters(args.storage, n, variant)
    what = (f"{spl} fused pull-stream/collide steps per launch" if spl > 1 else "fused pull-stream/collide")
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic,
                    kernel=f"step_{variant}<D3Q7,{args.storage}> ({what})", steps_per_launch=spl,
                    launch_ms=round(launch_ms, 5), algorithmic_bytes_per_launch=N * bpu,
                    measured_traffic_GBs=None if traffic is None else round(traffic / (launch_ms / 1e3) / 1e9, 1),
                    # the one-step scheme's bytes per lattice update at this update rate: above the
                    # HBM peak when the launches fuse several steps
                    one_step_equivalent_GBs=round(N * bpu * spl / (launch_ms / 1e3) / 1e9, 1),
                    frac_of_copy=round(achieved / copy_gbs, 4), copy_GBs=round(copy_gbs, 1))

    nrbc_result = None if args.no_nrbc else nrbc_leg()
    nrbc3d_result = None if args.no_nrbc else nrbc3d_leg()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(shape, rho, u, theta, args.cpu_seconds)
        log("cpu baseline", cpu)

    line = {
        "metric": METRIC,
        "value": main_mode["MLUPS"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"3D LEE-LBM D3Q7 {n}^3 periodic, 8 seeded Gaussian pressure pulses "
                               f"(amplitude 1e-3, sigma 12 cells), tau=1/2, {K} steps",
                   "lattice": "D3Q7", "cells": N, "storage": args.storage, "variant": args.variant,
                   "global_batch": 1, "parallelism": "none (1 GPU)"},
        "timing": {"protocol": f"HIP events on the library's stream; value = median of {reps} timed regions of "
                               f"exactly {K} steps from the initial state; each storage mode also reports {reps} "
                               "sustained regions of >= 100 ms of whole launches (median MLUPS)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "storage_modes": storage_modes,
        "error_reference": "GPU FP64 path (parity with the FP64 oracle <= 1e-12 in the test suite)",
        "learned_closure": nrbc_result,
        "learned_closure_3d": nrbc3d_result,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
