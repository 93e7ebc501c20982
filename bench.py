#!/usr/bin/env python3
"""Benchmark of the QLA hot path on one MI355X.

One benchmark step is the whole job of the 4096^2 plain workload: set the index
from a device-resident n (coefficient checks), initialise the packet, advance
20000 QLA steps recording the FP64 energy every 100 steps on the device, and read
the fields out to a device buffer. Inputs are resident in HBM before the timed
region starts. `value` is lattice-site updates per second (GLUPS) of that job in
FP64; the same job in FP32 is reported under "fp32".

The roofline entry is for the dominant kernel, the fused step: algorithmic bytes
per launch (FP64: 56 B per site = 3 amplitudes read and written + n read; FP32:
28 B) over its average launch duration, measured with HIP events on the stream
the library launches on, against the MI355X HBM peak of 8 TB/s.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE = {"f64": 56, "f32": 28}
METRIC = "lattice-site updates/s (GLUPS) + HBM GB/s; batched/surrogate instances/s at error"


def run_job(qla, torch, w, n_dev, prec_code, out_dev, energies, stream_ptr, record_kernel):
    """The whole job once; returns (ctx, list of (start, end) events around advances)."""
    ctx = qla.qla_create(w.nx, w.ny, w.delta, prec_code, qla.QLA_V_SKEW_HALF, stream_ptr)
    try:
        qla.qla_set_index_device(ctx, n_dev, w.nx)
        p = w.packet
        qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)
        pairs = []
        chunks = w.steps // w.energy_every
        qla.qla_energy_device(ctx, energies[0:1])
        for c in range(chunks):
            if record_kernel:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                qla.qla_advance(ctx, w.energy_every)
                b.record()
                pairs.append((a, b))
            else:
                qla.qla_advance(ctx, w.energy_every)
            qla.qla_energy_device(ctx, energies[c + 1:c + 2])
        qla.qla_get_fields_device(ctx, out_dev, 1)
    except Exception:
        qla.qla_destroy(ctx)
        raise
    return ctx, pairs


def bench_precision(qla, torch, w, prec, steps, warmup):
    code = qla.QLA_F64 if prec == "f64" else qla.QLA_F32
    import workloads
    n_host = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    n_dev = torch.from_numpy(n_host).to("cuda")
    out_dev = torch.empty((3, w.ny, w.nx), dtype=torch.float64, device="cuda")
    energies = torch.zeros(w.steps // w.energy_every + 1, dtype=torch.float64, device="cuda")
    # The library enqueues on this stream; torch's events are recorded on it too.
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    if not sp:
        raise RuntimeError("bench needs a non-default torch stream")
    for _ in range(warmup):
        ctx, _ = run_job(qla, torch, w, n_dev, code, out_dev, energies, sp, False)
        torch.cuda.synchronize()
        qla.qla_destroy(ctx)
    times, kernel_ms, drift = [], [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record()
        ctx, pairs = run_job(qla, torch, w, n_dev, code, out_dev, energies, sp, True)
        t1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        qla.qla_destroy(ctx)
        times.append(max(t0.elapsed_time(t1) / 1e3, 0.0) or wall)
        adv = sum(a.elapsed_time(b) for a, b in pairs)
        kernel_ms.append(adv / w.steps)
        e = energies.cpu().numpy()
        drift.append(float(abs(e / e[0] - 1).max()))
        print(f"[bench] {prec} step done: {times[-1]:.3f} s, step kernel "
              f"{kernel_ms[-1] * 1e3:.1f} us, max |E/E0-1| {drift[-1]:.2e}",
              file=sys.stderr, flush=True)
    t = max(times)
    sites = w.nx * w.ny * w.steps
    k_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    achieved = BYTES_PER_SITE[prec] * w.nx * w.ny / k_s / 1e9
    return {
        "glups": sites / t / 1e9,
        "seconds": t,
        "kernel_us": k_s * 1e6,
        "kernel_glups": w.nx * w.ny / k_s / 1e9,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "energy_max_rel_drift": max(drift),
    }


def cpu_baseline(w, sample_steps):
    import numpy as np
    import oracle
    import workloads
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    q = oracle.packet_from(n, w.packet)
    t0 = time.perf_counter()
    oracle.advance(q, n, w.delta, sample_steps)
    dt = time.perf_counter() - t0
    del q
    return {"value": round(w.nx * w.ny * sample_steps / dt / 1e9, 6), "unit": "GLUPS",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"first {sample_steps} steps of the {w.nx}x{w.ny} workload, FP64, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="qla_4096_ellipse_20000")
    ap.add_argument("--qla-steps", type=int, default=0, help="override the QLA step count")
    ap.add_argument("--precisions", default="f64,f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=3)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (a reference kernel of "
                         "known traffic for hardware counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; the multi-GPU halo-exchange path "
              "is not part of it (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import dataclasses
    import torch
    import workloads
    from paper_2604_21128_amd import qla
    qla.load()   # fails loudly if the HIP library is not built
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib * 2**20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = workloads.workload_by_name(args.workload)
    if args.qla_steps:
        w = dataclasses.replace(w, steps=args.qla_steps)
    precs = [p for p in args.precisions.split(",") if p]
    results = {}
    stream = torch.cuda.Stream()   # default priority
    with torch.cuda.stream(stream):
        for p in precs:
            results[p] = bench_precision(qla, torch, w, p, args.steps, args.warmup)
    main_p = precs[0]
    r = results[main_p]
    line = {
        "metric": METRIC,
        "value": round(r["glups"], 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["seconds"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_p,
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "qla_steps": w.steps,
                   "energy_every": w.energy_every, "delta": w.delta, "potential": "skew_half",
                   "ellipse": dataclasses.asdict(w.ellipse), "packet": dataclasses.asdict(w.packet)},
        "roofline": r["roofline"],
        "step_kernel_us": round(r["kernel_us"], 2),
        "step_kernel_glups": round(r["kernel_glups"], 2),
        "energy_max_rel_drift": r["energy_max_rel_drift"],
    }
    for p in precs[1:]:
        rp = results[p]
        line[p] = {"value": round(rp["glups"], 3), "unit": "GLUPS",
                   "ms_per_step": round(rp["seconds"] * 1e3, 3), "roofline": rp["roofline"],
                   "step_kernel_us": round(rp["kernel_us"], 2),
                   "energy_max_rel_drift": rp["energy_max_rel_drift"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
