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


POTENTIALS = {"skew_half": 0, "paper": 1, "none": 2, "bstream": 3}


def full_tuning(t):
    """(rows per segment, prefetch rows, steps per pass, columns per lane); the last
    defaults to 1 where a recorded tuning has only the first three."""
    t = tuple(int(v) for v in t)
    return t if len(t) == 4 else t + (1,)


def apply_tuning(qla, ctx, tuning):
    t = full_tuning(tuning)
    qla.qla_set_tuning(ctx, *t[:3])
    qla.qla_set_lane_columns(ctx, t[3])


def current_tuning(qla, ctx):
    return tuple(qla.qla_get_tuning(ctx)) + (qla.qla_get_lane_columns(ctx),)


def run_job(qla, torch, w, n_dev, prec_code, out_dev, energies, stream_ptr, record_kernel,
            tuning=None, potential=0):
    """The whole job once; returns (ctx, list of (start, end) events around advances).
    With tuning=None the context autotunes (untimed warm-up only)."""
    ctx = qla.qla_create(w.nx, w.ny, w.delta, prec_code, potential, stream_ptr)
    try:
        qla.qla_set_index_device(ctx, n_dev, w.nx)
        if tuning is None:
            qla.qla_autotune(ctx)
        else:
            apply_tuning(qla, ctx, tuning)
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


def bench_precision(qla, torch, w, prec, steps, warmup, forced_tuning=None, potential=0):
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
    tuning = full_tuning(forced_tuning) if forced_tuning else None
    for _ in range(max(1, warmup)):
        ctx, _ = run_job(qla, torch, w, n_dev, code, out_dev, energies, sp, False, tuning,
                         potential)
        torch.cuda.synchronize()
        if tuning is None:
            tuning = current_tuning(qla, ctx)
        qla.qla_destroy(ctx)
    times, kernel_ms, drift = [], [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record()
        ctx, pairs = run_job(qla, torch, w, n_dev, code, out_dev, energies, sp, True, tuning,
                             potential)
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
    k_s = sum(kernel_ms) / len(kernel_ms) / 1e3          # seconds per QLA step
    rows, pf, fused, cols = tuning
    launch_s = k_s * fused                               # one launch applies `fused` steps
    algorithmic = BYTES_PER_SITE[prec] * w.nx * w.ny * fused
    achieved = algorithmic / launch_s / 1e9
    traffic = measured_traffic(w, prec, tuning)
    return {
        "glups": sites / t / 1e9,
        "seconds": t,
        "kernel_us": k_s * 1e6,
        "kernel_glups": w.nx * w.ny / k_s / 1e9,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (round(traffic / launch_s / 1e9, 1) if traffic else None)},
        "launch": {"steps_per_launch": fused, "rows_per_segment": rows, "prefetch_rows": pf,
                   "columns_per_lane": cols,
                   "launch_us": round(launch_s * 1e6, 2),
                   "algorithmic_bytes_per_launch": algorithmic,
                   "hbm_bytes_per_launch": traffic},
        "energy_max_rel_drift": max(drift),
    }


STEP_SOURCES = ("paper_2604_21128_amd/csrc/qla_step.hip", "paper_2604_21128_amd/csrc/qla_device.h")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "qla_step_ez_4096_ellipse.json")


def step_kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(w, prec, tuning):
    """HBM bytes per launch of the step kernel from the committed counter summary,
    or None if the kernel source or its tuning changed since the counters were taken."""
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256") != step_kernel_sha() or rec.get("workload") != w.name:
        return None
    r = rec.get(prec)
    if not r or full_tuning(r.get("tuning", ())) != full_tuning(tuning):
        return None
    return r["hbm_bytes_per_launch"]


def recorded_tuning(w):
    """The tuning under which the committed counters were taken, if the step kernel is
    unchanged since (it was the autotuner's choice then); else {} and the run autotunes."""
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return {}
    if rec.get("kernel_sha256") != step_kernel_sha() or rec.get("workload") != w.name:
        return {}
    return {p: rec[p]["tuning"] for p in ("f64", "f32") if p in rec}


def summarize_counters(fetch_dir, write_dir, trace_dir, tuning_json):
    """Turn rocprofv3 outputs (one FETCH_SIZE run, one WRITE_SIZE run, one kernel trace)
    into profiles/qla_step_ez_4096_ellipse.{md,json}. The FETCH_SIZE and WRITE_SIZE
    values of every kernel are scaled by what the counters read for the 1 GiB reference
    copy in the same run."""
    import collections
    import csv
    import glob
    def load(d, ctr):
        out = collections.defaultdict(list)
        for fn in glob.glob(os.path.join(d, "*counter_collection.csv")):
            for r in csv.DictReader(open(fn)):
                if r["Counter_Name"] == ctr:
                    out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return out
    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    ref = "__amd_rocclr_copyBuffer"
    kib = 1048576.0
    fcopy = max(fe[ref]); wcopy = max(wr[ref])
    fs, ws = kib / fcopy, kib / wcopy
    tuning = json.loads(tuning_json)
    w = __import__("workloads").plain_4096()
    n = w.nx * w.ny
    rec = {"workload": w.name, "kernel_sha256": step_kernel_sha(), "fetch_scale": fs,
           "write_scale": ws}
    lines = [f"# qla_step_ez_kernel on the {w.nx}x{w.ny} ellipse workload (MI355X, gfx950)", "",
             "Commands (from /tmp with TMPDIR=/tmp; R = repository root; tuning fixed to the "
             "autotuned values below):", "", "```"]
    tj = "'" + json.dumps(tuning) + "'"

    def shown(d):  # the output folders as given, relative to the repository as $R/...
        rel = os.path.relpath(os.path.abspath(d), ROOT)
        return d if rel.startswith("..") else "$R/" + rel
    tdir, fdir, wdir = shown(trace_dir), shown(fetch_dir), shown(write_dir)
    lines += [f"rocprofv3 --kernel-trace --stats --output-format csv -d {tdir} "
              f"-o trace -- python3 $R/bench.py --steps 1 --warmup 1 --qla-steps 2000 "
              f"--no-cpu-baseline --no-extras --tuning-json {tj}",
              f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {fdir} -o fetch "
              f"-- python3 $R/bench.py --steps 1 --warmup 1 --qla-steps 100 --no-cpu-baseline "
              f"--no-extras --copy-probe-mib 1024 --tuning-json {tj}",
              f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {wdir} -o write "
              f"-- python3 $R/bench.py --steps 1 --warmup 1 --qla-steps 100 --no-cpu-baseline "
              f"--no-extras --copy-probe-mib 1024 --tuning-json {tj}",
              f"python3 $R/bench.py --summarize-counters {fdir} {wdir} {tdir} {tj}", "```", ""]
    lines += ["## Kernel trace (--stats)", "", "| kernel | calls | average (us) | min (us) | max (us) |",
              "|---|---|---|---|---|"]
    avg_ns = {}
    for fn in glob.glob(os.path.join(trace_dir, "*kernel_stats.csv")):
        for r in csv.DictReader(open(fn)):
            name = r["Name"].replace("(anonymous namespace)::", "")
            short = name.split("(qla::")[0].split("(double")[0].split("(float")[0]
            avg_ns[name] = float(r["AverageNs"])
            lines.append(f"| `{short[:80]}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                         f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} |")
    lines += ["", "## HBM traffic per dispatch (hardware counters, KiB)", "",
              f"Reference: a 1 GiB device copy (`{ref}`, 1048576 KiB read and written) reads "
              f"FETCH_SIZE = {fcopy:.1f} and WRITE_SIZE = {wcopy:.1f}; scale factors "
              f"{fs:.4f} (fetch) and {ws:.4f} (write).", "",
              "| kernel | steps/launch | FETCH raw | WRITE raw | read scaled | write scaled | "
              "algorithmic read | algorithmic write | traffic / algorithmic |",
              "|---|---|---|---|---|---|---|---|---|"]
    for k in fe:
        if "qla_step_ez_kernel" not in k:
            continue
        prec = "f64" if "<double" in k else "f32"
        e = 8 if prec == "f64" else 4
        t = tuning[prec]
        fused = int(t[2])
        fr = sum(fe[k]) / len(fe[k]); wv = sum(wr[k]) / len(wr[k])
        ar, aw = 4 * n * e / 1024, 3 * n * e / 1024
        hbm = (fr * fs + wv * ws) * 1024
        rec[prec] = {"tuning": t, "hbm_bytes_per_launch": hbm,
                     "algorithmic_bytes_per_launch": 7 * n * e * fused}
        lines.append(f"| step {prec} | {fused} | {fr:.0f} | {wv:.0f} | {fr*fs:.0f} | {wv*ws:.0f} | "
                     f"{ar:.0f} | {aw:.0f} | {(fr*fs+wv*ws)/(ar+aw):.3f} |")
    lines += ["", "Algorithmic bytes per launch count every step the launch applies (56 B per site "
              "update in FP64, 28 B in FP32); the read and write columns are per launch.", ""]
    base = os.path.join(ROOT, "profiles", "qla_step_ez_4096_ellipse")
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines))
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print("\n".join(lines))


def precision_study(qla, torch, w, snapshot_every, cpu_steps=3):
    """Run the workload in FP64 and FP32 side by side; at every snapshot compare the
    FP32 fields with the FP64 ones (relative L2 over the three planes) and record both
    energy drifts. Norms are diagnostics computed on the device."""
    import workloads
    n_dev = torch.from_numpy(workloads.ellipse_index(w.nx, w.ny, w.ellipse)).to("cuda")
    sp = torch.cuda.current_stream().cuda_stream
    ctxs = {}
    for prec, code in (("f64", qla.QLA_F64), ("f32", qla.QLA_F32)):
        c = qla.qla_create(w.nx, w.ny, w.delta, code, qla.QLA_V_SKEW_HALF, sp)
        qla.qla_set_index_device(c, n_dev, w.nx)
        qla.qla_autotune(c)   # tuned for this lattice (state kept)
        p = w.packet
        qla.qla_init_packet(c, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)
        ctxs[prec] = c
    f64 = torch.empty((3, w.ny, w.nx), dtype=torch.float64, device="cuda")
    f32 = torch.empty_like(f64)
    e0 = {k: qla.qla_energy(c) for k, c in ctxs.items()}
    snaps = []
    t_run = {"f64": 0.0, "f32": 0.0}
    for step in range(snapshot_every, w.steps + 1, snapshot_every):
        for prec, c in ctxs.items():
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            qla.qla_advance(c, snapshot_every)
            b.record()
            torch.cuda.synchronize()
            t_run[prec] += a.elapsed_time(b) / 1e3
        qla.qla_get_fields_device(ctxs["f64"], f64, 0)
        qla.qla_get_fields_device(ctxs["f32"], f32, 0)
        torch.cuda.synchronize()
        err = float(torch.linalg.vector_norm(f32 - f64) / torch.linalg.vector_norm(f64))
        ed = {k: qla.qla_energy(c) / e0[k] - 1 for k, c in ctxs.items()}
        snaps.append({"step": step, "field_rel_l2_f32_vs_f64": err,
                      "energy_drift_f64": ed["f64"], "energy_drift_f32": ed["f32"]})
        print(f"[study] step {step}: f32 vs f64 rel L2 {err:.3e}, drift f64 {ed['f64']:.2e} "
              f"f32 {ed['f32']:.2e}", file=sys.stderr, flush=True)
    tunings = {k: current_tuning(qla, c) for k, c in ctxs.items()}
    if cpu_steps:
        rate, dt = oracle_rate(w, cpu_steps)
        cpu = {"value": round(rate, 6), "unit": "GLUPS", "cores": __import__("oracle").threads(),
               "kind": "oracle", "sample": f"first {cpu_steps} steps of the {w.nx}x{w.ny} "
                                           f"workload, FP64, {dt:.1f} s"}
        print(f"[study] CPU oracle: {rate:.4f} GLUPS on {cpu['cores']} threads", file=sys.stderr,
              flush=True)
    else:
        cpu = None
    for c in ctxs.values():
        qla.qla_destroy(c)
    sites = w.nx * w.ny * w.steps
    return {"workload": w.name, "nx": w.nx, "ny": w.ny, "qla_steps": w.steps,
            "snapshot_every": snapshot_every,
            "tuning": {k: dict(zip(("rows_per_segment", "prefetch_rows", "steps_per_pass",
                                    "columns_per_lane"), t)) for k, t in tunings.items()},
            "glups": {k: sites / v / 1e9 for k, v in t_run.items()},
            "seconds": t_run, "cpu_baseline": cpu, "snapshots": snaps}


def batched_study(qla, torch, count, seed, error_samples):
    """The batched workload: `count` instances drawn by workloads.sample_instances, each run
    4 N steps in FP32. Times one captured batched run and the same instances run one after
    another with the single-lattice kernel, and measures the batched FP32 field error
    against FP64 single-lattice runs of sampled instances."""
    import numpy as np
    import workloads
    inst = workloads.sample_instances(count, seed=seed)
    sp = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    b = qla.qla_batch_create([i.n_side for i in inst], [i.n_side for i in inst],
                             [i.delta for i in inst], qla.QLA_F32, qla.QLA_V_SKEW_HALF, sp)
    ctxs = [qla.qla_batch_context(b, k) for k in range(count)]
    ns = []
    for k, i in enumerate(inst):
        n = workloads.ellipse_index(i.n_side, i.n_side, i.ellipse)
        ns.append(n)
        qla.qla_set_index(ctxs[k], n)

    def init_all():
        for k, i in enumerate(inst):
            p = i.packet
            qla.qla_init_packet(ctxs[k], p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)

    init_all()
    steps = [i.steps for i in inst]
    qla.qla_batch_plan(b, steps, 0)
    info = qla.qla_batch_plan_info(b)
    heights = {}
    for i in range(count):
        h = qla.qla_batch_segment_rows(b, i)
        heights[h] = heights.get(h, 0) + 1
    info["segment_rows_histogram"] = {str(h): c for h, c in sorted(heights.items())}
    print(f"[batch] {count} instances set up and planned in {time.perf_counter() - t0:.1f} s: "
          f"{info}", file=sys.stderr, flush=True)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    times = []
    for rep in range(2):
        init_all()
        torch.cuda.synchronize()
        a, z = ev(), ev()
        a.record()
        qla.qla_batch_run(b)
        z.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(z) / 1e3)
        print(f"[batch] batched run {rep}: {times[-1]:.3f} s", file=sys.stderr, flush=True)
    t_batch = min(times)
    # field error of the batched FP32 result against FP64 single-lattice runs
    rng = np.random.default_rng(seed + 1)
    picks = sorted(rng.choice(count, size=min(error_samples, count), replace=False).tolist())
    errs = []
    for k in picks:
        i = inst[k]
        got = qla.qla_get_fields(ctxs[k], i.n_side, i.n_side)
        with qla.Lattice(i.n_side, i.n_side, i.delta, qla.QLA_F64, qla.QLA_V_SKEW_HALF, sp) as lat:
            lat.set_index(ns[k])
            lat.init_packet(i.packet)
            lat.advance(i.steps)
            want = lat.fields()
        errs.append(float(np.linalg.norm(got - want) / np.linalg.norm(want)))
    # the same instances one after another with the single-lattice kernel (plain QLA)
    init_all()
    torch.cuda.synchronize()
    a, z = ev(), ev()
    a.record()
    for k, i in enumerate(inst):
        qla.qla_advance(ctxs[k], i.steps)
    z.record()
    torch.cuda.synchronize()
    t_plain = a.elapsed_time(z) / 1e3
    qla.qla_batch_destroy(b)
    updates = info["site_updates"]
    return {"workload": f"qla_batched_{count}_instances_256_1024", "instances": count,
            "seed": seed, "site_updates": updates,
            "batched": {"seconds": t_batch, "instances_per_s": count / t_batch,
                        "glups": updates / t_batch / 1e9, "plan": info},
            "plain_sequential": {"seconds": t_plain, "instances_per_s": count / t_plain,
                                 "glups": updates / t_plain / 1e9},
            "speedup": t_plain / t_batch,
            "field_rel_l2_fp32_batched_vs_fp64": {"instances": picks, "max": max(errs),
                                                  "median": float(np.median(errs))}}


def surrogate_study(qla, torch, args):
    """The learned-surrogate workload: QLA-generated pairs on a fixed grid (instances drawn
    as in the batched workload), training of the neural operator on the GPU, then the
    held-out set through surrogate + energy check + QLA fallback, against plain QLA."""
    import numpy as np
    import workloads
    from paper_2604_21128_amd import surrogate as S
    side, steps, B = args.side, args.surrogate_steps, args.batch
    log = lambda m: print(f"[surrogate] {m}", file=sys.stderr, flush=True)
    lam = dict(lam_min=args.lam_range[0], lam_max=args.lam_range[1])
    train_i = workloads.sample_instances(args.train_count, seed=10, fixed_side=side, **lam)
    test_i = workloads.sample_instances(args.test_count, seed=11, fixed_side=side, **lam)

    def index_fn(insts):
        return lambda c0, k: workloads.ellipse_index_batch(
            side, side, [i.ellipse for i in insts[c0:c0 + k]], device="cuda")

    def packets(insts):
        return [S.PacketSpec(i.packet.x0, i.packet.y0, i.packet.sigma, i.packet.lam,
                             i.packet.phi, i.packet.amp, i.packet.planar) for i in insts]
    delta = workloads.DELTA
    t0 = time.perf_counter()
    train = S.qla_pairs(index_fn(train_i), len(train_i), packets(train_i), delta, steps,
                        chunk=args.chunk, log=log)
    test = S.qla_pairs(index_fn(test_i), len(test_i), packets(test_i), delta, steps,
                       chunk=args.chunk, keep_f32=True, log=log)
    gen_s = time.perf_counter() - t0
    log(f"pairs ready in {gen_s:.1f} s")
    sur = S.Surrogate(side, side, max_batch=B, seed=args.seed)

    def field_errors(out):
        d = (out - test.targets_f32).flatten(1).norm(dim=1)
        return (d / test.targets_f32.flatten(1).norm(dim=1)).cpu().numpy()

    # the untrained network, for comparison
    out0, e_0 = S.predict_all(sur, test.inputs, B)
    err_untrained = field_errors(out0)
    del out0
    hist = S.train(sur, train.inputs, train.targets, B, args.epochs, args.lr,
                   time_budget_s=args.train_budget_s, log=log)
    pred, energy = S.predict_all(sur, test.inputs, B)
    err_pred = field_errors(pred)
    ok = S.accept(energy, test.e0, args.accept_tol).cpu().numpy()
    e_rel = (energy / test.e0 - 1).abs().cpu().numpy()
    del pred
    out, ok2, t = S.run_with_fallback(sur, test.inputs, test.e0, index_fn(test_i),
                                      packets(test_i), delta, steps, B, args.accept_tol,
                                      args.chunk)
    err_final = field_errors(out)
    del out
    # the same held-out set with the band gate in front of the network
    frac = S.band_fractions(sur, test.inputs, B).cpu().numpy()
    out_g, ok_g, t_g = S.run_with_fallback(sur, test.inputs, test.e0, index_fn(test_i),
                                           packets(test_i), delta, steps, B, args.accept_tol,
                                           args.chunk, band_min=args.band_min)
    err_gated = field_errors(out_g)
    ok_g = ok_g.cpu().numpy()
    del out_g
    n_test = len(test_i)
    t_plain = test.qla_seconds
    t_sur = t["surrogate_s"] + t["fallback_qla_s"]
    t_gate = t_g["surrogate_s"] + t_g["fallback_qla_s"]
    losses = hist["losses"]
    tail = losses[-max(1, len(losses) // 20):]
    q = lambda a: {"median": float(np.median(a)), "p90": float(np.percentile(a, 90)),
                   "max": float(np.max(a))}
    res = {
        "metric": "lattices/s through surrogate + energy check + QLA fallback",
        "value": n_test / t_sur, "unit": "lattices/s", "higher_is_better": True,
        "vs_plain_qla": t_plain / t_sur, "dtype": "bf16 (network), f32 (QLA)",
        "data": "synthetic",
        "workload": f"qla_surrogate_fno_{side}_{steps}_steps_lambda_"
                    f"{args.lam_range[0]:g}_{args.lam_range[1]:g}",
        "grid": side, "qla_steps": steps, "wavelength_range": list(args.lam_range),
        "train_instances": len(train_i),
        "test_instances": n_test,
        "network": dict(sur.shape, input="n - 2, q2, q3, q4", output="q2, q3, q4",
                        params=int(qla.qla_fno_param_count(sur.h)), dtype="bf16 storage, "
                        "fp32 accumulation"),
        "training": {"steps": hist["steps"], "batch": B, "epochs": hist["steps"] * B
                     / len(train_i), "lr": args.lr, "seconds": hist["seconds"],
                     "samples_per_s": hist["steps"] * B / hist["seconds"],
                     "loss_first": float(np.mean(losses[:20])), "loss_last": float(np.mean(tail))},
        "qla_pair_generation": {"seconds_total": gen_s, "qla_seconds": train.qla_seconds
                                + test.qla_seconds,
                                "glups": (train.site_updates + test.site_updates)
                                / (train.qla_seconds + test.qla_seconds) / 1e9},
        "held_out": {
            "field_rel_l2_untrained": q(err_untrained),
            "field_rel_l2_prediction": q(err_pred),
            "energy_rel_error": q(e_rel),
            "accept_tol": args.accept_tol,
            "accepted": int(ok.sum()),
            "field_rel_l2_accepted": q(err_pred[ok]) if ok.any() else None,
            "field_rel_l2_after_fallback": q(err_final),
        },
        "throughput": {
            "plain_qla_instances_per_s": n_test / t_plain,
            "surrogate_with_fallback_instances_per_s": n_test / t_sur,
            "surrogate_forward_and_check_s": t["surrogate_s"],
            "fallback_qla_s": t["fallback_qla_s"], "rejected": t["rejected"],
            "plain_qla_s": t_plain, "gain": t_plain / t_sur,
            "surrogate_only_instances_per_s": n_test / t["surrogate_s"],
        },
        "band_gate": {
            "rule": "inputs whose q2, q3, q4 planes hold less than band_min of their energy in "
                    "the kept Fourier modes go straight to QLA",
            "band_min": args.band_min,
            "band_fraction": {"min": float(frac.min()), "median": float(np.median(frac)),
                              "max": float(frac.max())},
            "gated_out": t_g["gated_out"],
            "accepted": int(ok_g.sum()),
            "field_rel_l2_after_fallback": q(err_gated),
            "surrogate_and_gate_s": t_g["surrogate_s"], "fallback_qla_s": t_g["fallback_qla_s"],
            "instances_per_s": n_test / t_gate, "gain": t_plain / t_gate,
        },
    }
    if args.save_params:
        np.save(args.save_params, sur.params())
    sur.close()
    return res


def size_study(qla, torch, sides, precs, steps):
    """Lattice size against throughput on one GPU: the paper's ellipse scaled onto square
    lattices of each side (index generated on the device), the +x packet, the autotuned
    step, `steps` steps timed with HIP events; up to the sizes that fill HBM (80 B per
    site in FP64, 60 in FP32; planes beyond 2 GiB use per-row descriptors)."""
    import workloads
    base = workloads.paper_16384()
    sp = torch.cuda.current_stream().cuda_stream
    free, _ = torch.cuda.mem_get_info()
    rows = []
    for prec in precs:
        code = qla.QLA_F64 if prec == "f64" else qla.QLA_F32
        per_site = 80 if prec == "f64" else 60
        for side in sides:
            if side * side * per_site > 0.9 * free:
                print(f"[size] {prec} {side}^2 skipped: needs "
                      f"{side * side * per_site / 1e9:.0f} GB", file=sys.stderr, flush=True)
                continue
            f = side / base.nx
            e, p = base.ellipse, base.packet
            ctx = qla.qla_create(side, side, base.delta, code, qla.QLA_V_SKEW_HALF, sp)
            try:
                qla.qla_set_index_ellipse(ctx, side / 2, side / 2, e.a * f, e.b * f, e.rot,
                                          e.n_in, e.n_out, e.width)
                qla.qla_init_packet(ctx, p.x0 * f, side / 2, p.sigma, p.lam)
                e0 = qla.qla_energy(ctx)
                qla.qla_autotune(ctx)
                tuning = current_tuning(qla, ctx)
                qla.qla_advance(ctx, 2)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                qla.qla_advance(ctx, steps)
                b.record()
                torch.cuda.synchronize()
                sec = a.elapsed_time(b) / 1e3
                drift = qla.qla_energy(ctx) / e0 - 1
            finally:
                qla.qla_destroy(ctx)
            r = {"precision": prec, "side": side, "sites": side * side,
                 "device_gb": round(side * side * per_site / 1e9, 1), "steps": steps,
                 "glups": side * side * steps / sec / 1e9, "seconds": sec,
                 "energy_rel_drift": drift,
                 "tuning": dict(zip(("rows_per_segment", "prefetch_rows", "steps_per_pass",
                                     "columns_per_lane"), tuning))}
            rows.append(r)
            print(f"[size] {prec} {side}^2: {r['glups']:.1f} GLUPS ({r['device_gb']} GB), "
                  f"tuning {tuning}", file=sys.stderr, flush=True)
    return {"workload": "paper ellipse scaled to square lattices", "steps": steps, "rows": rows}


def divergence_study(qla, torch, w, snapshot_every):
    """Both polarisations on one workload (FP64): energy drift and the relative discrete
    divergence ||div|| / ||(dFx/dx, dFy/dy)|| of B (E_z triple) or D (B_z triple) at each
    snapshot."""
    import numpy as np
    import workloads
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    sp = torch.cuda.current_stream().cuda_stream
    out = {"workload": w.name, "steps": w.steps, "snapshot_every": snapshot_every,
           "triples": {}}
    for triple, name in ((qla.QLA_TRIPLE_EZ, "ez"), (qla.QLA_TRIPLE_BZ, "bz")):
        rows = []
        with qla.Lattice(w.nx, w.ny, w.delta, qla.QLA_F64, qla.QLA_V_SKEW_HALF, sp,
                         triple=triple) as lat:
            lat.set_index(n)
            lat.init_packet(w.packet)
            e0 = lat.energy()
            done = 0
            while done < w.steps:
                k = min(snapshot_every, w.steps - done)
                lat.advance(k)
                done += k
                l2, mx, scale = lat.divergence()
                rows.append({"step": done, "energy_drift": lat.energy() / e0 - 1,
                             "div_l2": l2, "div_max": mx, "scale": scale,
                             "rel_div": l2 / scale if scale > 0 else None})
        print(f"[divergence] {name}: final rel_div {rows[-1]['rel_div']:.3e}, energy drift "
              f"{rows[-1]['energy_drift']:.2e}", file=sys.stderr, flush=True)
        out["triples"][name] = rows
    return out


def oracle_rate(w, sample_steps):
    """The CPU oracle on the first `sample_steps` steps of workload w: (GLUPS, seconds)."""
    import oracle
    import workloads
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    q = oracle.packet_from(n, w.packet)
    t0 = time.perf_counter()
    oracle.advance(q, n, w.delta, sample_steps)
    dt = time.perf_counter() - t0
    return w.nx * w.ny * sample_steps / dt / 1e9, dt


def cpu_baseline(w, sample_steps):
    import oracle
    import workloads
    rate, dt = oracle_rate(w, sample_steps)
    # the small parity workload, all of it
    s = workloads.parity_small()
    ns = workloads.ellipse_index(s.nx, s.ny, s.ellipse)
    qs = oracle.packet_from(ns, s.packet)
    t1 = time.perf_counter()
    oracle.advance(qs, ns, s.delta, s.steps)
    ds = time.perf_counter() - t1
    return {"value": round(rate, 6), "unit": "GLUPS",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"first {sample_steps} steps of the {w.nx}x{w.ny} workload, FP64, "
                      f"{dt:.1f} s",
            "small_workload": {"workload": s.name, "steps": s.steps, "seconds": round(ds, 3),
                               "glups": round(s.nx * s.ny * s.steps / ds / 1e9, 6)}}


def copy_bandwidth(torch, mib=1024, reps=5):
    """A plain device copy of `mib` MiB timed with events: the practical streaming rate
    (bytes read + written per second) beside the 8 TB/s spec."""
    src = torch.ones(mib * 2**20 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del src, dst
    return round(2 * mib * 2**20 / best / 1e9, 1)


def paper_mode_drift(qla, torch):
    """Energy drift of the printed potentials against the default ones on the small
    parity workload (256^2 ellipse, 200 steps, FP64)."""
    import workloads
    s = workloads.parity_small()
    n = workloads.ellipse_index(s.nx, s.ny, s.ellipse)
    sp = torch.cuda.current_stream().cuda_stream
    out = {"workload": s.name, "steps": s.steps}
    for mode, name in ((qla.QLA_V_PAPER, "paper"), (qla.QLA_V_SKEW_HALF, "skew_half")):
        with qla.Lattice(s.nx, s.ny, s.delta, qla.QLA_F64, mode, sp) as lat:
            lat.set_index(n)
            lat.init_packet(s.packet)
            e0 = lat.energy()
            lat.advance(s.steps)
            out[name + "_energy_drift"] = lat.energy() / e0 - 1
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="qla_4096_ellipse_20000")
    ap.add_argument("--qla-steps", type=int, default=0, help="override the QLA step count")
    ap.add_argument("--precisions", default="f64,f32")
    ap.add_argument("--potential", default="skew_half", choices=sorted(POTENTIALS),
                    help="potential mode of the measured job (skew_half: the default "
                         "half-angle potentials; bstream: the B-streaming scheme)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the copy-bandwidth probe and the potential-mode drift run (for "
                         "profiling runs, whose per-kernel averages must cover the job only)")
    ap.add_argument("--cpu-sample-steps", type=int, default=12)
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR",
                                                               "TRACE_DIR", "TUNING_JSON"))
    ap.add_argument("--precision-study", action="store_true",
                    help="FP32 against FP64 on the 8192^2 bubble workload (field L2, energy drift "
                         "per snapshot); prints its own JSON line")
    ap.add_argument("--snapshot-every", type=int, default=1000)
    ap.add_argument("--batched", action="store_true",
                    help="the batched workload (512 instances, FP32); prints its own JSON line")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--error-samples", type=int, default=6)
    ap.add_argument("--size-study", action="store_true",
                    help="throughput against lattice size (--sides, --precisions) up to the "
                         "sizes that fill HBM; prints its own JSON line")
    ap.add_argument("--sides", default="1024,2048,4096,8192,16384,23170,32768,40960,46340")
    ap.add_argument("--size-steps", type=int, default=100)
    ap.add_argument("--divergence-study", action="store_true",
                    help="both polarisations on --workload: energy drift and relative "
                         "divergence per snapshot (--snapshot-every); prints its own JSON line")
    ap.add_argument("--surrogate", action="store_true",
                    help="the learned-surrogate workload; prints its own JSON line")
    ap.add_argument("--side", type=int, default=512)
    ap.add_argument("--surrogate-steps", type=int, default=1024)
    ap.add_argument("--lam-range", type=float, nargs=2, default=(8.0, 32.0),
                    help="packet wavelength range (cells) of the surrogate's instances")
    ap.add_argument("--train-count", type=int, default=20000)
    ap.add_argument("--test-count", type=int, default=1000)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--epochs", type=float, default=1.0)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--train-budget-s", type=float, default=None)
    ap.add_argument("--accept-tol", type=float, default=1e-2)
    ap.add_argument("--band-min", type=float, default=0.5,
                    help="surrogate: also report a run that sends inputs with less than this "
                         "share of their field energy in the kept modes straight to QLA")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--save-params", default="")
    ap.add_argument("--tuning-json", default="",
                    help='fixed tuning instead of autotuning: per precision, rows per '
                         'segment, prefetch rows, steps per pass and optionally columns per '
                         'lane, e.g. {"f64": [176, 3, 2], "f32": [56, 3, 2, 2]}')
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (a reference kernel of "
                         "known traffic for hardware counters)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only; the multi-GPU halo-exchange path "
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
    if args.batched:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = batched_study(qla, torch, args.instances, 0, args.error_samples)
        print(json.dumps(out), flush=True)
        return
    if args.size_study:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = size_study(qla, torch, [int(v) for v in args.sides.split(",")],
                             [p for p in args.precisions.split(",") if p], args.size_steps)
        print(json.dumps(out), flush=True)
        return
    if args.divergence_study:
        w = workloads.workload_by_name(args.workload)
        if args.qla_steps:
            w = dataclasses.replace(w, steps=args.qla_steps)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = divergence_study(qla, torch, w, args.snapshot_every)
        print(json.dumps(out), flush=True)
        return
    if args.surrogate:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = surrogate_study(qla, torch, args)
        print(json.dumps(out), flush=True)
        return
    if args.precision_study:
        w = workloads.bubble_8192()
        if args.qla_steps:
            w = dataclasses.replace(w, steps=args.qla_steps)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = precision_study(qla, torch, w, args.snapshot_every,
                                  0 if args.no_cpu_baseline else 3)
        print(json.dumps(out), flush=True)
        return
    w = workloads.workload_by_name(args.workload)
    if args.qla_steps:
        w = dataclasses.replace(w, steps=args.qla_steps)
    precs = [p for p in args.precisions.split(",") if p]
    results = {}
    stream = torch.cuda.Stream()   # default priority
    with torch.cuda.stream(stream):
        forced = json.loads(args.tuning_json) if args.tuning_json else (
            recorded_tuning(w) if args.potential == "skew_half" else {})
        for p in precs:
            results[p] = bench_precision(qla, torch, w, p, args.steps, args.warmup, forced.get(p),
                                         POTENTIALS[args.potential])
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
                   "energy_every": w.energy_every, "delta": w.delta, "potential": args.potential,
                   "ellipse": dataclasses.asdict(w.ellipse), "packet": dataclasses.asdict(w.packet)},
        "roofline": r["roofline"],
        "launch": r["launch"],
        "step_kernel_us": round(r["kernel_us"], 2),
        "step_kernel_glups": round(r["kernel_glups"], 2),
        "energy_max_rel_drift": r["energy_max_rel_drift"],
    }
    if not args.no_extras:
        with torch.cuda.stream(stream):
            line["copy_gbs"] = copy_bandwidth(torch)
            line["potential_modes_small_workload"] = paper_mode_drift(qla, torch)
            if args.potential == "skew_half" and "f64" in precs:
                # the same job with the B-streaming scheme (no potentials, fully unitary)
                rb = bench_precision(qla, torch, w, "f64", 1, 1, None, POTENTIALS["bstream"])
                line["bstream_f64"] = {"value": round(rb["glups"], 3), "unit": "GLUPS",
                                       "roofline_frac": rb["roofline"]["frac"],
                                       "launch": rb["launch"],
                                       "energy_max_rel_drift": rb["energy_max_rel_drift"]}
    for p in precs[1:]:
        rp = results[p]
        line[p] = {"value": round(rp["glups"], 3), "unit": "GLUPS",
                   "ms_per_step": round(rp["seconds"] * 1e3, 3), "roofline": rp["roofline"],
                   "launch": rp["launch"],
                   "step_kernel_us": round(rp["kernel_us"], 2),
                   "energy_max_rel_drift": rp["energy_max_rel_drift"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
