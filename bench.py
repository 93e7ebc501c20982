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
# The measured job: the largest single-GPU workload, the 8192^2 vacuum bubble in n = 2
# over 40000 steps, FP64 against FP32 at every snapshot.
HEADLINE = "qla_8192_bubble_40000"


def default_chunk(w):
    """QLA steps per benchmark step: 2000 on the 40000-step bubble job (20 benchmark steps
    are the whole job; a snapshot at the end of each), the whole job otherwise."""
    return 2000 if w.name == HEADLINE else w.steps


def default_cpu_steps(w):
    """Oracle steps for cpu_baseline: about 15 s on 16 host threads (0.02 GLUPS)."""
    return max(1, round(3e8 / (w.nx * w.ny)))


def compare_precisions(torch, w, chunk, precs, snaps, energies):
    """Per snapshot (end of each chunk of the first timed job): relative L2 distance of
    the second precision's physical fields (Ez, Bx, By) from the first's, over the three
    planes, and both energy drifts |E/E0 - 1| at that step."""
    a, b = precs[0], precs[1]
    rows = []
    for c, (sa, sb) in enumerate(zip(snaps[a], snaps[b])):
        step = min((c + 1) * chunk, w.steps)
        k = step // w.energy_every
        rel = float(torch.linalg.vector_norm(sb - sa) / torch.linalg.vector_norm(sa))
        rows.append({"step": step, "field_rel_l2": rel,
                     "energy_drift_" + a: float(energies[a][k] / energies[a][0] - 1),
                     "energy_drift_" + b: float(energies[b][k] / energies[b][0] - 1)})
    return {"field_rel_l2_final": rows[-1]["field_rel_l2"],
            "field_rel_l2_max": max(r["field_rel_l2"] for r in rows),
            "energy_drift_max_" + b: max(abs(r["energy_drift_" + b]) for r in rows),
            "snapshots": rows}


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


POTENTIAL_NAMES = {v: k for k, v in POTENTIALS.items()}


class Job:
    """One lattice context running a workload in one precision, chunk by chunk.

    The job: set n(x, y) from device memory (the coefficient checks of Eqs. 2e4 and
    2e13), initialise the packet, advance w.steps QLA steps recording the FP64 energy
    on the device every w.energy_every steps, and read the physical fields out to a
    device buffer at the end of every chunk (the snapshots). A benchmark step is one
    chunk; the job's set-up falls into its first chunk, and once the last chunk is done
    the next chunk starts the job again. The context and every buffer are allocated
    before any timing starts."""

    def __init__(self, qla, torch, w, prec, potential, n_dev, stream_ptr, chunk, jobs,
                 snapshots):
        self.qla, self.torch, self.w, self.prec = qla, torch, w, prec
        self.n_dev, self.chunk = n_dev, chunk
        self.chunks_per_job = -(-w.steps // chunk)
        code = qla.QLA_F64 if prec == "f64" else qla.QLA_F32
        self.ctx = qla.qla_create(w.nx, w.ny, w.delta, code, potential, stream_ptr)
        n_e = w.steps // w.energy_every + 1
        self.energies = torch.zeros((jobs, n_e), dtype=torch.float64, device="cuda")
        self.out = torch.empty((3, w.ny, w.nx), dtype=torch.float64, device="cuda")
        self.snap = [torch.empty_like(self.out) for _ in range(snapshots)]
        self.tuning = None
        self.written = []   # (job row, energy index) written while `pairs` were recorded

    def close(self):
        self.qla.qla_destroy(self.ctx)
        self.snap, self.out = [], None

    def tune(self, tuning):
        """Fix the tuning, or autotune on this lattice (tuning None)."""
        q = self.qla
        q.qla_set_index_device(self.ctx, self.n_dev, self.w.nx)
        if tuning is None:
            q.qla_autotune(self.ctx)
        else:
            apply_tuning(q, self.ctx, tuning)
        self.tuning = current_tuning(q, self.ctx)

    def run_chunk(self, i, pairs=None):
        """Benchmark step i: chunk i % chunks_per_job of job i // chunks_per_job.
        Appends (start, end, qla steps) events around each advance to `pairs`."""
        q, w, torch = self.qla, self.w, self.torch
        c, j = i % self.chunks_per_job, i // self.chunks_per_job
        row = j % self.energies.shape[0]
        e = self.energies[row]
        if c == 0:
            q.qla_set_index_device(self.ctx, self.n_dev, w.nx)
            p = w.packet
            q.qla_init_packet(self.ctx, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)
            q.qla_energy_device(self.ctx, e[0:1])
            if pairs is not None:
                self.written.append((row, 0))
        s, s1 = c * self.chunk, min((c + 1) * self.chunk, w.steps)
        while s < s1:
            nxt = min(s1, (s // w.energy_every + 1) * w.energy_every)
            if pairs is not None:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                q.qla_advance(self.ctx, nxt - s)
                b.record()
                pairs.append((a, b, nxt - s))
            else:
                q.qla_advance(self.ctx, nxt - s)
            s = nxt
            if s % w.energy_every == 0:
                k = s // w.energy_every
                q.qla_energy_device(self.ctx, e[k:k + 1])
                if pairs is not None:
                    self.written.append((row, k))
        dst = self.snap[c] if j == 0 and c < len(self.snap) else self.out
        q.qla_get_fields_device(self.ctx, dst, 1)
        return (s1 - c * self.chunk)

    def qla_steps_of(self, i):
        c = i % self.chunks_per_job
        return min((c + 1) * self.chunk, self.w.steps) - c * self.chunk


def bench_job(qla, torch, w, prec, steps, warmup, chunk, tuning=None, potential=0,
              snapshots=0, jobs=1):
    """Time `steps` benchmark steps (chunks of `chunk` QLA steps) of workload w in one
    precision after `warmup` untimed ones; returns (result dict, Job). The caller closes
    the Job (its snapshots hold the physical fields at the end of each chunk of the first
    timed job)."""
    import workloads
    n_dev = torch.from_numpy(workloads.ellipse_index(w.nx, w.ny, w.ellipse)).to("cuda")
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    if not sp:
        raise RuntimeError("bench needs a non-default torch stream")
    job = Job(qla, torch, w, prec, potential, n_dev, sp, chunk, max(1, jobs), snapshots)
    try:
        job.tune(full_tuning(tuning) if tuning else None)
        for i in range(warmup):
            job.run_chunk(i)
        torch.cuda.synchronize()
        pairs = []
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record()
        qsteps = 0
        for i in range(steps):
            qsteps += job.run_chunk(i, pairs)
        t1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
    except Exception:
        job.close()
        raise
    t = t0.elapsed_time(t1) / 1e3 or wall
    rows, pf, fused, cols = job.tuning
    adv_s = sum(a.elapsed_time(b) for a, b, _ in pairs) / 1e3
    launches = sum(k // fused + k % fused for _, _, k in pairs)
    # every launch but the remainder singles applies `fused` steps
    launch_s = adv_s / launches
    k_s = adv_s / sum(k for _, _, k in pairs)           # seconds per QLA step
    e = job.energies.cpu().numpy()
    drift = max((abs(e[row, k] / e[row, 0] - 1) for row, k in job.written if k > 0),
                default=0.0)
    print(f"[bench] {w.name} {prec}: {steps} steps of {chunk} QLA steps in {t:.3f} s "
          f"(wall {wall:.3f} s), step kernel {launch_s * 1e6:.1f} us per launch, "
          f"max |E/E0-1| {drift:.2e}", file=sys.stderr, flush=True)
    sites = w.nx * w.ny
    res = {
        "glups": sites * qsteps / t / 1e9,
        "seconds": t,
        "qla_steps_timed": qsteps,
        "kernel_us": k_s * 1e6,
        "kernel_glups": sites / k_s / 1e9,
        "roofline": step_roofline(w, prec, POTENTIAL_NAMES[potential], job.tuning, launch_s),
        "launch": {"steps_per_launch": fused, "rows_per_segment": rows, "prefetch_rows": pf,
                   "columns_per_lane": cols, "launch_us": round(launch_s * 1e6, 2),
                   "launches_timed": launches,
                   "algorithmic_bytes_per_launch": BYTES_PER_SITE[prec] * sites * fused},
        "energy_max_rel_drift": drift,
    }
    return res, job


def step_roofline(w, prec, potential, tuning, launch_s):
    """Roofline entry of the fused step kernel. `achieved` counts the algorithmic bytes
    of every step a launch applies (56 B per site update in FP64, 28 B in FP32) over the
    measured launch time: with two steps per launch it is an effective rate and `frac`
    may pass 1. `traffic` is the HBM rate from the committed FETCH_SIZE + WRITE_SIZE
    counters of this kernel, workload, potential mode and tuning (None when the kernel
    source or the tuning changed since), `hbm_frac` its fraction of peak, and
    `valu_busy` the share of SIMD issue cycles spent on vector instructions."""
    fused = full_tuning(tuning)[2]
    algorithmic = BYTES_PER_SITE[prec] * w.nx * w.ny * fused
    achieved = algorithmic / launch_s / 1e9
    rec = counter_entry(w, prec, potential, tuning)
    traffic = rec["hbm_bytes_per_launch"] / launch_s / 1e9 if rec else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic, 1) if traffic else None,
            "frac_kind": f"effective: algorithmic bytes of all {fused} steps of a launch",
            "hbm_frac": round(traffic / HBM_PEAK_GBS, 4) if traffic else None,
            "hbm_bytes_per_launch": rec["hbm_bytes_per_launch"] if rec else None,
            "valu_busy": rec.get("valu_busy") if rec else None,
            "counters": (os.path.relpath(counter_path(w), ROOT) if rec else None)}


STEP_SOURCES = ("paper_2604_21128_amd/csrc/qla_step.hip", "paper_2604_21128_amd/csrc/qla_device.h")
# committed counter summaries of the step kernel, per workload
COUNTER_FILES = {"qla_4096_ellipse_20000": "qla_step_ez_4096_ellipse",
                 "qla_8192_bubble_40000": "qla_step_ez_8192_bubble"}


def step_kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_path(w):
    base = COUNTER_FILES.get(w.name, "qla_step_ez_" + w.name)
    return os.path.join(ROOT, "profiles", base + ".json")


def counter_entry(w, prec, potential, tuning=None):
    """The committed counter record of the step kernel for workload w, precision and
    potential mode (and tuning, if given), or None if there is none or the kernel's
    sources changed since the counters were taken."""
    try:
        with open(counter_path(w)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256") != step_kernel_sha() or rec.get("workload") != w.name:
        return None
    for r in rec.get("records", []):
        if r["precision"] != prec or r["potential"] != potential:
            continue
        if tuning is None or full_tuning(r["tuning"]) == full_tuning(tuning):
            return r
    return None


def recorded_tuning(w, potential):
    """Per precision, the tuning under which the committed counters were taken (the
    autotuner's choice then), if the kernel is unchanged since; else the run autotunes."""
    out = {}
    for p in ("f64", "f32"):
        r = counter_entry(w, p, potential)
        if r:
            out[p] = r["tuning"]
    return out


def summarize_counters(args):
    """Turn rocprofv3 outputs into profiles/<name>.{md,json} for the step kernel on
    --workload: one FETCH_SIZE run, one WRITE_SIZE run, one kernel trace and optional
    SQ counter runs, all of the same command. FETCH_SIZE and WRITE_SIZE of every
    kernel are scaled by what the counters read for the 1 GiB reference copy of the same
    run. Kernels are told apart by precision and potential-mode template arguments."""
    import collections
    import csv
    import glob
    import workloads
    fetch_dir, write_dir, trace_dir = args.summarize_counters
    sq_dirs = args.sq_dirs or []
    w = workloads.workload_by_name(args.workload)
    tuning = json.loads(args.tuning_json)
    potential = args.potential
    vcode = POTENTIALS[potential]

    def kernel_key(name):
        if "qla_step_ez_kernel" not in name:
            return None
        prec = "f64" if "<double" in name else "f32"
        # template arguments: <T, VMODE, CLS, ...>
        args_ = name.split("qla_step_ez_kernel<", 1)[1].split(">", 1)[0].split(",")
        vm = int(args_[1].strip())
        return (prec, vm)

    def load(dirs, ctr=None):
        out = collections.defaultdict(lambda: collections.defaultdict(list))
        for d in dirs:
            for fn in glob.glob(os.path.join(d, "*counter_collection.csv")):
                for r in csv.DictReader(open(fn)):
                    if ctr and r["Counter_Name"] != ctr:
                        continue
                    out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return out
    fe, wr = load([fetch_dir], "FETCH_SIZE"), load([write_dir], "WRITE_SIZE")
    ref = [k for k in fe if "copyBuffer" in k]
    if not ref:
        raise SystemExit("no reference copy kernel in the FETCH_SIZE run")
    kib = 1048576.0
    fcopy = max(fe[ref[0]]["FETCH_SIZE"])
    wcopy = max(wr[[k for k in wr if "copyBuffer" in k][0]]["WRITE_SIZE"])
    fs, ws = kib / fcopy, kib / wcopy
    sq = load(sq_dirs)
    n = w.nx * w.ny
    base = os.path.splitext(counter_path(w))[0]
    rec = {"workload": w.name, "kernel_sha256": step_kernel_sha(), "fetch_scale": fs,
           "write_scale": ws, "records": []}
    # keep the records of other potential modes taken under the same kernel
    try:
        old = json.load(open(base + ".json"))
        if old.get("kernel_sha256") == rec["kernel_sha256"]:
            rec["records"] = [r for r in old.get("records", []) if r["potential"] != potential]
    except (OSError, ValueError):
        pass
    avg_ns = collections.defaultdict(list)
    for fn in glob.glob(os.path.join(trace_dir, "*kernel_stats.csv")):
        for r in csv.DictReader(open(fn)):
            avg_ns[r["Name"]].append((float(r["AverageNs"]), int(r["Calls"]),
                                      float(r["MinNs"]), float(r["MaxNs"])))
    for k in fe:
        key = kernel_key(k)
        if not key or key[1] != vcode:
            continue
        prec = key[0]
        e = 8 if prec == "f64" else 4
        t = full_tuning(tuning[prec])
        fused = t[2]
        fr = sum(fe[k]["FETCH_SIZE"]) / len(fe[k]["FETCH_SIZE"])
        wk = [x for x in wr if kernel_key(x) == key]
        wv = sum(wr[wk[0]]["WRITE_SIZE"]) / len(wr[wk[0]]["WRITE_SIZE"])
        r = {"precision": prec, "potential": potential, "tuning": list(t),
             "fetch_kib_raw": fr, "write_kib_raw": wv,
             "hbm_bytes_per_launch": (fr * fs + wv * ws) * 1024,
             "compulsory_bytes_per_launch": 7 * n * e,
             "algorithmic_bytes_per_launch": 7 * n * e * fused}
        for name, rows in avg_ns.items():
            if kernel_key(name) == key:
                r["trace_avg_ns"], r["trace_calls"] = rows[0][0], rows[0][1]
        s = {c: sum(v) / len(v) for x in sq if kernel_key(x) == key for c, v in sq[x].items()}
        if s:
            r["sq"] = s
            if "SQ_ACTIVE_INST_VALU" in s and "GRBM_GUI_ACTIVE" in s:
                # quad-cycles of VALU issue over the SIMDs' quad-cycles (GRBM_GUI_ACTIVE
                # is summed over the 8 XCDs)
                simds, xcds = 1024, 8
                r["valu_busy"] = round(s["SQ_ACTIVE_INST_VALU"]
                                       / (simds * s["GRBM_GUI_ACTIVE"] / xcds / 4), 4)
        rec["records"].append(r)
    rec["records"].sort(key=lambda r: (r["potential"], r["precision"]))
    rel = lambda d: "$R/" + os.path.relpath(os.path.abspath(d), ROOT) \
        if not os.path.relpath(os.path.abspath(d), ROOT).startswith("..") else d
    cmds = getattr(args, "profile_commands", None) or []
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    write_counter_markdown(w, rec, base + ".md", cmds)
    print(open(base + ".md").read())


def write_counter_markdown(w, rec, path, cmds):
    n = w.nx * w.ny
    lines = [f"# qla_step_ez_kernel on the {w.nx}x{w.ny} workload `{w.name}` (MI355X, gfx950)",
             "", f"Step kernel sources sha256 `{rec['kernel_sha256'][:16]}`. A reference 1 GiB "
             f"device copy in the same runs calibrates the counters: FETCH_SIZE x "
             f"{rec['fetch_scale']:.4f}, WRITE_SIZE x {rec['write_scale']:.4f}.", ""]
    if cmds:
        lines += ["Commands (from /tmp with TMPDIR=/tmp; R = repository root):", "", "```"]
        lines += cmds + ["```", ""]
    lines += ["| precision | potential | tuning (rows, prefetch, steps/launch, cols/lane) | "
              "trace avg (us) | HBM read+write per launch (MB) | compulsory one pass (MB) | "
              "HBM / compulsory | measured HBM rate (TB/s) | effective rate (TB/s) | "
              "VALU busy |", "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rec["records"]:
        t_us = r.get("trace_avg_ns", 0) / 1e3
        hbm = r["hbm_bytes_per_launch"]
        comp = r["compulsory_bytes_per_launch"]
        rate = hbm / (t_us * 1e-6) / 1e12 if t_us else float("nan")
        eff = r["algorithmic_bytes_per_launch"] / (t_us * 1e-6) / 1e12 if t_us else float("nan")
        vb = r.get("valu_busy")
        lines.append(f"| {r['precision']} | {r['potential']} | {tuple(r['tuning'])} | "
                     f"{t_us:.1f} | {hbm / 1e6:.1f} | {comp / 1e6:.1f} | {hbm / comp:.3f} | "
                     f"{rate:.2f} | {eff:.2f} | {vb if vb is not None else '-'} |")
    lines += ["", "Compulsory bytes are one read of the three amplitude planes and n and one "
              "write of the amplitude planes (7 planes of n sites), whatever the launch's step "
              "count; the effective rate charges every step of a launch with them (56 B per "
              "site update in FP64, 28 B in FP32) and so can exceed the HBM peak with two "
              "steps per launch. VALU busy: SQ_ACTIVE_INST_VALU quad-cycles over the 1024 "
              "SIMDs' quad-cycles during the dispatch (GRBM_GUI_ACTIVE / 8 XCDs).", ""]
    sq_rows = [r for r in rec["records"] if r.get("sq")]
    if sq_rows:
        names = sorted({c for r in sq_rows for c in r["sq"]})
        lines += ["## SQ and GRBM counters per dispatch (device totals)", "",
                  "| counter | " + " | ".join(f"{r['precision']} {r['potential']}"
                                               for r in sq_rows) + " |",
                  "|---|" + "---|" * len(sq_rows)]
        for c in names:
            lines.append(f"| {c} | " + " | ".join(f"{r['sq'].get(c, float('nan')):.0f}"
                                                  for r in sq_rows) + " |")
        lines.append("")
    with open(path, "w") as f:
        f.write("\n".join(lines))


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


def wgrad_ops(name, Mo, K, P, flops, nbytes):
    """A pointwise layer's weight gradient (Mo x K): the matrix-core weight-gradient kernel and
    its fixed-order sum of the per-block partials where the channel counts fit it (at most
    128 each, at most 8 tiles of 32 x 32, pixels a multiple of 64), else the split GEMM."""
    up = lambda n: 1 if n <= 32 else 2 if n <= 64 else 4 if n <= 128 else 0
    if up(Mo) and up(K) and up(Mo) * up(K) <= 8 and P % 64 == 0:
        return [(name, "wgrad_kernel", flops, nbytes),
                (name + " (block sums)", "wgrad_final_kernel", 0, 0)]
    return [(name, "gemm_kernel", flops, nbytes)]


def fno_ops(H, W, C, m, L, Cin, Cout, C2, nparam, training):
    """The surrogate network's kernel launches for one sample, in launch order: (op, kernel
    name fragment, algorithmic flops, algorithmic HBM bytes). Bytes count one read of each
    input tensor and one write of each output tensor an op needs (BF16 activations, FP32
    spectra, losses and outputs); flops count multiply-adds as two. Inference runs the fused
    projection; training keeps the first projection GEMM and the pre-activations, and runs
    the narrow second projection (3 output channels) and its input gradient on the vector
    units."""
    P = H * W
    act = C * P * 2                     # one BF16 activation tensor
    zx = C * H * 2 * m * 2              # x-transformed rows (BF16, re/im interleaved)
    spec = C * 4 * m * m * 4            # kept modes, FP32 (T, S, dT, dS)
    ops = [("lift", "lift_kernel", 2 * C * Cin * P, Cin * P * 2 + act)]
    # one-pass x and y transforms (Z stays on chip) on grids of a multiple of 32 rows of a
    # multiple of 128 cells up to 512, with at most 16 modes
    one_pass = H % 32 == 0 and W % 128 == 0 and W <= 512 and 1 <= m <= 16
    # the inverse y transform (and the backward dZ, and dS where the one-pass kernel does not
    # fit) as one kernel per plane: m <= 16
    inv_y = 1 <= m <= 16
    # the layer kernel (forward, and the backward input gradient): width 64, rows of a
    # multiple of 256 cells, 2m <= 32
    layer = "layer_mix_kernel" if C == 64 and W % 256 == 0 and 2 * m <= 32 else "gemm_kernel"
    for l in range(L):
        last = l + 1 == L
        if one_pass:
            ops += [(f"L{l} x and y transforms", "spectral_in_kernel",
                     2 * C * H * 2 * m * W + 2 * 2 * C * 4 * m * m * H, act + spec)]
        else:
            ops += [(f"L{l} x transform", "gemm_kernel", 2 * C * H * 2 * m * W, act + zx),
                    (f"L{l} y transform (re)", "gemm_kernel", 2 * C * 4 * m * m * H,
                     zx // 2 + spec),
                    (f"L{l} y transform (im)", "gemm_kernel", 2 * C * 4 * m * m * H,
                     zx // 2 + 2 * spec)]
        ops += [(f"L{l} mode mixing", "mix_forward_kernel", 8 * C * C * 2 * m * m,
                 spec + 2 * C * C * 2 * m * m * 4 + spec // 2)]
        if inv_y:
            ops += [(f"L{l} inverse y", "spectral_out_kernel", 2 * 2 * C * H * m * 4 * m,
                     spec // 2 + zx)]
        else:
            ops += [(f"L{l} inverse y (re)", "gemm_kernel", 2 * C * H * m * 4 * m,
                     spec // 2 + zx // 2),
                    (f"L{l} inverse y (im)", "gemm_kernel", 2 * C * H * m * 4 * m,
                     spec // 2 + zx // 2)]
        ops += [(f"L{l} pointwise + inverse x + GELU", layer,
                 2 * C * C * P + 2 * C * H * W * 2 * m,
                 act + zx + act * (2 if training and not last else 1))]
    if not training:
        ops += [("projection (fused)", "projection_fused_kernel", 2 * C2 * C * P + 2 * Cout * C2 * P,
                 act + Cout * P * 4),
                ("output copy", "copyBuffer", 0, 2 * Cout * P * 4)]
        return ops
    hid = C2 * P * 2
    # training's first projection: its own kernel for width 64 on rows of a multiple of 256
    # cells with 64 or 128 projection channels, else the GEMM
    # (with the narrow second projection formed in the same pass from the staged hidden layer)
    proj1 = ("proj1_train_kernel" if C == 64 and W % 256 == 0 and C2 % 64 == 0 and C2 <= 128
             else "gemm_kernel")
    if proj1 == "proj1_train_kernel" and Cout <= 4:
        ops += [("projection 1 + projection 2", proj1, 2 * C2 * C * P + 2 * Cout * C2 * P,
                 act + 2 * hid + Cout * P * 4)]
    else:
        ops += [("projection 1", proj1, 2 * C2 * C * P, act + 2 * hid),
                ("projection 2", "narrow_projection_kernel", 2 * Cout * C2 * P,
                 hid + Cout * P * 4)]
    ops += [
            ("loss sums", "loss_partial_kernel", 4 * Cout * P, Cout * P * 6),
            ("loss sums, blocks in order", "loss_sums_kernel", 0, 0),
            ("loss", "loss_final_kernel", 0, 0),
            ("loss gradient", "loss_grad_kernel", 3 * Cout * P, Cout * P * (6 + 2))]
    ops += wgrad_ops("projection 2 weight grad", Cout, C2, P, 2 * Cout * C2 * P,
                     Cout * P * 2 + hid)
    if proj1 == "proj1_train_kernel" and Cout <= 4:
        # dzq (stored) and dz = Q1^T dzq in one pass over zq
        ops += [("projection 2 + projection 1 input grads", "proj_grad_kernel",
                 2 * Cout * C2 * P + 2 * C2 * C * P, Cout * P * 2 + 2 * hid + act)]
        ops += wgrad_ops("projection 1 weight grad", C2, C, P, 2 * C2 * C * P, hid + act)
    else:
        ops += [("projection 2 input grad", "narrow_projection_grad_kernel", 2 * Cout * C2 * P,
                 Cout * P * 2 + 2 * hid)]
        ops += wgrad_ops("projection 1 weight grad", C2, C, P, 2 * C2 * C * P, hid + act)
        ops += [("projection 1 input grad", "gemm_kernel", 2 * C2 * C * P, hid + act)]
    for l in reversed(range(L)):
        ops += wgrad_ops(f"L{l} weight grad", C, C, P, 2 * C * C * P, 2 * act)
        if one_pass:
            # dU = dz IX^T and dS = IY^T dU in one pass over dz (dU stays on chip)
            ops += [(f"L{l} dS = IY^T (dz IX^T)", "spectral_in_kernel",
                     2 * C * H * 2 * m * W + 2 * 2 * C * 4 * m * m * H, act + spec)]
        else:
            ops += [(f"L{l} dU = dz IX^T", "gemm_kernel", 2 * C * H * W * 2 * m, act + zx)]
            if inv_y:
                ops += [(f"L{l} dS", "spectral_y_kernel", 2 * 2 * C * 4 * m * m * H, zx + spec)]
            else:
                ops += [(f"L{l} dS (re)", "gemm_kernel", 2 * C * 4 * m * m * H, zx // 2 + spec),
                        (f"L{l} dS (im)", "gemm_kernel", 2 * C * 4 * m * m * H,
                         zx // 2 + 2 * spec)]
        ops += [(f"L{l} mode-mixing weight grad", "mix_backward_weight_kernel",
                 8 * C * C * 2 * m * m, 2 * spec),
                (f"L{l} mode-mixing input grad", "mix_backward_input_kernel",
                 8 * C * C * 2 * m * m, 2 * spec)]
        if inv_y:
            ops += [(f"L{l} dZ", "spectral_out_kernel", 2 * 2 * C * H * m * 4 * m, spec // 2 + zx)]
        else:
            ops += [(f"L{l} dZ (re)", "gemm_kernel", 2 * C * H * m * 4 * m, spec // 2 + zx // 2),
                    (f"L{l} dZ (im)", "gemm_kernel", 2 * C * H * m * 4 * m, spec // 2 + zx // 2)]
        ops += [(f"L{l} dv = W^T dz + dZ Fx^T, GELU'", layer,
                 2 * C * C * P + 2 * C * H * W * 2 * m, act + zx + (act if l > 0 else 0) + act)]
    ops += wgrad_ops("lift weight grad", C, Cin, P, 2 * C * Cin * P, act + Cin * P * 2)
    return ops


FNO_SHAPE = dict(channels=64, modes=12, layers=4, proj_channels=128)


def fno_marker(qla, torch, z, e):
    """A dispatch of a kernel the network never launches (the energy of a tiny plane z,
    into e), which delimits the measured passes in a kernel trace."""
    qla.qla_energy_noalloc(z[0], z[1], z[2], 8, 8, 8, qla.QLA_F64, e,
                           torch.cuda.current_stream().cuda_stream)


def fno_kernel_study(qla, torch, args):
    """The surrogate network's kernels alone at the configured shape (side^2 lattice,
    width 64, 12 modes per axis, 4 layers, projection 128, batch --batch) on random BF16
    inputs and targets: --fno-reps forward passes and training steps, each timed with
    events; per-sample algorithmic flops and bytes from fno_ops. Marker dispatches
    (fno_marker) bracket the measured forward passes and training steps."""
    from paper_2604_21128_amd import surrogate as S
    B, side, reps = args.batch, args.side, args.fno_reps
    sur = S.Surrogate(side, side, max_batch=B, seed=args.seed, **FNO_SHAPE)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed)
    x = torch.randn((B, 4, side, side), device="cuda", generator=gen).to(torch.bfloat16)
    y = torch.randn((B, 3, side, side), device="cuda", generator=gen).to(torch.bfloat16)
    x, y = x.view(torch.int16), y.view(torch.int16)
    out = torch.empty((B, 3, side, side), dtype=torch.float32, device="cuda")
    mz = torch.zeros((3, 8, 8), dtype=torch.float64, device="cuda")
    me = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(2):
        sur.predict(x, out)
        sur.train_step(x, y, 1e-5)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    fno_marker(qla, torch, mz, me)
    a, b = ev(), ev()
    a.record()
    for _ in range(reps):
        sur.predict(x, out)
    b.record()
    fno_marker(qla, torch, mz, me)
    c, d = ev(), ev()
    c.record()
    for _ in range(reps):
        sur.train_step(x, y, 1e-5)
    d.record()
    fno_marker(qla, torch, mz, me)
    torch.cuda.synchronize()
    t_fwd = a.elapsed_time(b) / 1e3 / reps
    t_train = c.elapsed_time(d) / 1e3 / reps
    nparam = int(qla.qla_fno_param_count(sur.h))
    sur.close()
    shape = (side, side, FNO_SHAPE["channels"], FNO_SHAPE["modes"], FNO_SHAPE["layers"], 4, 3,
             FNO_SHAPE["proj_channels"], nparam)
    f_ops, t_ops = fno_ops(*shape, training=False), fno_ops(*shape, training=True)
    ff, fb = sum(o[2] for o in f_ops), sum(o[3] for o in f_ops)
    tf, tb = sum(o[2] for o in t_ops), sum(o[3] for o in t_ops) + 7 * nparam * 4 / B
    return {"workload": f"fno_{side}_width64_modes12_layers4_batch{B}", "batch": B,
            "params": nparam, "reps": reps,
            "forward": {"seconds_per_batch": t_fwd, "samples_per_s": B / t_fwd,
                        "gflop_per_sample": ff / 1e9, "gbytes_per_sample": fb / 1e9,
                        "tflops": ff * B / t_fwd / 1e12, "tbytes_per_s": fb * B / t_fwd / 1e12},
            "training": {"seconds_per_step": t_train, "samples_per_s": B / t_train,
                         "gflop_per_sample": tf / 1e9, "gbytes_per_sample": tb / 1e9,
                         "tflops": tf * B / t_train / 1e12,
                         "tbytes_per_s": tb * B / t_train / 1e12}}


def summarize_fno(args):
    """profiles/surrogate_fno_kernels.{md,json} from a kernel trace and FETCH_SIZE /
    WRITE_SIZE runs of `bench.py --fno-kernels`: every dispatch between the last three
    marker dispatches (one forward pass and one training step when --fno-reps 1) is matched
    in order to fno_ops; durations from the trace, HBM bytes from the counters (scaled by
    the reference copy of the same run), algorithmic flops and bytes from the model."""
    import csv
    import glob
    trace_dir, fetch_dir, write_dir = args.summarize_fno
    B, side = args.batch, args.side

    def dispatches(d, counter=None):
        rows = []
        pat = "*kernel_trace.csv" if counter is None else "*counter_collection.csv"
        for fn in glob.glob(os.path.join(d, pat)):
            for r in csv.DictReader(open(fn)):
                if counter is not None and r["Counter_Name"] != counter:
                    continue
                key = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
                val = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) \
                    if counter is None else float(r["Counter_Value"])
                rows.append((key, r["Kernel_Name"], val))
        rows.sort()
        return [(n, v) for _, n, v in rows]

    def sections(rows):
        idx = [i for i, (n, _) in enumerate(rows) if "energy_final_kernel" in n]
        if len(idx) < 3:
            raise SystemExit("fewer than three marker dispatches")
        i0, i1, i2 = idx[-3:]
        strip = lambda s: [r for r in s if "energy_partial_kernel" not in r[0]]
        return strip(rows[i0 + 1:i1]), strip(rows[i1 + 1:i2])
    tr = sections(dispatches(trace_dir))
    fe_all, wr_all = dispatches(fetch_dir, "FETCH_SIZE"), dispatches(write_dir, "WRITE_SIZE")
    fcopy = max(v for n, v in fe_all if "copyBuffer" in n)
    wcopy = max(v for n, v in wr_all if "copyBuffer" in n)
    fs, ws = 1048576.0 / fcopy, 1048576.0 / wcopy
    fe, wr = sections(fe_all), sections(wr_all)
    nparam = args.fno_params
    shape = (side, side, FNO_SHAPE["channels"], FNO_SHAPE["modes"], FNO_SHAPE["layers"], 4, 3,
             FNO_SHAPE["proj_channels"], nparam)
    out = {"batch": B, "side": side, "fetch_scale": fs, "write_scale": ws, "passes": {}}
    lines = [f"# Surrogate network kernels: roofline per launch (MI355X, gfx950)", "",
             f"Fourier neural operator on {side}x{side} lattices, width 64, 12 modes per axis, "
             f"4 layers, projection 128, batch {B}, {nparam} parameters; random BF16 inputs and "
             "targets (`bench.py --fno-kernels`). Flops and bytes are algorithmic (fno_ops in "
             "bench.py: multiply-adds count two; one read of every input tensor and one write of "
             "every output tensor an op needs); HBM bytes are FETCH_SIZE + WRITE_SIZE scaled by "
             f"the 1 GiB reference copy of the same runs (x {fs:.4f}, x {ws:.4f}). Peaks: BF16 "
             "dense MFMA 2500 TFLOP/s, HBM 8 TB/s.", ""]
    cmds = getattr(args, "profile_commands", None) or []
    if cmds:
        lines += ["Commands (from /tmp with TMPDIR=/tmp; R = repository root):", "", "```"]
        lines += cmds + ["```", ""]
    for pi, name in enumerate(("forward (inference)", "training step")):
        ops = fno_ops(*shape, training=(pi == 1))
        rows = tr[pi]
        j = 0
        table, tot = [], {"us": 0.0, "flop": 0.0, "bytes": 0.0, "hbm": 0.0}
        for k, (n, dur) in enumerate(rows):
            f_b = fe[pi][k][1] * fs * 1024 if k < len(fe[pi]) else float("nan")
            w_b = wr[pi][k][1] * ws * 1024 if k < len(wr[pi]) else float("nan")
            short = n.replace("(anonymous namespace)::", "").split("(")[0]
            if j < len(ops) and ops[j][1] in n:
                op, _, fl, by = ops[j]
                fl, by = fl * B, by * B
                j += 1
            else:
                op, fl, by = "(" + short.split("::")[-1][:40] + ")", 0.0, 0.0
                if "adam_kernel" in n:
                    op, by = "Adam update", 7 * nparam * 4
                elif "cast_kernel" in n:
                    op = "BF16 weight copy"
            us = dur / 1e3
            hbm = f_b + w_b
            table.append({"op": op, "kernel": short[:60], "us": us, "gflop": fl / 1e9,
                          "mb": by / 1e6, "hbm_mb": hbm / 1e6,
                          "tflops": fl / (us * 1e-6) / 1e12 if us else 0.0,
                          "tbs": hbm / (us * 1e-6) / 1e12 if us else 0.0})
            tot["us"] += us
            tot["flop"] += fl
            tot["bytes"] += by
            tot["hbm"] += hbm
        if j != len(ops):
            raise SystemExit(f"{name}: matched {j} of {len(ops)} modelled ops")
        out["passes"][name] = {"ops": table, "total": tot}
        lines += [f"## {name}: {len(rows)} dispatches, {tot['us']:.0f} us of kernel time per "
                  f"batch ({B / (tot['us'] * 1e-6):.0f} samples/s of kernel time)", "",
                  f"Whole pass: {tot['flop'] / 1e9:.1f} GFLOP, {tot['bytes'] / 1e9:.2f} GB "
                  f"algorithmic, {tot['hbm'] / 1e9:.2f} GB measured HBM; "
                  f"{tot['flop'] / (tot['us'] * 1e-6) / 1e12:.1f} TFLOP/s "
                  f"({tot['flop'] / (tot['us'] * 1e-6) / 2.5e15:.3f} of the MFMA peak), "
                  f"{tot['hbm'] / (tot['us'] * 1e-6) / 1e12:.2f} TB/s measured "
                  f"({tot['hbm'] / (tot['us'] * 1e-6) / 8e12:.3f} of peak).", "",
                  "| op | kernel | us | GFLOP | algorithmic MB | HBM MB | TFLOP/s | HBM TB/s | "
                  "bound, fraction |", "|---|---|---|---|---|---|---|---|---|"]
        for r in table:
            fm, fh = r["tflops"] / 2500.0, r["tbs"] / 8.0
            bound = f"mfma {fm:.3f}" if fm > fh else f"hbm {fh:.3f}"
            lines.append(f"| {r['op']} | `{r['kernel']}` | {r['us']:.1f} | {r['gflop']:.2f} | "
                         f"{r['mb']:.1f} | {r['hbm_mb']:.1f} | {r['tflops']:.1f} | "
                         f"{r['tbs']:.2f} | {bound} |")
        lines.append("")
    base = os.path.join(ROOT, "profiles", "surrogate_fno_kernels")
    with open(base + ".json", "w") as f:
        json.dump(out, f, indent=1)
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def summarize_batch(args):
    """profiles/batched_512_trace.md from a kernel trace of `bench.py --batched`: the last
    captured run is the last unbroken sequence of batched-kernel dispatches as long as the
    plan's pass count; per pass its duration, the idle time before it, and the rate of the
    site updates it applies (every lattice still running advances two steps per pass)."""
    import csv
    import glob
    import numpy as np
    import workloads
    trace_dir = args.summarize_batch
    rows = []
    for fn in glob.glob(os.path.join(trace_dir, "*kernel_trace.csv")):
        for r in csv.DictReader(open(fn)):
            rows.append((int(r.get("Dispatch_Id") or r.get("Correlation_Id")), r["Kernel_Name"],
                         float(r["Start_Timestamp"]), float(r["End_Timestamp"])))
    rows.sort()
    inst = workloads.sample_instances(args.instances, seed=0)
    fused = args.batch_steps_per_pass
    sides = np.array([i.n_side for i in inst], dtype=np.float64)
    passes_of = np.array([i.steps // fused for i in inst])
    npass = int(passes_of.max())
    runs, cur = [], []
    for r in rows:
        if "qla_batch_kernel" in r[1]:
            cur.append(r)
        else:
            if cur:
                runs.append(cur)
            cur = []
    if cur:
        runs.append(cur)
    full = [r for r in runs if len(r) == npass]
    if not full:
        raise SystemExit(f"no run of {npass} batched dispatches in the trace")
    run = full[-1]
    start = np.array([r[2] for r in run])
    end = np.array([r[3] for r in run])
    dur = (end - start) * 1e-9
    gap = np.concatenate([[0.0], np.maximum(start[1:] - end[:-1], 0.0) * 1e-9])
    p = np.arange(npass)
    work = np.array([fused * (sides[passes_of > k] ** 2).sum() for k in p])
    span = (end[-1] - start[0]) * 1e-9
    lines = ["# Batched run: where the time goes (MI355X, gfx950)", "",
             f"Kernel trace of the captured run of {args.instances} lattices (sides 256-1024, "
             f"4 x side steps each, FP32, {fused} steps per pass): {npass} launches of `{run[0][1].replace('(anonymous namespace)::', '').split('(')[0]}`.", ""]
    cmds = getattr(args, "profile_commands", None) or []
    if cmds:
        lines += ["Commands (from /tmp with TMPDIR=/tmp; R = repository root):", "", "```"]
        lines += cmds + ["```", ""]
    total = work.sum()
    lines += [f"- span of the run: {span * 1e3:.1f} ms; kernels busy {dur.sum() * 1e3:.1f} ms; "
              f"idle between launches {gap.sum() * 1e3:.1f} ms ({gap.sum() / span:.1%}; median gap "
              f"{np.median(gap[1:]) * 1e6:.1f} us)",
              f"- site updates {total:.3e}: {total / span / 1e9:.1f} GLUPS over the span, "
              f"{total / dur.sum() / 1e9:.1f} GLUPS over kernel time", "",
              "| passes | lattices running | site updates per pass | mean launch (us) | "
              "mean gap (us) | GLUPS in these launches | share of the span |",
              "|---|---|---|---|---|---|---|"]
    edges = [0, 64, 128, 256, 384, 512, 768, 1024, 1536, npass]
    for a, b in zip(edges[:-1], edges[1:]):
        if a >= npass:
            break
        sl = slice(a, min(b, npass))
        running = int((passes_of > a).sum())
        lines.append(f"| {a}-{min(b, npass) - 1} | {running}-{int((passes_of > min(b, npass) - 1).sum())} | "
                     f"{work[sl].mean():.3e} | {dur[sl].mean() * 1e6:.1f} | {gap[sl].mean() * 1e6:.1f} | "
                     f"{work[sl].sum() / dur[sl].sum() / 1e9:.1f} | "
                     f"{(dur[sl].sum() + gap[sl].sum()) / span:.1%} |")
    base = os.path.join(ROOT, "profiles", "batched_512_trace")
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


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
    ap.add_argument("--steps", type=int, default=20,
                    help="timed benchmark steps: chunks of --chunk-steps QLA steps of the "
                         "workload's job (20 chunks of 2000 = the whole 40000-step job)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--chunk-steps", type=int, default=0,
                    help="QLA steps per benchmark step (default: 2000 on the 8192^2 bubble "
                         "job, the whole job on the others)")
    ap.add_argument("--qla-steps", type=int, default=0, help="override the QLA step count")
    ap.add_argument("--precisions", default="f64,f32")
    ap.add_argument("--potential", default="skew_half", choices=sorted(POTENTIALS),
                    help="potential mode of the measured job (skew_half: the default "
                         "half-angle potentials; bstream: the B-streaming scheme)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the copy-bandwidth probe and the potential-mode drift run (for "
                         "profiling runs, whose per-kernel averages must cover the job only)")
    ap.add_argument("--cpu-sample-steps", type=int, default=0,
                    help="oracle steps timed for cpu_baseline (default: 5 at 8192^2, 12 at "
                         "4096^2, about 15 s on 16 host threads)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR",
                                                               "TRACE_DIR"),
                    help="write profiles/ counter summaries for --workload, --potential and "
                         "--tuning-json from rocprofv3 output folders")
    ap.add_argument("--sq-dirs", nargs="*", default=[],
                    help="with --summarize-counters: folders of SQ/GRBM counter runs")
    ap.add_argument("--profile-commands-file", default="",
                    help="with --summarize-counters: text file of the commands that made the "
                         "counter runs, copied into the summary")
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
    ap.add_argument("--fno-kernels", action="store_true",
                    help="the surrogate network's kernels alone (--side, --batch, --fno-reps): "
                         "forward and training throughput with per-sample flops and bytes; "
                         "prints its own JSON line")
    ap.add_argument("--fno-reps", type=int, default=20)
    ap.add_argument("--summarize-fno", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/surrogate_fno_kernels.{md,json} from a kernel trace and "
                         "FETCH_SIZE / WRITE_SIZE runs of --fno-kernels --fno-reps 1")
    ap.add_argument("--summarize-batch", metavar="TRACE_DIR",
                    help="write profiles/batched_512_trace.md from a kernel trace of --batched")
    ap.add_argument("--batch-steps-per-pass", type=int, default=2,
                    help="with --summarize-batch: the plan's steps per pass")
    ap.add_argument("--fno-params", type=int, default=0,
                    help="with --summarize-fno: the network's parameter count")
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
        if args.profile_commands_file:
            with open(args.profile_commands_file) as f:
                args.profile_commands = [l.rstrip("\n") for l in f if l.strip()]
        summarize_counters(args)
        return
    if args.summarize_batch:
        if args.profile_commands_file:
            with open(args.profile_commands_file) as f:
                args.profile_commands = [l.rstrip("\n") for l in f if l.strip()]
        summarize_batch(args)
        return
    if args.summarize_fno:
        if args.profile_commands_file:
            with open(args.profile_commands_file) as f:
                args.profile_commands = [l.rstrip("\n") for l in f if l.strip()]
        summarize_fno(args)
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
    if args.fno_kernels:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = fno_kernel_study(qla, torch, args)
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
    chunk = args.chunk_steps or default_chunk(w)
    precs = [p for p in args.precisions.split(",") if p]
    pot = POTENTIALS[args.potential]
    stream = torch.cuda.Stream()   # default priority
    cpj = -(-w.steps // chunk)
    keep = min(args.steps, cpj) if len(precs) > 1 else 0
    jobs = -(-args.steps // cpj)
    results, snaps, energies = {}, {}, {}
    with torch.cuda.stream(stream):
        forced = json.loads(args.tuning_json) if args.tuning_json else \
            recorded_tuning(w, args.potential)
        for p in precs:
            r, job = bench_job(qla, torch, w, p, args.steps, args.warmup, chunk, forced.get(p),
                               pot, snapshots=keep, jobs=jobs)
            results[p] = r
            snaps[p], energies[p] = job.snap, job.energies[0].cpu().numpy()
            qla.qla_destroy(job.ctx)      # the snapshots stay for the comparison
        comparison = compare_precisions(torch, w, chunk, precs, snaps, energies) \
            if keep else None
        snaps.clear()
    main_p = precs[0]
    r = results[main_p]
    line = {
        "metric": METRIC,
        "value": round(r["glups"], 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["seconds"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_p,
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "qla_steps": w.steps,
                   "qla_steps_per_bench_step": chunk, "qla_steps_timed": r["qla_steps_timed"],
                   "energy_every": w.energy_every, "snapshot_every": chunk, "delta": w.delta,
                   "potential": args.potential,
                   "ellipse": dataclasses.asdict(w.ellipse),
                   "packet": dataclasses.asdict(w.packet)},
        "roofline": r["roofline"],
        "launch": r["launch"],
        "step_kernel_us": round(r["kernel_us"], 2),
        "step_kernel_glups": round(r["kernel_glups"], 2),
        "energy_max_rel_drift": r["energy_max_rel_drift"],
    }
    for p in precs[1:]:
        rp = results[p]
        line[p] = {"value": round(rp["glups"], 3), "unit": "GLUPS",
                   "ms_per_step": round(rp["seconds"] / args.steps * 1e3, 3),
                   "roofline": rp["roofline"], "launch": rp["launch"],
                   "step_kernel_us": round(rp["kernel_us"], 2),
                   "energy_max_rel_drift": rp["energy_max_rel_drift"]}
    if comparison:
        line[precs[1]]["vs_" + main_p] = comparison
    if not args.no_extras:
        with torch.cuda.stream(stream):
            line["copy_gbs"] = copy_bandwidth(torch)
            line["potential_modes_small_workload"] = paper_mode_drift(qla, torch)
            if w.name == HEADLINE and args.potential == "skew_half":
                # the 4096^2 ellipse job, whole job per step, both precisions and the
                # B-streaming scheme
                w2 = workloads.plain_4096()
                extra = {}
                for p in precs:
                    tun = recorded_tuning(w2, "skew_half").get(p)
                    rp, job = bench_job(qla, torch, w2, p, 1, 1, w2.steps, tun, pot)
                    job.close()
                    extra[p] = {"value": round(rp["glups"], 3), "unit": "GLUPS",
                                "roofline": rp["roofline"], "launch": rp["launch"],
                                "energy_max_rel_drift": rp["energy_max_rel_drift"]}
                tun = recorded_tuning(w2, "bstream").get("f64")
                rb, job = bench_job(qla, torch, w2, "f64", 1, 1, w2.steps, tun,
                                    POTENTIALS["bstream"])
                job.close()
                extra["bstream_f64"] = {"value": round(rb["glups"], 3), "unit": "GLUPS",
                                        "roofline": rb["roofline"], "launch": rb["launch"],
                                        "energy_max_rel_drift": rb["energy_max_rel_drift"]}
                line[w2.name] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps or default_cpu_steps(w))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
