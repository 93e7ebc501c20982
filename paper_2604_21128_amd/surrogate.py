"""Learned surrogate of long QLA runs, with QLA as its reference and fallback.

A Fourier neural operator (the qla_fno_* calls of libqla) maps a lattice's medium
and initial fields, (n - n_shift, q2, q3, q4), to its fields (q2, q3, q4) a fixed
number of QLA steps (Eq. 2e14) later. Training pairs come from the batched QLA
kernels; training and inference run on the library's BF16 matrix-core kernels. A
prediction is accepted only when the energy of Eq. (A13), which QLA conserves, is
within a relative tolerance of the initial energy; otherwise the lattice is advanced
by QLA itself.

This module only marshals arguments and sequences library calls: torch supplies
device memory, streams and timing events. Every call is enqueued on the torch stream
that is current when a `Surrogate` is made, so torch's reuse of freed memory is
ordered with the library's work.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Optional, Sequence

import numpy as np
import torch

from . import qla


@dataclasses.dataclass(frozen=True)
class PacketSpec:
    """Arguments of qla_init_packet (a Gaussian-envelope E_z packet)."""
    x0: float
    y0: float
    sigma: float
    lam: float
    phi: float = 0.0
    amp: float = 1.0
    planar: bool = True


class Surrogate:
    """Owns one qla_fno network of fixed shape on the current torch stream."""

    IN_CHANNELS, OUT_CHANNELS = 4, 3

    def __init__(self, height: int, width: int, channels: int = 64, modes: int = 12,
                 layers: int = 4, proj_channels: int = 128, max_batch: int = 16, seed: int = 0,
                 n_shift: float = 2.0):
        self.H, self.W, self.max_batch, self.n_shift = height, width, max_batch, n_shift
        self.shape = dict(channels=channels, modes=modes, layers=layers,
                          proj_channels=proj_channels)
        self.stream = torch.cuda.current_stream()
        self.h = qla.qla_fno_create(height, width, self.IN_CHANNELS, self.OUT_CHANNELS, channels,
                                    modes, layers, proj_channels, max_batch, seed,
                                    self.stream.cuda_stream)

    def close(self):
        if self.h:
            qla.qla_fno_destroy(self.h)
            self.h = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def sample_in(self) -> int:
        return self.IN_CHANNELS * self.H * self.W

    @property
    def sample_out(self) -> int:
        return self.OUT_CHANNELS * self.H * self.W

    def params(self) -> np.ndarray:
        return qla.qla_fno_get_params(self.h)

    def set_params(self, p: np.ndarray) -> None:
        qla.qla_fno_set_params(self.h, p)

    def train_step(self, inputs: torch.Tensor, targets: torch.Tensor, lr: float,
                   loss_out: Optional[torch.Tensor] = None) -> None:
        b = inputs.shape[0]
        qla.qla_fno_train_step(self.h, inputs, targets, b, lr, loss_out)

    def predict(self, inputs: torch.Tensor, out: torch.Tensor,
                energy_out: Optional[torch.Tensor] = None) -> None:
        """Forward pass of a batch; optionally the energy of each prediction."""
        b = inputs.shape[0]
        qla.qla_fno_forward(self.h, inputs, b, out)
        if energy_out is not None:
            qla.qla_fno_output_energy(self.h, b, energy_out)


def _bf16_planes(count: int, planes: int, H: int, W: int, device) -> torch.Tensor:
    # BF16 bit patterns held in int16 storage (the library reads raw 16-bit values)
    return torch.empty((count, planes, H, W), dtype=torch.int16, device=device)


@dataclasses.dataclass
class Pairs:
    inputs: torch.Tensor              # [N, 4, H, W] BF16 bits: n - n_shift, q2, q3, q4 at t = 0
    targets: torch.Tensor             # [N, 3, H, W] BF16 bits: q2, q3, q4 after `steps`
    e0: torch.Tensor                  # [N] float64 initial energy (Eq. A13)
    targets_f32: Optional[torch.Tensor]  # [N, 3, H, W] float32, if kept
    qla_seconds: float                # time of the QLA runs alone
    site_updates: int


def qla_pairs(index_fn: Callable[[int, int], torch.Tensor], count: int,
              packets: Sequence[PacketSpec], delta: float, steps: int, n_shift: float = 2.0,
              chunk: int = 512, keep_f32: bool = False, precision: int = qla.QLA_F32,
              log=None) -> Pairs:
    """Run QLA on `count` (n, packet) pairs with the batched kernels and pack the pairs.

    index_fn(first, k) returns the refractive indices of lattices first .. first + k - 1
    as a float64 [k, H, W] GPU tensor. QLA runs in chunks of `chunk` lattices, each one
    planned batch run (captured graph) of `steps` steps.
    """
    N = count
    probe = index_fn(0, 1)
    _, H, W = probe.shape
    dev = probe.device
    del probe
    stream = torch.cuda.current_stream()
    inputs = _bf16_planes(N, 4, H, W, dev)
    targets = _bf16_planes(N, 3, H, W, dev)
    e0 = torch.zeros(N, dtype=torch.float64, device=dev)
    t32 = torch.empty((N, 3, H, W), dtype=torch.float32, device=dev) if keep_f32 else None
    stage = torch.empty((3, H, W), dtype=torch.float64, device=dev)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    qla_s, updates = 0.0, 0
    for c0 in range(0, N, chunk):
        k = min(chunk, N - c0)
        ns = index_fn(c0, k)
        b = qla.qla_batch_create([W] * k, [H] * k, [delta] * k, precision=precision,
                                 hip_stream=stream.cuda_stream)
        try:
            for i in range(k):
                ctx = qla.qla_batch_context(b, i)
                p = packets[c0 + i]
                qla.qla_set_index_device(ctx, ns[i], W)
                qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)
                qla.qla_energy_device(ctx, e0[c0 + i:c0 + i + 1])
                qla.qla_get_fields_device(ctx, stage)
                qla.qla_fno_pack(stage, ns[i], W, H, n_shift, inputs[c0 + i], None,
                                 stream.cuda_stream)
            qla.qla_batch_plan(b, [steps] * k, 0)
            start.record(stream)
            qla.qla_batch_run(b)
            stop.record(stream)
            for i in range(k):
                ctx = qla.qla_batch_context(b, i)
                qla.qla_get_fields_device(ctx, stage)
                qla.qla_fno_pack(stage, None, W, H, 0.0, None, targets[c0 + i],
                                 stream.cuda_stream)
                if t32 is not None:
                    t32[c0 + i].copy_(stage)
            stop.synchronize()
            qla_s += start.elapsed_time(stop) / 1e3
            updates += qla.qla_batch_plan_info(b)["site_updates"]
        finally:
            qla.qla_batch_destroy(b)
        del ns
        if log:
            log(f"qla pairs {c0 + k}/{N}: {qla_s:.2f} s of QLA, "
                f"{updates / max(qla_s, 1e-9) / 1e9:.1f} GLUPS")
    return Pairs(inputs, targets, e0, t32, qla_s, updates)


def train(sur: Surrogate, inputs: torch.Tensor, targets: torch.Tensor, batch: int,
          epochs: float, lr: float, lr_final: float = 0.02, seed: int = 0,
          time_budget_s: Optional[float] = None, log=None, log_every: int = 200) -> dict:
    """Adam on the relative-L2 loss over contiguous batches in a shuffled order.

    The learning rate follows a cosine from lr down to lr * lr_final over the run.
    Returns the per-step losses and the wall time.
    """
    N = inputs.shape[0]
    nb = N // batch
    total = max(1, int(round(epochs * nb)))
    losses = torch.zeros(total, dtype=torch.float32, device=inputs.device)
    rng = np.random.default_rng(seed)
    order = np.array([], dtype=np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for step in range(total):
        if order.size == 0:
            order = rng.permutation(nb)
        j = int(order[0]) * batch
        order = order[1:]
        a = lr * (lr_final + (1 - lr_final) * 0.5 * (1 + math.cos(math.pi * step / total)))
        sur.train_step(inputs[j:j + batch], targets[j:j + batch], a, losses[step:step + 1])
        done = step + 1
        if (step + 1) % log_every == 0 or step + 1 == total:
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            recent = float(losses[max(0, step + 1 - log_every):step + 1].mean())
            if log:
                log(f"train step {step + 1}/{total}: loss {recent:.4f}, {el:.1f} s")
            if time_budget_s is not None and el > time_budget_s:
                break
    torch.cuda.synchronize()
    return {"losses": losses[:done].cpu().numpy(), "seconds": time.perf_counter() - t0,
            "steps": done}


def predict_all(sur: Surrogate, inputs: torch.Tensor, batch: int):
    """FP32 predictions [N, 3, H, W] and their energies [N] (float64)."""
    N = inputs.shape[0]
    out = torch.empty((N, 3, sur.H, sur.W), dtype=torch.float32, device=inputs.device)
    energy = torch.zeros(N, dtype=torch.float64, device=inputs.device)
    for j in range(0, N, batch):
        k = min(batch, N - j)
        sur.predict(inputs[j:j + k], out[j:j + k], energy[j:j + k])
    return out, energy


def band_fractions(sur: Surrogate, inputs: torch.Tensor, batch: int, first_channel: int = 1,
                   channels: int = 3) -> torch.Tensor:
    """Share of each input's field energy (planes q2, q3, q4 by default) in the modes the
    Fourier layers keep, [N] float64 (qla_fno_band_fraction)."""
    N = inputs.shape[0]
    frac = torch.zeros(N, dtype=torch.float64, device=inputs.device)
    for j in range(0, N, batch):
        k = min(batch, N - j)
        qla.qla_fno_band_fraction(sur.h, inputs[j:j + k], k, first_channel, channels,
                                  frac[j:j + k])
    return frac


def accept(energy: torch.Tensor, e0: torch.Tensor, tol: float = 1e-2) -> torch.Tensor:
    """The acceptance test: |E_pred / E_0 - 1| < tol (QLA conserves E exactly)."""
    return (energy / e0 - 1.0).abs() < tol


def run_with_fallback(sur: Surrogate, inputs: torch.Tensor, e0: torch.Tensor,
                      index_fn: Callable[[int, int], torch.Tensor],
                      packets: Sequence[PacketSpec], delta: float, steps: int, batch: int,
                      tol: float = 1e-2, chunk: int = 512, band_min: Optional[float] = None):
    """Surrogate first, QLA for every rejected lattice. Returns the fields [N, 3, H, W]
    (float32), the acceptance mask and the GPU time of each part.

    With band_min, lattices whose initial fields hold less than that share of their
    energy in the network's kept modes (band_fractions) skip the network and go
    straight to QLA: the Fourier layers cannot carry such fields, so their predictions
    would almost all fail the energy check after costing a forward pass."""
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    N = inputs.shape[0]
    gated_out = 0
    if band_min is None:
        out, energy = predict_all(sur, inputs, batch)
        ok = accept(energy, e0, tol)
    else:
        frac = band_fractions(sur, inputs, batch)
        sel = torch.nonzero(frac >= band_min).flatten()
        gated_out = N - int(sel.numel())
        if gated_out == 0:          # every input passes: predict in place
            out, energy = predict_all(sur, inputs, batch)
            ok = accept(energy, e0, tol)
        else:                       # predict the passing inputs, gathered once
            out = torch.zeros((N, 3, sur.H, sur.W), dtype=torch.float32, device=inputs.device)
            ok = torch.zeros(N, dtype=torch.bool, device=inputs.device)
            if sel.numel():
                sub_out, sub_e = predict_all(sur, inputs.index_select(0, sel), batch)
                out.index_copy_(0, sel, sub_out)
                ok.index_copy_(0, sel, accept(sub_e, e0.index_select(0, sel), tol))
                del sub_out
    t1.record(stream)
    t1.synchronize()
    fno_s = t0.elapsed_time(t1) / 1e3
    rejected = torch.nonzero(~ok).flatten().cpu().numpy()
    qla_s = 0.0
    if rejected.size:
        def sub_index(first, k):
            return torch.stack([index_fn(int(i), 1)[0] for i in rejected[first:first + k]])
        sub = qla_pairs(sub_index, int(rejected.size), [packets[i] for i in rejected], delta,
                        steps, sur.n_shift, chunk, keep_f32=True)
        out[torch.as_tensor(rejected, device=out.device)] = sub.targets_f32
        qla_s = sub.qla_seconds
    return out, ok, {"surrogate_s": fno_s, "fallback_qla_s": qla_s,
                     "rejected": int(rejected.size), "gated_out": gated_out}
