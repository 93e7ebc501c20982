"""Seeded synthetic inputs for the QLA time step: refractive-index maps n(x, y),
wave-packet parameters and the named workload configurations.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
none of the lattice algorithm's arithmetic: it only describes *what* is
simulated (the dielectric geometry and the packet placement), never how a step
is taken. The packet *fields* are computed separately by each side from the
parameters defined here.

Geometry follows the paper's scattering set-up (Section V, "QLA 2D Initial
Conditions"): an elliptical dielectric in vacuum, or the reverse "bubble", with
a thin continuous boundary layer in which n rises smoothly from one value to the
other. The layer profile is a tanh of a first-order signed distance to the
ellipse, so its thickness is about `width` cells all the way round.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

__all__ = [
    "Ellipse", "Packet", "Workload", "ellipse_index", "slab_index",
    "parity_small", "plain_4096", "bubble_8192", "paper_16384", "workload_by_name",
    "sample_instances", "Instance", "ellipse_index_batch",
]


@dataclasses.dataclass(frozen=True)
class Ellipse:
    """Ellipse in cell units. `a` lies along the rotated x' axis; `rot` in radians."""
    xc: float
    yc: float
    a: float
    b: float
    rot: float
    n_in: float
    n_out: float
    width: float


@dataclasses.dataclass(frozen=True)
class Packet:
    """Gaussian-envelope plane-wave packet in E_z.

    Ez0(s) = amp * exp(-s^2 / (2 sigma^2)) * cos(2 pi s / lam), with s the
    (minimum-image) distance from the packet centre along the propagation
    direction `phi` (radians, 0 = +x). With `planar` the packet is uniform across
    the direction of travel (the paper's 1D packet); otherwise the envelope is a
    2D Gaussian about (x0, y0).
    """
    x0: float
    y0: float
    sigma: float
    lam: float
    phi: float = 0.0
    amp: float = 1.0
    planar: bool = True


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    delta: float
    ellipse: Ellipse
    packet: Packet
    steps: int
    energy_every: int


def ellipse_index(nx: int, ny: int, e: Ellipse) -> np.ndarray:
    """n(x, y) on an nx-by-ny lattice, float64, row-major [y, x] (x fastest).

    n = n_out + (n_in - n_out) * (1 - tanh(d / width)) / 2, with d the first-order
    signed distance (rho^2 - 1) / (2 |grad rho^2| / 2) to the ellipse
    rho^2 = (x'/a)^2 + (y'/b)^2 = 1 in rotated coordinates about (xc, yc).
    At the exact centre the gradient vanishes and n = n_in.
    """
    x = np.arange(nx, dtype=np.float64)[None, :] - e.xc
    y = np.arange(ny, dtype=np.float64)[:, None] - e.yc
    cr, sr = math.cos(e.rot), math.sin(e.rot)
    xp = x * cr + y * sr
    yp = -x * sr + y * cr
    rho2 = (xp / e.a) ** 2 + (yp / e.b) ** 2
    g = np.sqrt((xp / (e.a * e.a)) ** 2 + (yp / (e.b * e.b)) ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        d = np.where(g > 0.0, (rho2 - 1.0) / (2.0 * g), -np.inf)
    prof = 0.5 * (1.0 - np.tanh(d / e.width))
    return np.ascontiguousarray(e.n_out + (e.n_in - e.n_out) * prof, dtype=np.float64)


def slab_index(nx: int, ny: int, x_a: float, x_b: float, n_in: float, n_out: float,
               width: float) -> np.ndarray:
    """A slab n_in for x_a < x < x_b inside n_out, uniform in y, tanh edges `width` cells."""
    x = np.arange(nx, dtype=np.float64)
    prof = 0.5 * (np.tanh((x - x_a) / width) - np.tanh((x - x_b) / width))
    row = n_out + (n_in - n_out) * prof
    return np.ascontiguousarray(np.broadcast_to(row[None, :], (ny, nx)), dtype=np.float64)


# --- the named workloads -----------------------------------------------------------------
# delta, the lattice spacing in physical units (one step advances time by delta^2), is not
# given by the paper; 0.25 is used throughout (light crosses 0.25 cells per step in vacuum).
DELTA = 0.25


def parity_small() -> Workload:
    """256^2 periodic lattice, 200 steps: centred ellipse a=40, b=20, n=2 in vacuum,
    tanh edge 3 cells; +x packet at x0=60, sigma 12, wavelength 16."""
    return Workload(
        name="qla_256_ellipse_200", nx=256, ny=256, delta=DELTA,
        ellipse=Ellipse(128.0, 128.0, 40.0, 20.0, 0.0, 2.0, 1.0, 3.0),
        packet=Packet(x0=60.0, y0=128.0, sigma=12.0, lam=16.0),
        steps=200, energy_every=100)


def plain_4096() -> Workload:
    """4096^2 lattice, 20000 steps: ellipse a=600, b=300, n=2 in vacuum, tanh edge 8;
    packet sigma 150, wavelength 64, starting 4 sigma left of the ellipse edge."""
    return Workload(
        name="qla_4096_ellipse_20000", nx=4096, ny=4096, delta=DELTA,
        ellipse=Ellipse(2048.0, 2048.0, 600.0, 300.0, 0.0, 2.0, 1.0, 8.0),
        packet=Packet(x0=2048.0 - 600.0 - 8.0 - 4 * 150.0, y0=2048.0, sigma=150.0, lam=64.0),
        steps=20000, energy_every=100)


def bubble_8192() -> Workload:
    """8192^2 lattice, 40000 steps: vacuum bubble a=1200, b=600 in uniform n=2."""
    return Workload(
        name="qla_8192_bubble_40000", nx=8192, ny=8192, delta=DELTA,
        ellipse=Ellipse(4096.0, 4096.0, 1200.0, 600.0, 0.0, 1.0, 2.0, 8.0),
        packet=Packet(x0=4096.0 - 1200.0 - 8.0 - 4 * 150.0, y0=4096.0, sigma=150.0, lam=64.0),
        steps=40000, energy_every=1000)


def paper_16384() -> Workload:
    """The paper's own 2D lattice (Section V): 16384^2, an elliptical dielectric n = 3 in
    vacuum. The paper gives the ellipse as 1600 x 716 and its boundary layer as 40 x 18
    cells; read here as full axes (semi-axes 800 and 358) with a tanh edge of 20 cells.
    Packet wavelength 100 cells as in the paper, which gives neither a width nor a start:
    sigma 150 and a start 4 sigma left of the ellipse's edge are chosen here. 20000 steps,
    energy every 1000."""
    return Workload(
        name="qla_16384_ellipse_20000", nx=16384, ny=16384, delta=DELTA,
        ellipse=Ellipse(8192.0, 8192.0, 800.0, 358.0, 0.0, 3.0, 1.0, 20.0),
        packet=Packet(x0=8192.0 - 800.0 - 20.0 - 4 * 150.0, y0=8192.0, sigma=150.0, lam=100.0),
        steps=20000, energy_every=1000)


def workload_by_name(name: str) -> Workload:
    for f in (parity_small, plain_4096, bubble_8192, paper_16384):
        w = f()
        if w.name == name:
            return w
    raise KeyError(name)


# --- batched instances ------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Instance:
    n_side: int
    ellipse: Ellipse
    packet: Packet
    steps: int
    delta: float = DELTA


def sample_instances(count: int, seed: int = 0, n_min: int = 256, n_max: int = 1024,
                     fixed_side: int | None = None, lam_min: float = 8.0,
                     lam_max: float = 32.0, steps: int | None = None) -> List[Instance]:
    """Independent scattering instances drawn with numpy's PCG64.

    Side N log-uniform in [n_min, n_max] (or `fixed_side`); semi-axes uniform in
    [0.05, 0.25] N; rotation uniform in [0, pi); n uniform in [1.5, 3]; dielectric in
    vacuum or vacuum bubble in dielectric with probability 1/2; wavelength uniform in
    [lam_min, lam_max] cells (default [8, 32]); envelope sigma = 0.75 wavelength; tanh
    edge 3 cells. The packet moves in +x and starts 3 sigma left of the ellipse's
    rotated half-width. Each instance runs 4 N steps unless `steps` is given.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        if fixed_side is None:
            side = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        else:
            side = int(fixed_side)
        a = rng.uniform(0.05, 0.25) * side
        b = rng.uniform(0.05, 0.25) * side
        rot = rng.uniform(0.0, math.pi)
        n_d = rng.uniform(1.5, 3.0)
        bubble = rng.uniform() < 0.5
        lam = rng.uniform(lam_min, lam_max)
        sigma = 0.75 * lam
        width = 3.0
        n_in, n_out = (1.0, n_d) if bubble else (n_d, 1.0)
        xc = yc = side / 2.0
        half_w = math.sqrt((a * math.cos(rot)) ** 2 + (b * math.sin(rot)) ** 2)
        x0 = (xc - half_w - width - 3.0 * sigma) % side
        out.append(Instance(
            n_side=side,
            ellipse=Ellipse(xc, yc, a, b, rot, n_in, n_out, width),
            packet=Packet(x0=x0, y0=yc, sigma=sigma, lam=lam),
            steps=4 * side if steps is None else int(steps)))
    return out


def ellipse_index_batch(nx: int, ny: int, ellipses, device=None):
    """`ellipse_index` for many ellipses at once, as a torch float64 tensor
    [len(ellipses), ny, nx] on `device` (same formula, evaluated by torch)."""
    import torch
    k = len(ellipses)
    t = lambda vals: torch.tensor(vals, dtype=torch.float64, device=device).view(k, 1, 1)
    xc, yc = t([e.xc for e in ellipses]), t([e.yc for e in ellipses])
    a, b = t([e.a for e in ellipses]), t([e.b for e in ellipses])
    cr, sr = t([math.cos(e.rot) for e in ellipses]), t([math.sin(e.rot) for e in ellipses])
    n_in, n_out = t([e.n_in for e in ellipses]), t([e.n_out for e in ellipses])
    width = t([e.width for e in ellipses])
    x = torch.arange(nx, dtype=torch.float64, device=device).view(1, 1, nx) - xc
    y = torch.arange(ny, dtype=torch.float64, device=device).view(1, ny, 1) - yc
    xp = x * cr + y * sr
    yp = -x * sr + y * cr
    rho2 = (xp / a) ** 2 + (yp / b) ** 2
    g = torch.sqrt((xp / (a * a)) ** 2 + (yp / (b * b)) ** 2)
    d = torch.where(g > 0.0, (rho2 - 1.0) / (2.0 * torch.where(g > 0.0, g, 1.0)),
                    torch.full_like(g, -math.inf))
    prof = 0.5 * (1.0 - torch.tanh(d / width))
    return (n_out + (n_in - n_out) * prof).contiguous()
