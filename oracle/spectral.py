"""Spectral solution of the 2D Maxwell equations in Dyson variables (test only).

Integrates Eqs. (2d1)-(2d6) for an isotropic n(x, y) on a periodic box with
Fourier-spectral derivatives and classical fourth-order Runge-Kutta in time.
It is the continuum target that the lattice algorithm must approach to second
order in the lattice spacing (Section IV, Eq. 2e14), and it is independent of
the lattice algorithm: it never forms a collision, a stream or a potential.
"""
from __future__ import annotations

import numpy as np


def _derivatives(nx: int, ny: int, lx: float, ly: float):
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=lx / nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=ly / ny)
    if nx % 2 == 0:
        kx[nx // 2] = 0.0
    if ny % 2 == 0:
        ky[ny // 2] = 0.0
    ikx = 1j * kx[None, :]
    iky = 1j * ky[:, None]

    def dx(f):
        return np.real(np.fft.ifft2(ikx * np.fft.fft2(f)))

    def dy(f):
        return np.real(np.fft.ifft2(iky * np.fft.fft2(f)))

    return dx, dy


def rhs_factory(n: np.ndarray, lx: float, ly: float):
    """d/dt q for q[6, ny, nx] sampled on the uniform periodic grid of n."""
    ny, nx = n.shape
    dx, dy = _derivatives(nx, ny, lx, ly)
    inv_n = 1.0 / n
    nx_n2 = dx(n) / (n * n)   # (dn/dx) / n^2
    ny_n2 = dy(n) / (n * n)   # (dn/dy) / n^2

    def rhs(q):
        q0, q1, q2, q3, q4, q5 = q
        out = np.empty_like(q)
        out[0] = inv_n * dy(q5)                                          # (2d1)
        out[1] = -inv_n * dx(q5)                                         # (2d2)
        out[2] = -inv_n * dy(q3) + inv_n * dx(q4)                        # (2d3)
        out[3] = -inv_n * dy(q2) + q2 * ny_n2                            # (2d4)
        out[4] = inv_n * dx(q2) - q2 * nx_n2                             # (2d5)
        out[5] = inv_n * dy(q0) - inv_n * dx(q1) - q0 * ny_n2 + q1 * nx_n2   # (2d6)
        return out

    return rhs


def solve(q0: np.ndarray, n: np.ndarray, lx: float, ly: float, t_end: float,
          cfl: float = 0.25) -> np.ndarray:
    """Integrate from q0 to time t_end with RK4; dt <= cfl * min grid spacing * min(n)."""
    ny, nx = n.shape
    h = min(lx / nx, ly / ny)
    nsteps = max(1, int(np.ceil(t_end / (cfl * h * float(np.min(n))))))
    dt = t_end / nsteps
    rhs = rhs_factory(n, lx, ly)
    q = np.array(q0, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        k1 = rhs(q)
        k2 = rhs(q + 0.5 * dt * k1)
        k3 = rhs(q + 0.5 * dt * k2)
        k4 = rhs(q + dt * k3)
        q = q + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return q
