"""Fourier symbol of one QLA step in a homogeneous medium (test infrastructure only).

For a single lattice mode q(x, y) = v exp(i (kx x + ky y)) (x, y in cells) every
operator of Eqs. (2e6) and (2e9) acts as a 6x6 matrix on v: a collision is its
constant matrix, and a streaming operator that takes a component's value from
x +- 1 multiplies that component by exp(+- i kx) (likewise in y). With n uniform,
all potential angles vanish (beta ~ dn/dx = 0, Eq. 2e13) and one step of
Eq. (2e14) is the product M(k) = U_y(ky) U_x(kx) (Eq. 2e10).

This is an independent route to the oracle's result: the oracle's real-space
passes must reproduce M(k)^s exactly for a single mode, and M(k) must approach
exp(dt G(K)), G being the Fourier symbol of Eqs. (2d1)-(2d6) with dt = delta^2
and K = k / delta the physical wavenumber (Section IV).
"""
from __future__ import annotations

import numpy as np


def _rot_block(M, i, j, c, s):
    """Set the (i, j) plane of M to [[c, -s], [s, c]] (rows i, j)."""
    M[i, i], M[i, j] = c, -s
    M[j, i], M[j, j] = s, c


def collision_x(theta: float) -> np.ndarray:
    """Eq. (2e3), isotropic: (q1, q5) and (q2, q4) rotated by +theta."""
    c, s = np.cos(theta), np.sin(theta)
    M = np.eye(6, dtype=complex)
    _rot_block(M, 1, 5, c, s)
    _rot_block(M, 2, 4, c, s)
    return M


def collision_y(theta: float) -> np.ndarray:
    """Eq. (2e8), isotropic: (q0, q5) and (q2, q3) rotated by -theta."""
    c, s = np.cos(theta), np.sin(theta)
    M = np.eye(6, dtype=complex)
    _rot_block(M, 0, 5, c, -s)
    _rot_block(M, 2, 3, c, -s)
    return M


def shift(comps, k: float, sign: int) -> np.ndarray:
    """Streaming that takes the listed components from the +-1 neighbour: exp(+-ik)."""
    d = np.ones(6, dtype=complex)
    for c in comps:
        d[c] = np.exp(1j * sign * k)
    return np.diag(d)


def u_x(kx: float, theta: float) -> np.ndarray:
    """Symbol of U_x, Eq. (2e6), multiplied out left to right as printed."""
    C = collision_x(theta)
    Cd = C.conj().T
    S14p, S14m = shift((1, 4), kx, +1), shift((1, 4), kx, -1)
    S25p, S25m = shift((2, 5), kx, +1), shift((2, 5), kx, -1)
    factors = [S25p, Cd, S25m, C, S14m, Cd, S14p, C,
               S25m, C, S25p, Cd, S14p, C, S14m, Cd]
    out = np.eye(6, dtype=complex)
    for F in factors:
        out = out @ F
    return out


def u_y(ky: float, theta: float) -> np.ndarray:
    """Symbol of U_y, Eq. (2e9), multiplied out left to right as printed."""
    C = collision_y(theta)
    Cd = C.conj().T
    S03p, S03m = shift((0, 3), ky, +1), shift((0, 3), ky, -1)
    S25p, S25m = shift((2, 5), ky, +1), shift((2, 5), ky, -1)
    factors = [S25p, Cd, S25m, C, S03m, Cd, S03p, C,
               S25m, C, S25p, Cd, S03p, C, S03m, Cd]
    out = np.eye(6, dtype=complex)
    for F in factors:
        out = out @ F
    return out


def step(kx: float, ky: float, n: float, delta: float) -> np.ndarray:
    """One homogeneous step, Eq. (2e10), collision angle delta / (4 n) (Eq. 2e4)."""
    theta = delta / (4.0 * n)
    return u_y(ky, theta) @ u_x(kx, theta)


def maxwell_generator(Kx: float, Ky: float, n: float) -> np.ndarray:
    """Fourier symbol G of Eqs. (2d1)-(2d6) for uniform n (gradient terms vanish):
    d/dt v = G v for v exp(i (Kx x + Ky y)), x and y physical, c = 1."""
    G = np.zeros((6, 6), dtype=complex)
    ix, iy = 1j * Kx / n, 1j * Ky / n
    G[0, 5] = iy            # (2d1)
    G[1, 5] = -ix           # (2d2)
    G[2, 3] = -iy           # (2d3)
    G[2, 4] = ix
    G[3, 2] = -iy           # (2d4)
    G[4, 2] = ix            # (2d5)
    G[5, 0] = iy            # (2d6)
    G[5, 1] = -ix
    return G
