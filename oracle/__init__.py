"""CPU oracle for the QLA time step (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg import
this package. It shares no code with the GPU library. The heavy lifting is the
plain FP64 C implementation in `qla_oracle.c` (one full-lattice pass per
operator of Eq. 2e14, OpenMP over rows); this module loads it with ctypes and
adds numpy front ends. `symbol.py` (Fourier symbol of one homogeneous step) and
`spectral.py` (spectral solution of Eqs. 2d1-2d6) are independent references
used only to pin the oracle.

Layout: a state is a float64 array q[6, ny, nx] holding (q0..q5) of Eq. (3b3),
x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "qla_oracle.c")

V_SKEW_HALF, V_PAPER, V_NONE, V_BSTREAM = 0, 1, 2, 3

# Operator codes, in the order of the C enum.
(OP_CX, OP_CX_DAG, OP_CY, OP_CY_DAG,
 OP_S14_PX, OP_S14_MX, OP_S25_PX, OP_S25_MX,
 OP_S03_PY, OP_S03_MY, OP_S25_PY, OP_S25_MY,
 OP_VX, OP_VY, OP_UX, OP_UY, OP_STEP) = range(17)

_SAN_LIB_PATH = os.path.join(_HERE, "liboracle_san.so")
# With QLA_ORACLE_SANITIZE=1 in the environment the oracle loads a build instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer (the process must preload libasan first;
# see sanitizer_env()).
SANITIZE_ENV = "QLA_ORACLE_SANITIZE"

_lib = None


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the C oracle with gcc into liboracle.so next to its source.

    sanitize=True builds liboracle_san.so instead: the same source under
    -fsanitize=address,undefined, halting on the first undefined-behaviour report."""
    path = _SAN_LIB_PATH if sanitize else _LIB_PATH
    if force or not os.path.exists(path) or \
            os.path.getmtime(path) < os.path.getmtime(_SRC_PATH):
        tmp = path + ".tmp"
        flags = ["-O2", "-fopenmp", "-fPIC", "-shared", "-Wall"]
        if sanitize:
            flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fPIC", "-shared",
                     "-Wall", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
        subprocess.run(["gcc", *flags, "-o", tmp, _SRC_PATH, "-lm"], check=True)
        os.replace(tmp, path)
    return path


def sanitizer_env(base=None) -> dict:
    """Environment for a child process that loads the sanitized oracle: libasan preloaded
    (it must come before any other library), leak checks off (the interpreter's own
    allocations are not the oracle's), UBSan halting with a stack trace."""
    env = dict(os.environ if base is None else base)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=97"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=98"
    env[SANITIZE_ENV] = "1"
    return env


def _load():
    global _lib
    if _lib is None:
        sanitize = os.environ.get(SANITIZE_ENV) == "1"
        lib = ctypes.CDLL(build(sanitize=sanitize))
        dp = ctypes.POINTER(ctypes.c_double)
        lib.qla_oracle_coefficients.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                dp, dp, dp, dp]
        lib.qla_oracle_coefficients.restype = ctypes.c_int
        lib.qla_oracle_apply.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_int, dp, dp]
        lib.qla_oracle_apply.restype = ctypes.c_int
        lib.qla_oracle_advance.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, dp, dp, ctypes.c_longlong]
        lib.qla_oracle_advance.restype = ctypes.c_int
        lib.qla_oracle_energy.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        lib.qla_oracle_energy.restype = ctypes.c_double
        lib.qla_oracle_packet.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        lib.qla_oracle_packet.restype = ctypes.c_int
        lib.qla_oracle_threads.argtypes = []
        lib.qla_oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _index(n: np.ndarray) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.float64)
    if n.ndim != 2:
        raise ValueError("n must be a 2D [ny, nx] array")
    return n


def _state(q: np.ndarray, ny: int, nx: int) -> np.ndarray:
    if q.shape != (6, ny, nx) or q.dtype != np.float64 or not q.flags.c_contiguous:
        raise ValueError("state must be a C-contiguous float64 array of shape (6, ny, nx)")
    return q


def threads() -> int:
    return int(_load().qla_oracle_threads())


def coefficients(n: np.ndarray, delta: float):
    """(theta, beta_x, beta_y) per site: Eq. (2e4) and Eq. (2e13) with centred differences."""
    n = _index(n)
    ny, nx = n.shape
    th, bx, by = (np.empty_like(n) for _ in range(3))
    rc = _load().qla_oracle_coefficients(nx, ny, float(delta), _ptr(n), _ptr(th), _ptr(bx),
                                         _ptr(by))
    if rc:
        raise ValueError(f"qla_oracle_coefficients failed ({rc})")
    return th, bx, by


def packet(n: np.ndarray, x0: float, y0: float, sigma: float, lam: float, phi: float = 0.0,
           amp: float = 1.0, planar: bool = True) -> np.ndarray:
    """Initial state q[6, ny, nx] of a one-way E_z packet (Section V initial conditions)."""
    n = _index(n)
    ny, nx = n.shape
    q = np.zeros((6, ny, nx), dtype=np.float64)
    rc = _load().qla_oracle_packet(nx, ny, _ptr(n), float(x0), float(y0), float(sigma),
                                   float(lam), float(phi), float(amp), int(bool(planar)), _ptr(q))
    if rc:
        raise ValueError(f"qla_oracle_packet failed ({rc})")
    return q


def packet_from(n: np.ndarray, p) -> np.ndarray:
    """`packet` for a workloads.Packet description."""
    return packet(n, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)


def apply(op: int, q: np.ndarray, n: np.ndarray, delta: float, vmode: int = V_SKEW_HALF):
    """Apply one operator (OP_* code) to q in place and return q."""
    n = _index(n)
    ny, nx = n.shape
    _state(q, ny, nx)
    rc = _load().qla_oracle_apply(int(op), nx, ny, float(delta), int(vmode), _ptr(n), _ptr(q))
    if rc:
        raise ValueError(f"qla_oracle_apply failed ({rc})")
    return q


def advance(q: np.ndarray, n: np.ndarray, delta: float, steps: int,
            vmode: int = V_SKEW_HALF) -> np.ndarray:
    """Advance q in place by `steps` steps of Eq. (2e14) and return it."""
    n = _index(n)
    ny, nx = n.shape
    _state(q, ny, nx)
    rc = _load().qla_oracle_advance(nx, ny, float(delta), int(vmode), _ptr(n), _ptr(q),
                                    int(steps))
    if rc:
        raise ValueError(f"qla_oracle_advance failed ({rc})")
    return q


def energy(q: np.ndarray) -> float:
    """Eq. (A13): sum of q_c^2 over components and sites (no cell-area factor)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    if q.ndim != 3 or q.shape[0] != 6:
        raise ValueError("state must have shape (6, ny, nx)")
    return float(_load().qla_oracle_energy(q.shape[2], q.shape[1], _ptr(q)))


def physical_fields(q: np.ndarray, n: np.ndarray):
    """(Ez, Bx, By) from the E_z triple: Ez = q2 / n, Bx = q3, By = q4 (Eq. 3b3, c = 1)."""
    return q[2] / n, q[3].copy(), q[4].copy()


def physical_fields_bz(q: np.ndarray, n: np.ndarray):
    """(Ex, Ey, Bz) from the B_z triple: Ex = q0 / n, Ey = q1 / n, Bz = q5 (Eq. 3b3, c = 1)."""
    return q[0] / n, q[1] / n, q[5].copy()


def packet_bz(n: np.ndarray, x0: float, y0: float, sigma: float, lam: float, phi: float = 0.0,
              amp: float = 1.0, planar: bool = True) -> np.ndarray:
    """Initial state q[6, ny, nx] of a one-way B_z packet (the other polarisation).

    Bz0 = amp exp(-r^2 / (2 sigma^2)) cos(2 pi s / lam), s the minimum-image displacement
    along phi (r = s if planar, else the full distance), as for the E_z packet. A plane
    wave travelling along k = (cos phi, sin phi) in a uniform medium has E = -(1/n) k x B,
    so n E = (-sin phi, cos phi) Bz: q0 = -sin(phi) q5, q1 = cos(phi) q5, q5 = Bz0.
    """
    n = _index(n)
    ny, nx = n.shape
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    dx = x - x0
    dy = y - y0
    dx -= nx * np.floor(dx / nx + 0.5)
    dy -= ny * np.floor(dy / ny + 0.5)
    s = dx * np.cos(phi) + dy * np.sin(phi)
    r2 = s * s if planar else dx * dx + dy * dy
    bz = amp * np.exp(-r2 / (2.0 * sigma * sigma)) * np.cos(2.0 * np.pi * s / lam)
    q = np.zeros((6, ny, nx), dtype=np.float64)
    q[5] = bz
    q[0] = -np.sin(phi) * bz
    q[1] = np.cos(phi) * bz
    return q


def divergence(q: np.ndarray, n: np.ndarray, delta: float):
    """Discrete divergences of the in-plane fields, centred differences, periodic.

    div_B = d(Bx)/dx + d(By)/dy with (Bx, By) = (q3, q4) (the E_z triple), and
    div_D = d(Dx)/dx + d(Dy)/dy with D = n^2 E = (n q0, n q1) (the B_z triple), where
    d f/dx at x is (f[x + 1] - f[x - 1]) / (2 delta). Returns (div_B, div_D), each [ny, nx].
    """
    n = _index(n)

    def ddx(f):
        return (np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1)) / (2.0 * delta)

    def ddy(f):
        return (np.roll(f, -1, axis=0) - np.roll(f, 1, axis=0)) / (2.0 * delta)

    div_b = ddx(q[3]) + ddy(q[4])
    div_d = ddx(n * q[0]) + ddy(n * q[1])
    return div_b, div_d
