"""Pins of the CPU oracle to what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: the printed
LCU matrices (Eqs. 2f1-2f7), the Fourier algebra of the printed operator
products (Eqs. 2e6, 2e9, 2e10), the continuum Maxwell equations (Eqs. 2d1-2d6),
unitarity, closed-form translation in vacuum, a spectral solution of the PDE,
and the textbook normal-incidence Fresnel reflectance.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import spectral, symbol

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lcu_matrices.txt")


# --------------------------------------------------------------------------------------
# helpers
def _load_golden():
    mats, name = {}, None
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                name = line[1:-1]
                mats[name] = []
            else:
                mats[name].append(line.split())
    return mats


def _eval(mat, beta):
    out = np.zeros((6, 6))
    for r, row in enumerate(mat):
        for c, tok in enumerate(row):
            sign = -1.0 if tok.startswith("-") else 1.0
            t = tok.lstrip("-")
            if t in ("0", "1"):
                v = float(t)
            else:
                k = int(t[1])
                v = math.cos(beta[k]) if t[0] == "c" else math.sin(beta[k])
            out[r, c] = sign * v
    return out


def _site_matrices(op, n, delta, vmode):
    """Dense 6x6 matrix of a site-local operator at every site, column by column."""
    ny, nx = n.shape
    cols = []
    for c in range(6):
        q = np.zeros((6, ny, nx))
        q[c] = 1.0
        oracle.apply(op, q, n, delta, vmode)
        cols.append(q)
    # M[y, x, r, c]
    return np.stack(cols, axis=-1).transpose(1, 2, 0, 3)


def _smooth_random_index(nx, ny, seed, lo=1.0, hi=3.0):
    rng = np.random.default_rng(seed)
    x = np.arange(nx)[None, :] * 2 * np.pi / nx
    y = np.arange(ny)[:, None] * 2 * np.pi / ny
    f = np.zeros((ny, nx))
    for _ in range(4):
        a, b = rng.integers(0, 3, size=2)
        f += rng.normal() * np.cos(a * x + b * y + rng.uniform(0, 2 * np.pi))
    f = (f - f.min()) / (np.ptp(f) + 1e-300)
    return lo + (hi - lo) * f


# --------------------------------------------------------------------------------------
# potentials against the printed linear combination of unitaries
def test_lcu_sum_pins_vx_including_row_q5():
    g = _load_golden()
    rng = np.random.default_rng(1)
    n = rng.uniform(1.0, 3.0, size=(4, 5))
    delta = 0.7
    _, bx, by = oracle.coefficients(n, delta)
    M = _site_matrices(oracle.OP_VX, n, delta, oracle.V_PAPER)
    for y in range(4):
        for x in range(5):
            beta = [bx[y, x], by[y, x], bx[y, x], by[y, x]]  # isotropic: b0=b2, b1=b3
            lcu = 0.5 * sum(_eval(g[k], beta) for k in ("L_x1", "L_x2", "L_x3", "L_x4"))
            np.testing.assert_allclose(M[y, x], lcu, atol=1e-15)
            printed = _eval(g["V_x"], beta)
            # the printed V_x agrees with its own LCU everywhere except the q5 <- q1 entry
            diff = np.argwhere(np.abs(printed - lcu) > 1e-15)
            if abs(bx[y, x]) > 1e-12:
                assert [tuple(d) for d in diff] == [(5, 1)]


def test_lcu_sum_pins_vy_outside_row_q3():
    g = _load_golden()
    rng = np.random.default_rng(2)
    n = rng.uniform(1.0, 3.0, size=(5, 4))
    delta = 0.7
    _, bx, by = oracle.coefficients(n, delta)
    M = _site_matrices(oracle.OP_VY, n, delta, oracle.V_PAPER)
    for y in range(5):
        for x in range(4):
            beta = [bx[y, x], by[y, x], bx[y, x], by[y, x]]
            lcu = 0.5 * sum(_eval(g[k], beta) for k in ("L_y1", "L_y2", "L_y3", "L_y4"))
            # the LCU reproduces the printed V_y exactly (including its row q3) ...
            np.testing.assert_allclose(lcu, _eval(g["V_y"], beta), atol=1e-15)
            keep = [0, 1, 2, 4, 5]
            np.testing.assert_allclose(M[y, x][keep], lcu[keep], atol=1e-15)
            # ... whose row q3 is not the identity at beta = 0, contradicting Eq. (2e10);
            # the oracle's row q3 has cos/sin exchanged.
            np.testing.assert_allclose(M[y, x][3], [0, 0, math.sin(beta[3]), math.cos(beta[3]), 0, 0],
                                       atol=1e-15)


def test_vy_row_q3_reading_is_the_homogeneous_limit_and_eq_2d4_sign():
    # beta = 0 (uniform n): every potential must be the identity (Eq. 2e10 is the
    # homogeneous scheme); to first order Eq. (2d4) needs q3 += +beta3 q2.
    n = np.full((4, 4), 1.6)
    M = _site_matrices(oracle.OP_VY, n, 0.5, oracle.V_PAPER)
    np.testing.assert_array_equal(M[0, 0], np.eye(6))
    n = 1.5 + 0.01 * np.arange(8)[:, None] * np.ones((1, 4))
    delta = 0.1
    _, _, by = oracle.coefficients(n, delta)
    M = _site_matrices(oracle.OP_VY, n, delta, oracle.V_PAPER)
    y = 3
    assert by[y, 0] > 0
    assert abs(M[y, 0][3, 2] - by[y, 0]) < by[y, 0] ** 3


def test_beta_is_delta_squared_gradient_over_n_squared():
    # Eq. (2e13) with a centred difference: second-order accurate in the cell size.
    nx, delta = 64, 0.3
    x = np.arange(nx)
    k = 2 * np.pi / nx
    n = np.broadcast_to(2.0 + 0.5 * np.sin(k * x)[None, :], (3, nx)).copy()
    th, bx, by = oracle.coefficients(n, delta)
    dndx_phys = 0.5 * k * np.cos(k * x) / delta          # d n / d(physical x)
    exact = delta ** 2 * dndx_phys / n[0] ** 2
    err = np.abs(bx[0] - exact).max() / np.abs(exact).max()
    assert err < k * k / 6 * 1.01 and err > k * k / 6 * 0.5   # sin(k)/k - 1 ~ -k^2/6
    np.testing.assert_array_equal(by, 0.0)
    np.testing.assert_allclose(th, delta / (4 * n), rtol=0, atol=0)


# --------------------------------------------------------------------------------------
# unitarity
def test_collisions_and_streams_are_orthogonal():
    rng = np.random.default_rng(3)
    n = rng.uniform(1.0, 3.0, size=(6, 7))
    q0 = rng.normal(size=(6, 6, 7))
    for fwd, back in ((oracle.OP_CX, oracle.OP_CX_DAG), (oracle.OP_CY, oracle.OP_CY_DAG),
                      (oracle.OP_S14_PX, oracle.OP_S14_MX), (oracle.OP_S25_PX, oracle.OP_S25_MX),
                      (oracle.OP_S03_PY, oracle.OP_S03_MY), (oracle.OP_S25_PY, oracle.OP_S25_MY)):
        q = q0.copy()
        oracle.apply(fwd, q, n, 0.9)
        assert abs(oracle.energy(q) / oracle.energy(q0) - 1) < 1e-14
        oracle.apply(back, q, n, 0.9)
        np.testing.assert_allclose(q, q0, atol=1e-14)


@pytest.mark.parametrize("op", ["UX", "UY"])
def test_collide_stream_preserves_norm_in_any_medium(op):
    rng = np.random.default_rng(4)
    n = rng.uniform(1.0, 3.0, size=(9, 11))       # arbitrary, even discontinuous, n
    q = rng.normal(size=(6, 9, 11))
    e0 = oracle.energy(q)
    code = oracle.OP_UX if op == "UX" else oracle.OP_UY
    for _ in range(50):
        oracle.apply(code, q, n, 0.5)
    assert abs(oracle.energy(q) / e0 - 1) < 1e-13


def test_skew_half_step_conserves_energy_paper_step_does_not():
    n = _smooth_random_index(24, 20, seed=5)
    rng = np.random.default_rng(5)
    q = rng.normal(size=(6, 20, 24))
    e0 = oracle.energy(q)
    q1 = oracle.advance(q.copy(), n, 0.5, 100, oracle.V_SKEW_HALF)
    assert abs(oracle.energy(q1) / e0 - 1) < 1e-13
    q2 = oracle.advance(q.copy(), n, 0.5, 100, oracle.V_PAPER)
    assert abs(oracle.energy(q2) / e0 - 1) > 1e-6     # the printed potentials are not unitary


# --------------------------------------------------------------------------------------
# Fourier algebra and the continuum limit
@pytest.mark.parametrize("which", ["UX", "UY", "STEP"])
def test_oracle_reproduces_the_fourier_symbol_exactly(which):
    nx, ny, nval, delta = 16, 12, 1.7, 0.3
    kx, ky = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    theta = delta / (4 * nval)
    if which == "UX":
        M, code, steps = symbol.u_x(kx, theta), oracle.OP_UX, 1
    elif which == "UY":
        M, code, steps = symbol.u_y(ky, theta), oracle.OP_UY, 1
    else:
        M, code, steps = symbol.step(kx, ky, nval, delta), oracle.OP_STEP, 7
    rng = np.random.default_rng(6)
    v = rng.normal(size=6) + 1j * rng.normal(size=6)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    phase = np.exp(1j * (kx * X + ky * Y))
    q = np.ascontiguousarray(np.real(v[:, None, None] * phase[None]))
    n = np.full((ny, nx), nval)
    for _ in range(steps):
        oracle.apply(code, q, n, delta)
    w = np.linalg.matrix_power(M, steps) @ v
    expect = np.real(w[:, None, None] * phase[None])
    np.testing.assert_allclose(q, expect, atol=1e-13)


@pytest.mark.parametrize("K", [(3.0, 0.0), (0.0, 2.0), (2.0, 1.5)])
def test_step_recovers_maxwell_to_second_order(K):
    # U_y U_x = exp(delta^2 G + O(delta^4)) with G the symbol of Eqs. (2d1)-(2d6)
    # (Eq. 2e7, 2e10: dt = delta^2, error O(delta^2) relative to the generator).
    Kx, Ky = K
    nval = 1.7
    G = symbol.maxwell_generator(Kx, Ky, nval)
    errs = []
    for delta in (0.1, 0.05, 0.025, 0.0125):
        M = symbol.step(Kx * delta, Ky * delta, nval, delta)
        errs.append(np.abs(sla.logm(M) / delta ** 2 - G).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.9 < r < 4.1 for r in ratios), ratios
    assert errs[-1] < 1e-3 * np.abs(G).max()


# --------------------------------------------------------------------------------------
# free-space propagation (closed form: rigid translation at c = 1)
def _centroid(e_x):
    x = np.arange(e_x.size)
    return float((x * e_x).sum() / e_x.sum())


def test_vacuum_packet_moves_one_way_at_the_lattice_group_velocity():
    nx, ny, delta, steps = 512, 1, 0.25, 600
    lam, sigma, x0 = 16.0, 12.0, 100.0
    n = np.ones((ny, nx))
    q = oracle.packet(n, x0, 0.0, sigma, lam)
    assert np.array_equal(q[4], -q[2])                      # one-way pairing for +x
    e0 = oracle.energy(q)
    oracle.advance(q, n, delta, steps)
    e_x = (q ** 2).sum(axis=(0, 1))
    # group velocity (cells per step) of the carrier from the exact symbol
    k0, dk = 2 * np.pi / lam, 1e-4

    def phase(k):
        w = np.linalg.eigvals(symbol.step(k, 0.0, 1.0, delta))
        return np.sort(np.abs(np.angle(w)))[-1]
    vg = (phase(k0 + dk) - phase(k0 - dk)) / (2 * dk)
    assert 0.9 * delta < vg < delta                         # ~ delta cos(k0)
    shift = _centroid(e_x) - x0
    assert abs(shift / (steps * vg) - 1) < 5e-3
    back = e_x[: int(x0)].sum() / e_x.sum()                 # nothing moves towards -x
    assert back < 1e-6
    assert abs(e_x.sum() / e0 - 1) < 5e-12     # rounding of cos, sin only


def _gauss_packet_phys(x, x0, sigma, lam):
    return np.exp(-((x - x0) ** 2) / (2 * sigma ** 2)) * np.cos(2 * np.pi * (x - x0) / lam)


def test_vacuum_translation_error_falls_at_second_order():
    # Fixed physical problem on [0, 1): delta = 1 / N, steps = T / delta^2; the exact
    # solution is the initial packet translated by T (c = 1).
    T, x0, sigma, lam = 0.25, 0.3, 0.06, 0.15
    errs = []
    for N in (32, 64, 128, 256):
        delta = 1.0 / N
        x = np.arange(N) * delta
        n = np.ones((1, N))
        q = np.zeros((6, 1, N))
        q[2, 0] = _gauss_packet_phys(x, x0, sigma, lam)
        q[4, 0] = -q[2, 0]
        oracle.advance(q, n, delta, int(round(T / delta ** 2)))
        exact = _gauss_packet_phys(x, x0 + T, sigma, lam)
        errs.append(np.linalg.norm(q[2, 0] - exact) / np.linalg.norm(exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert ratios[-1] > 3.7 and ratios[-2] > 3.3, (errs, ratios)


# --------------------------------------------------------------------------------------
# second-order convergence to the continuum equations in an inhomogeneous medium
def _slab_phys(x, xa, xb, n_in, w):
    return 1.0 + (n_in - 1.0) * 0.5 * (np.tanh((x - xa) / w) - np.tanh((x - xb) / w))


def _run_slab(N, vmode, T):
    delta = 1.0 / N
    x = np.arange(N) * delta
    n = _slab_phys(x, 0.45, 0.85, 2.0, 0.03)[None, :].copy()
    q = np.zeros((6, 1, N))
    q[2, 0] = n[0] * _gauss_packet_phys(x, 0.25, 0.06, 0.15)
    q[4, 0] = -q[2, 0]
    oracle.advance(q, n, delta, int(round(T / delta ** 2)), vmode)
    return q


@pytest.fixture(scope="module")
def slab_reference():
    T, Nref = 0.25, 2048
    x = np.arange(Nref) / Nref
    n = _slab_phys(x, 0.45, 0.85, 2.0, 0.03)[None, :].copy()
    q = np.zeros((6, 1, Nref))
    q[2, 0] = n[0] * _gauss_packet_phys(x, 0.25, 0.06, 0.15)
    q[4, 0] = -q[2, 0]
    return T, Nref, spectral.solve(q, n, 1.0, 1.0 / Nref, T)


def _slab_errors(vmode, ref):
    T, Nref, qref = ref
    errs = []
    for N in (64, 128, 256):
        q = _run_slab(N, vmode, T)
        r = qref[:, :, :: Nref // N][2:5]
        errs.append(np.linalg.norm(q[2:5] - r) / np.linalg.norm(r))
    return errs


def test_skew_half_converges_at_second_order_through_a_dielectric_slab(slab_reference):
    errs = _slab_errors(oracle.V_SKEW_HALF, slab_reference)
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 3.6 and ratios[-2] > 2.5, (errs, ratios)
    assert errs[-1] < 0.15


def test_printed_potentials_do_not_converge(slab_reference):
    # Recorded reading: with the potentials as printed (V_PAPER) the error stalls.
    errs = _slab_errors(oracle.V_PAPER, slab_reference)
    assert errs[-1] > 0.3 and errs[-2] / errs[-1] < 2.0, errs


def test_skew_half_converges_in_2d_around_an_ellipse():
    T, Nref = 0.06, 256
    L = 1.0

    def index(N):
        c = (np.arange(N) + 0.0) / N
        X, Y = np.meshgrid(c, c)
        xp, yp = X - 0.5, Y - 0.5
        rho2 = (xp / 0.2) ** 2 + (yp / 0.12) ** 2
        return 1.0 + 0.5 * (1.0 - np.tanh((rho2 - 1.0) / 0.35))

    def init(N, n):
        c = np.arange(N) / N
        X, _ = np.meshgrid(c, c)
        q = np.zeros((6, N, N))
        q[2] = n * _gauss_packet_phys(X, 0.3, 0.05, 0.12)
        q[4] = -q[2]
        return q

    nref = index(Nref)
    qref = spectral.solve(init(Nref, nref), nref, L, L, T)
    errs = []
    for N in (32, 64, 128):
        n = index(N)
        q = init(N, n)
        oracle.advance(q, n, L / N, int(round(T * N * N)))
        r = qref[:, :: Nref // N, :: Nref // N][2:5]
        errs.append(np.linalg.norm(q[2:5] - r) / np.linalg.norm(r))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 3.3, (errs, ratios)


# --------------------------------------------------------------------------------------
# normal-incidence Fresnel reflectance (textbook special case)
def _fresnel_run(vmode, width=0.5, lam=32.0, n2=2.0):
    nx, delta = 1024, 0.5
    x = np.arange(nx, dtype=float)
    n = (1.0 + (n2 - 1.0) * 0.5 * (np.tanh((x - 512) / width) - np.tanh((x - 1000) / width)))
    n = n[None, :].copy()
    q = oracle.packet(n, 300.0, 0.0, 1.5 * lam, lam)
    e0 = oracle.energy(q)
    oracle.advance(q, n, delta, 900, vmode)
    e_x = (q ** 2).sum(axis=(0, 1))
    refl = e_x[:512].sum() / e0
    trans = e_x[512:1000].sum() / e0
    return refl, trans


def test_normal_incidence_reflectance_is_fresnel():
    r, t = _fresnel_run(oracle.V_SKEW_HALF)
    r_exact = ((2.0 - 1.0) / (2.0 + 1.0)) ** 2                 # 1/9
    assert abs(r / r_exact - 1) < 0.06, r
    assert abs(r + t - 1) < 1e-6
    # without the potentials the gradient terms of Eqs. (2d4)-(2d5) are half missing and
    # almost nothing reflects; the printed potentials create energy (R + T far above 1)
    r0, _ = _fresnel_run(oracle.V_NONE)
    assert r0 < 0.05 * r_exact
    rp, tp = _fresnel_run(oracle.V_PAPER)
    assert rp + tp > 1.5


# --------------------------------------------------------------------------------------
# the B_z triple (q0, q1, q5) and the divergence diagnostic
def test_vacuum_bz_packet_moves_one_way():
    nx, ny, delta, steps = 512, 1, 0.25, 600
    lam, sigma, x0 = 16.0, 12.0, 100.0
    n = np.ones((ny, nx))
    q = oracle.packet_bz(n, x0, 0.0, sigma, lam)
    assert np.array_equal(q[1], q[5]) and not q[2:5].any()
    e0 = oracle.energy(q)
    oracle.advance(q, n, delta, steps)
    assert not q[2:5].any()                                  # the triples never mix
    e_x = (q ** 2).sum(axis=(0, 1))
    assert _centroid(e_x) - x0 > 0.9 * steps * delta * 0.9
    assert e_x[: int(x0)].sum() / e_x.sum() < 1e-6           # nothing moves towards -x
    assert abs(e_x.sum() / e0 - 1) < 5e-12


def _bz_slab_run(N, T, axis, spectral_ref=False):
    # Bz packet in vacuum hitting a slab n = 2 along `axis` (1 = x, 0 = y)
    delta = 1.0 / N
    s = np.arange(N) * delta
    prof = _slab_phys(s, 0.45, 0.85, 2.0, 0.03)
    n = prof[None, :].copy() if axis == 1 else prof[:, None].copy()
    bz = _gauss_packet_phys(s, 0.25, 0.06, 0.15)
    q = np.zeros((6,) + n.shape)
    if axis == 1:
        q[5, 0] = bz
        q[1, 0] = bz              # n Ey = Bz: one way along +x
    else:
        q[5, :, 0] = bz
        q[0, :, 0] = -bz          # n Ex = -Bz: one way along +y
    if spectral_ref:
        ly, lx = (1.0 / N, 1.0) if axis == 1 else (1.0, 1.0 / N)
        return spectral.solve(q, n, lx, ly, T)
    oracle.advance(q, n, delta, int(round(T / delta ** 2)), oracle.V_SKEW_HALF)
    return q


@pytest.mark.parametrize("axis", [1, 0])
def test_skew_half_bz_triple_converges_at_second_order_through_a_slab(axis):
    # Eqs. (2d1), (2d2), (2d6): the B_z triple's gradient terms sit on q5; the same
    # half-angle rotations supply them (reading of the potentials).
    T, Nref = 0.25, 2048
    ref = _bz_slab_run(Nref, T, axis, spectral_ref=True)
    errs = []
    for N in (64, 128, 256):
        q = _bz_slab_run(N, T, axis)
        r = ref[:, :, :: Nref // N] if axis == 1 else ref[:, :: Nref // N, :]
        errs.append(np.linalg.norm(q[[0, 1, 5]] - r[[0, 1, 5]]) / np.linalg.norm(r[[0, 1, 5]]))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 3.6 and ratios[-2] > 2.5, (errs, ratios)
    assert errs[-1] < 0.15


def test_divergence_of_a_discrete_curl_vanishes():
    # B = (D_y psi, -D_x psi) with the same centred differences: div B = 0 exactly
    # (the two differences commute), up to rounding
    rng = np.random.default_rng(5)
    ny, nx, delta = 24, 40, 0.25
    psi = rng.normal(size=(ny, nx))
    n = rng.uniform(1.0, 3.0, size=(ny, nx))
    ddx = lambda f: (np.roll(f, -1, 1) - np.roll(f, 1, 1)) / (2 * delta)
    ddy = lambda f: (np.roll(f, -1, 0) - np.roll(f, 1, 0)) / (2 * delta)
    q = np.zeros((6, ny, nx))
    q[3], q[4] = ddy(psi), -ddx(psi)
    q[0], q[1] = ddy(psi) / n, -ddx(psi) / n          # D = n q = curl psi
    div_b, div_d = oracle.divergence(q, n, delta)
    scale = np.abs(ddx(q[3])).max()
    assert np.abs(div_b).max() < 1e-13 * scale and np.abs(div_d).max() < 1e-13 * scale


def test_divergence_of_a_single_mode():
    # centred difference of cos(k x): -sin(k delta) / delta * sin(k x), k = 2 pi m / nx
    ny, nx, delta, m = 8, 32, 0.5, 3
    x = np.arange(nx) * delta
    k = 2 * np.pi * m / (nx * delta)
    q = np.zeros((6, ny, nx))
    q[3] = np.cos(k * x)[None, :]
    q[1] = 2.0 * np.sin(2 * np.pi * np.arange(ny) / ny)[:, None]     # D_y = n q1 with n = 1
    n = np.ones((ny, nx))
    div_b, div_d = oracle.divergence(q, n, delta)
    np.testing.assert_allclose(div_b, (-np.sin(k * delta) / delta * np.sin(k * x))[None, :]
                               * np.ones((ny, 1)), atol=1e-13)
    ky = 2 * np.pi / (ny * delta)
    want = 2.0 * np.sin(ky * delta) / delta * np.cos(2 * np.pi * np.arange(ny) / ny)
    np.testing.assert_allclose(div_d, want[:, None] * np.ones((1, nx)), atol=1e-13)


# --------------------------------------------------------------------------------------
# V_BSTREAM: every collide-stream set streams the B-qubit of its pair, no potentials
# (a fully unitary scheme beyond the paper)
def test_bstream_sets_are_the_printed_sets_with_the_e_sets_replaced():
    # U_x of V_BSTREAM differs from Eq. (2e6) only where the printed sets stream q2:
    # in a medium of uniform n the two agree exactly (both are Eq. 2e10's scheme)
    rng = np.random.default_rng(3)
    n = np.full((6, 10), 1.7)
    q = rng.standard_normal((6, 6, 10))
    q[[0, 1, 5]] = 0.0
    a = oracle.apply(oracle.OP_UX, q.copy(), n, 0.3, oracle.V_NONE)
    b = oracle.apply(oracle.OP_UX, q.copy(), n, 0.3, oracle.V_BSTREAM)
    np.testing.assert_allclose(a[2:5], b[2:5], atol=1e-14)
    # with varying n they differ (the angle of the E or the B site enters the pair)
    n2 = rng.uniform(1.0, 2.5, size=(6, 10))
    a = oracle.apply(oracle.OP_UX, q.copy(), n2, 0.3, oracle.V_NONE)
    b = oracle.apply(oracle.OP_UX, q.copy(), n2, 0.3, oracle.V_BSTREAM)
    assert np.abs(a - b).max() > 1e-6


def test_bstream_converges_at_second_order_through_a_slab_without_potentials(slab_reference):
    errs = _slab_errors(oracle.V_BSTREAM, slab_reference)
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 3.6 and ratios[-2] > 2.5, (errs, ratios)
    assert errs[-1] < 0.15
    # energy: every operator is a rotation or a shift
    n, q = None, None
    T, N = 0.25, 128
    x = np.arange(N) / N
    n = _slab_phys(x, 0.45, 0.85, 2.0, 0.03)[None, :].copy()
    q = np.zeros((6, 1, N))
    q[2, 0] = n[0] * _gauss_packet_phys(x, 0.25, 0.06, 0.15)
    q[4, 0] = -q[2, 0]
    e0 = oracle.energy(q)
    oracle.advance(q, n, 1.0 / N, int(round(T * N * N)), oracle.V_BSTREAM)
    assert abs(oracle.energy(q) / e0 - 1) < 1e-11


@pytest.mark.parametrize("axis", ["x", "y"])
def test_bstream_converges_in_2d_around_an_ellipse(axis):
    T, Nref = 0.06, 256

    def index(N):
        c = np.arange(N) / N
        X, Y = np.meshgrid(c, c)
        rho2 = ((X - 0.5) / 0.2) ** 2 + ((Y - 0.5) / 0.12) ** 2
        return 1.0 + 0.5 * (1.0 - np.tanh((rho2 - 1.0) / 0.35))

    def init(N, n):
        c = np.arange(N) / N
        X, Y = np.meshgrid(c, c)
        q = np.zeros((6, N, N))
        if axis == "x":
            q[2] = n * _gauss_packet_phys(X, 0.3, 0.05, 0.12)
            q[4] = -q[2]
        else:
            q[2] = n * _gauss_packet_phys(Y, 0.3, 0.05, 0.12)
            q[3] = q[2]                      # one way along +y
        return q

    nref = index(Nref)
    qref = spectral.solve(init(Nref, nref), nref, 1.0, 1.0, T)
    errs = []
    for N in (32, 64, 128):
        n = index(N)
        q = init(N, n)
        oracle.advance(q, n, 1.0 / N, int(round(T * N * N)), oracle.V_BSTREAM)
        r = qref[:, :: Nref // N, :: Nref // N][2:5]
        errs.append(np.linalg.norm(q[2:5] - r) / np.linalg.norm(r))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 3.3, (errs, ratios)


def test_bstream_normal_incidence_reflectance_is_fresnel():
    r, t = _fresnel_run(oracle.V_BSTREAM)
    assert abs(r / (1.0 / 9.0) - 1) < 0.03, r
    assert abs(r + t - 1) < 1e-6


# --------------------------------------------------------------------------------------
# the packet's conventions (Section V initial conditions) and the physical readout
# (Eq. 3b3); each against a property the definition or Maxwell's equations fix
def test_packet_envelope_is_a_gaussian_of_standard_deviation_sigma():
    # With the carrier flattened (a wavelength far beyond the lattice) the planar packet
    # is its envelope alone. Read as a distribution over x it has mean x0 and standard
    # deviation sigma (the meaning of sigma), and at s = +-sigma it is exp(-1/2) of its
    # peak. An envelope exp(-s^2 / sigma^2) has standard deviation sigma / sqrt(2) and
    # the value exp(-1) there; a width of 2 sigma fails the other way.
    nx, x0, sigma, amp = 512, 200.0, 12.0, 1.5
    n = np.ones((1, nx))
    ez = oracle.packet(n, x0, 0.0, sigma, 1e12, amp=amp)[2, 0]
    x = np.arange(nx, dtype=np.float64)
    w = ez / ez.sum()
    mean = float((w * x).sum())
    sd = math.sqrt(float((w * (x - mean) ** 2).sum()))
    assert abs(mean - x0) < 1e-9
    assert abs(sd / sigma - 1) < 1e-9
    assert abs(ez[int(x0)] - amp) < 1e-12
    for s in (-sigma, sigma):
        assert abs(ez[int(x0 + s)] / amp - math.exp(-0.5)) < 1e-12


def test_packet_carrier_has_period_lambda():
    # With the envelope flattened the carrier is cos(2 pi s / lambda): +1 at s = 0 and
    # every whole wavelength, -1 half way, zero a quarter of the way (a period of 2 lambda
    # or of 2 pi lambda fails). The DFT of the field peaks at nx / lambda cycles.
    nx, x0, lam = 512, 256.0, 16.0
    n = np.ones((1, nx))
    ez = oracle.packet(n, x0, 0.0, 1e9, lam)[2, 0]
    for m in range(-4, 5):
        assert abs(ez[int(x0 + m * lam)] - 1.0) < 1e-12
        assert abs(ez[int(x0 + m * lam + lam / 2)] + 1.0) < 1e-12
        assert abs(ez[int(x0 + m * lam + lam / 4)]) < 1e-12
    spec = np.abs(np.fft.rfft(ez))
    assert int(np.argmax(spec)) == int(nx / lam)


def test_packet_travelling_along_y_is_ez_with_bx_only():
    # The paper's incident packet travels along y with E_z and the corresponding B_x
    # (Section V initial conditions). For a wave along +y in a uniform medium Maxwell's
    # equations give B = n k x E = n Ez x-hat (c = 1): Bx = +n Ez, By = 0. The planar
    # envelope depends on y alone.
    nx, ny, n_val = 16, 256, 2.0
    n = np.full((ny, nx), n_val)
    q = oracle.packet(n, 5.0, 120.0, 10.0, 32.0, phi=math.pi / 2)
    ez, bx, by = oracle.physical_fields(q, n)
    assert np.allclose(ez, ez[:, :1], rtol=0, atol=1e-15)       # uniform along x
    assert abs(float(np.abs(ez).max()) - 1.0) < 1e-12
    assert np.allclose(bx, n_val * ez, rtol=1e-14, atol=1e-15)
    assert np.abs(by).max() < 1e-15


def test_oblique_planar_packet_is_uniform_across_its_direction():
    # phi = pi/4: the planar packet depends on s = (dx + dy)/sqrt(2) only, so it is
    # unchanged by the lattice translation (-1, +1) along its wavefronts (away from the
    # minimum-image seams), and its magnetic field is n k x E.
    nx = ny = 128
    n = np.full((ny, nx), 1.5)
    phi = math.pi / 4
    q = oracle.packet(n, 64.0, 64.0, 8.0, 12.0, phi=phi)
    ez, bx, by = oracle.physical_fields(q, n)
    core = ez[40:88, 40:88]
    shifted = ez[41:89, 39:87]
    assert np.allclose(core, shifted, rtol=0, atol=1e-14)
    assert np.allclose(bx, 1.5 * math.sin(phi) * ez, rtol=1e-14, atol=1e-15)
    assert np.allclose(by, -1.5 * math.cos(phi) * ez, rtol=1e-14, atol=1e-15)


def test_physical_readout_carries_the_energy_density_of_eq_a13():
    # Eq. (A13): the energy density is n^2 Ez^2 + Bx^2 + By^2 (E_z triple) and
    # n^2 (Ex^2 + Ey^2) + Bz^2 (B_z triple), and it equals |Q|^2 site by site. A readout
    # Ez = n q2 (or q2 alone) breaks it wherever n != 1.
    rng = np.random.default_rng(5)
    ny, nx = 48, 64
    n = 1.0 + 2.0 * rng.random((ny, nx))
    q = rng.normal(size=(6, ny, nx))
    ez, bx, by = oracle.physical_fields(q, n)
    dens = n ** 2 * ez ** 2 + bx ** 2 + by ** 2
    assert np.allclose(dens, q[2] ** 2 + q[3] ** 2 + q[4] ** 2, rtol=1e-13, atol=0)
    ex, ey, bz = oracle.physical_fields_bz(q, n)
    dens = n ** 2 * (ex ** 2 + ey ** 2) + bz ** 2
    assert np.allclose(dens, q[0] ** 2 + q[1] ** 2 + q[5] ** 2, rtol=1e-13, atol=0)


@pytest.mark.parametrize("triple", ["ez", "bz"])
def test_physical_readout_of_a_travelling_wave_has_maxwells_impedance(triple):
    # A wave travelling along +x in a uniform medium of index n has B = n k x E and
    # E = -(1/n) k x B (c = 1): By = -n Ez for the E_z polarisation, Ey = Bz / n for the
    # B_z one. After the oracle has carried a packet 50 cells through n = 2 the physical
    # fields keep these ratios to the scheme's accuracy; a readout that multiplied by n
    # instead of dividing would be off by a factor n^2 = 4, a sign slip by -1.
    nx, n_val, delta, steps = 512, 2.0, 0.25, 400
    n = np.full((1, nx), n_val)
    if triple == "ez":
        q = oracle.packet(n, 150.0, 0.0, 24.0, 32.0)
    else:
        q = oracle.packet_bz(n, 150.0, 0.0, 24.0, 32.0)
    oracle.advance(q, n, delta, steps)
    if triple == "ez":
        e, _, b = oracle.physical_fields(q, n)
        ratio = -float((b * e).sum() / (e * e).sum())           # By = -ratio Ez
    else:
        _, e, b = oracle.physical_fields_bz(q, n)
        ratio = float((b * b).sum() / (e * b).sum())            # Ey = Bz / ratio
    assert abs(ratio / n_val - 1) < 1e-2, ratio
    # and the packet did move: its energy centroid advanced by about steps delta / n
    dens = (q ** 2).sum(axis=(0, 1))
    shift = _centroid(dens) - 150.0
    assert abs(shift / (steps * delta / n_val) - 1) < 0.1, shift
