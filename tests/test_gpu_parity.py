"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: relative L2 <= 1e-12 for FP64 amplitudes and <= 1e-5 for FP32
amplitudes against the FP64 oracle; coefficients and the initial packet to a few
ulps. Full-size lattices are checked on windows whose centre the oracle computes
exactly: after s steps an amplitude depends only on inputs within 4 s cells along
each axis (U_x and U_y each reach 4 cells, the potentials 1 for n), so the oracle
run on a periodic window is exact more than 4 s + 1 cells inside its edges.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}   # by precision code: QLA_F64, QLA_F32


@pytest.fixture(scope="module")
def qla():
    from paper_2604_21128_amd import qla as q
    q.load()
    return q


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle_state(n, q3):
    q = np.zeros((6,) + n.shape)
    q[2:5] = q3
    return q


def _random_fields(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3,) + shape)


def _random_index(ny, nx, seed, lo=1.0, hi=3.0):
    rng = np.random.default_rng(seed)
    base = rng.uniform(lo, hi)
    bump = rng.uniform(-0.5, 0.5, size=(ny, nx))
    return np.clip(base + bump, lo, hi)


# ---------------------------------------------------------------------------------------
# a1 coefficients, a2 packet, a6 energy, a7 readout
def test_coefficients_match_oracle(qla):
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    with qla.Lattice(w.nx, w.ny, w.delta) as lat:
        lat.set_index(n)
        th, bx, by = lat.coefficients()
    oth, obx, oby = oracle.coefficients(n, w.delta)
    np.testing.assert_allclose(th, oth, rtol=4e-16, atol=0)
    scale = max(np.abs(obx).max(), np.abs(oby).max())
    assert np.abs(bx - obx).max() <= 1e-15 * scale
    assert np.abs(by - oby).max() <= 1e-15 * scale


@pytest.mark.parametrize("prec", [0, 1])
def test_packet_matches_oracle(qla, prec):
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    with qla.Lattice(w.nx, w.ny, w.delta, precision=prec) as lat:
        lat.set_index(n)
        for p in (w.packet, workloads.Packet(x0=30.5, y0=200.0, sigma=9.0, lam=12.0, phi=0.7,
                                               amp=0.5, planar=False)):
            lat.init_packet(p)
            got = lat.fields()
            want = oracle.packet_from(n, p)[2:5]
            # FP64: exp and cos of the device library against the host's, each within
            # about 1 ulp, and their product: a few ulps of the largest value
            tol = 2e-15 if prec == 0 else 1e-7
            assert np.abs(got - want).max() <= tol * np.abs(want).max()
            phys = lat.fields(physical=True)
            ez, bxf, byf = oracle.physical_fields(oracle.packet_from(n, p), n)
            assert np.abs(phys[0] - ez).max() <= 4 * tol * np.abs(ez).max()
            np.testing.assert_array_equal(phys[1:], got[1:])


@pytest.mark.parametrize("prec", [0, 1])
def test_energy_matches_oracle(qla, prec):
    ny, nx = 77, 131
    q = _random_fields((ny, nx), 11)
    with qla.Lattice(nx, ny, 0.25, precision=prec) as lat:
        lat.set_index(np.full((ny, nx), 1.5))
        lat.set_fields(q)
        e = lat.energy()
        stored = lat.fields()
    want = oracle.energy(_oracle_state(np.ones((ny, nx)), stored))
    assert abs(e / want - 1) < 1e-12    # summation order differs from the oracle's


# ---------------------------------------------------------------------------------------
# the full step (a3 U_x, a4 U_y, a5 V_x, V_y)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("vmode", [0, 1, 2, 3])
def test_parity_small_workload(qla, prec, vmode):
    """256^2 ellipse, +x packet, 200 steps (the small parity workload), each potential mode."""
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    q0 = oracle.packet_from(n, w.packet)
    want = oracle.advance(q0.copy(), n, w.delta, w.steps, vmode)
    with qla.Lattice(w.nx, w.ny, w.delta, precision=prec, potential=vmode) as lat:
        lat.set_index(n)
        lat.init_packet(w.packet)
        lat.advance(w.steps)
        got = lat.fields()
        assert lat.steps == w.steps
    err = rel_l2(got, want[2:5])
    print(f"prec={prec} vmode={vmode} rel_l2={err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("fused", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nx,ny,steps,rows", [
    (8, 8, 5, 0),          # smallest lattice: one wave covers the row 8 times over
    (57, 121, 7, 0),       # one column past a strip, ragged rows
    (131, 77, 9, 1),       # ragged, smallest segment
    (200, 9, 6, 16),       # short and wide
    (9, 300, 6, 40),       # tall and narrow
    (112, 240, 4, 120),    # exact multiples of the strip
])
def test_parity_ragged_random(qla, prec, nx, ny, steps, rows, fused):
    n = _random_index(ny, nx, seed=nx * 1000 + ny)
    q = _random_fields((ny, nx), seed=ny)
    for vmode in (0, 1, 3):
        want = oracle.advance(_oracle_state(n, q), n, 0.4, steps, vmode)[2:5]
        with qla.Lattice(nx, ny, 0.4, precision=prec, potential=vmode) as lat:
            qla.qla_set_tuning(lat.ctx, rows, 0, fused)
            lat.set_index(n)
            lat.set_fields(q)
            lat.advance(steps)
            got = lat.fields()
        err = rel_l2(got, want)
        print(f"{nx}x{ny} steps={steps} rows={rows} prec={prec} vmode={vmode} rel_l2={err:.3e}")
        assert err <= TOL[prec]


def test_parity_large_angles(qla):
    """delta = 1.6: collision angles up to 0.4 rad and large potential angles (the
    long-series kernel variant)."""
    ny, nx = 40, 70
    n = 1.0 + 0.5 * (1 + np.sin(2 * np.pi * np.arange(nx) / nx))[None, :] \
        * (1 + np.cos(2 * np.pi * np.arange(ny) / ny))[:, None] / 2
    q = _random_fields((ny, nx), seed=5)
    for vmode in (0, 1, 3):
        want = oracle.advance(_oracle_state(n, q), n, 1.6, 12, vmode)[2:5]
        with qla.Lattice(nx, ny, 1.6, potential=vmode) as lat:
            lat.set_index(n)
            lat.set_fields(q)
            lat.advance(12)
            got = lat.fields()
        assert rel_l2(got, want) <= 1e-12


# ---------------------------------------------------------------------------------------
# full-size lattice, sampled windows
def _window_parity(qla, w, prec, steps, centres, seed):
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    q = _random_fields((w.ny, w.nx), seed=seed)
    with qla.Lattice(w.nx, w.ny, w.delta, precision=prec) as lat:
        lat.set_index(n)
        lat.set_fields(q)
        lat.advance(steps)
        got = lat.fields()
    margin = 4 * steps + 2
    half = margin + 12
    worst = 0.0
    for cx, cy in centres:
        ys = np.arange(cy - half, cy + half + 1) % w.ny
        xs = np.arange(cx - half, cx + half + 1) % w.nx
        nw = np.ascontiguousarray(n[np.ix_(ys, xs)])
        qw = np.ascontiguousarray(q[:, ys][:, :, xs])
        out = oracle.advance(_oracle_state(nw, qw), nw, w.delta, steps)[2:5]
        inner = slice(margin, 2 * half + 1 - margin)
        want = out[:, inner, inner]
        g = got[:, ys[inner]][:, :, xs[inner]]
        err = rel_l2(g, want)
        print(f"window centre=({cx},{cy}) prec={prec} rel_l2={err:.3e}")
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("prec", [0, 1])
def test_parity_full_size_4096_windows(qla, prec):
    w = workloads.plain_4096()
    e = w.ellipse
    centres = [(int(e.xc - e.a), int(e.yc)),          # left vertex: strong x gradient
               (int(e.xc), int(e.yc + e.b)),          # top co-vertex: strong y gradient
               (int(e.xc + 0.7 * e.a), int(e.yc - 0.7 * e.b)),
               (0, 0),                                # periodic corner
               (w.nx - 1, 1234)]
    assert _window_parity(qla, w, prec, 20, centres, seed=42) <= TOL[prec]


# The benchmark's tunings (rows per segment, prefetch rows, steps per pass, columns per
# lane): the ones recorded with the step kernel's hardware counters, which bench.py runs.
PROFILES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")


def _bench_tuning(name, prec):
    with open(os.path.join(PROFILES, name)) as f:
        rec = json.load(f)
    key = "f64" if prec == 0 else "f32"
    for r in rec["records"]:
        if r["precision"] == key and r["potential"] == "skew_half":
            t = tuple(r["tuning"])
            return t if len(t) == 4 else t + (1,)
    raise KeyError((name, key))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("which", ["4096_ellipse", "8192_bubble"])
def test_parity_job_first_50_steps_at_the_bench_tuning(qla, prec, which):
    """A benchmark job as bench.py runs it: the packet initialised on the GPU, the recorded
    tuning set explicitly, 50 steps. Checked on windows across the packet and at periodic
    seams against the oracle's own packet advanced 50 steps; then random fields at the same
    tuning, on windows at the medium's strongest gradients, where the packet has not yet
    arrived."""
    w = workloads.plain_4096() if which == "4096_ellipse" else workloads.bubble_8192()
    steps = 50
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    rows, pf, ts, cols = _bench_tuning(f"qla_step_ez_{which}.json", prec)
    margin = 4 * steps + 2
    half = margin + 12

    def run(init):
        with qla.Lattice(w.nx, w.ny, w.delta, precision=prec) as lat:
            qla.qla_set_tuning(lat.ctx, rows, pf, ts)
            qla.qla_set_lane_columns(lat.ctx, cols)
            lat.set_index(n)
            init(lat)
            lat.advance(steps)
            assert tuple(qla.qla_get_tuning(lat.ctx)) == (rows, pf, ts)
            assert qla.qla_get_lane_columns(lat.ctx) == cols
            return lat.fields()

    def windows(got, q0, centres, tag):
        worst = 0.0
        for cx, cy in centres:
            ys = np.arange(cy - half, cy + half + 1) % w.ny
            xs = np.arange(cx - half, cx + half + 1) % w.nx
            nw = np.ascontiguousarray(n[np.ix_(ys, xs)])
            qw = np.ascontiguousarray(q0[:, ys][:, :, xs])
            out = oracle.advance(qw, nw, w.delta, steps)[2:5]
            inner = slice(margin, 2 * half + 1 - margin)
            err = rel_l2(got[:, ys[inner]][:, :, xs[inner]], out[:, inner, inner])
            print(f"{w.name} {tag} prec={prec} tuning={(rows, pf, ts, cols)} "
                  f"window=({cx},{cy}) rel_l2={err:.3e}", flush=True)
            worst = max(worst, err)
        return worst

    got = run(lambda lat: lat.init_packet(w.packet))
    q0 = oracle.packet_from(n, w.packet)
    x0 = int(w.packet.x0)
    band = [(x0, 100), (x0 - 150, w.ny // 2), (x0 + 170, w.ny - 96), (x0, 0),
            (x0 + 60, w.ny - 1)]
    assert windows(got, q0, band, "packet") <= TOL[prec]
    del q0
    q = _random_fields((w.ny, w.nx), seed=50 + prec)
    got = run(lambda lat: lat.set_fields(q))
    e = w.ellipse
    edges = [(int(e.xc - e.a), int(e.yc)), (int(e.xc), int(e.yc + e.b)),
             (int(e.xc + 0.7 * e.a), int(e.yc - 0.7 * e.b)), (w.nx - 1, 0)]
    assert windows(got, _oracle_state(n, q), edges, "random") <= TOL[prec]


# ---------------------------------------------------------------------------------------
# state handling
def test_checkpoint_restore_continues_bitwise(qla):
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    for prec in (0, 1):
        with qla.Lattice(w.nx, w.ny, w.delta, precision=prec) as a:
            a.set_index(n)
            a.init_packet(w.packet)
            a.advance(30)
            mid = a.fields()
            a.advance(25)
            ref = a.fields()
        with qla.Lattice(w.nx, w.ny, w.delta, precision=prec) as b:
            b.set_index(n)
            b.set_fields(mid, step=30)
            b.advance(25)
            assert b.steps == 55
            np.testing.assert_array_equal(b.fields(), ref)


def test_runs_are_deterministic_and_tiling_independent(qla):
    """Segment height, prefetch depth and steps per pass (1 or 2) change only the order
    in which sites are visited, never a site's arithmetic: results are bitwise equal."""
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    outs, energies = [], []
    for rows, pf, ts in ((0, 0, 0), (8, 2, 1), (64, 3, 2), (1, 3, 1), (100, 2, 2), (1, 2, 2),
                         (0, 0, 1)):
        with qla.Lattice(w.nx, w.ny, w.delta) as lat:
            qla.qla_set_tuning(lat.ctx, rows, pf, ts)
            lat.set_index(n)
            lat.init_packet(w.packet)
            lat.advance(40)
            outs.append(lat.fields())
            energies.append(lat.energy())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    assert len(set(energies)) == 1


def test_zero_steps_is_identity(qla):
    q = _random_fields((16, 24), seed=3)
    with qla.Lattice(24, 16, 0.25) as lat:
        lat.set_index(np.full((16, 24), 2.0))
        lat.set_fields(q)
        lat.advance(0)
        np.testing.assert_array_equal(lat.fields(), q)


def test_energy_conserved_over_a_long_run(qla):
    """SKEW_HALF is unitary: FP64 energy drift stays at rounding level, and the
    three-shear rotations keep FP32 drift small (no systematic growth)."""
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        with qla.Lattice(w.nx, w.ny, w.delta, precision=prec) as lat:
            lat.set_index(n)
            lat.init_packet(w.packet)
            e0 = lat.energy()
            lat.advance(4000)
            drift = lat.energy() / e0 - 1
        print(f"prec={prec} energy drift over 4000 steps: {drift:.3e}")
        assert abs(drift) < tol


# ---------------------------------------------------------------------------------------
# errors forced from the host
def test_error_paths(qla):
    with qla.Lattice(16, 16, 0.25) as lat:
        with pytest.raises(qla.QlaError) as e:
            lat.advance(1)                                   # no index yet
        assert e.value.status == qla.QLA_ESTATE
        bad = np.full((16, 16), 1.5)
        bad[3, 4] = 0.0
        with pytest.raises(qla.QlaError) as e:
            lat.set_index(bad)
        assert e.value.status == qla.QLA_EINVAL
        bad[3, 4] = np.nan
        with pytest.raises(qla.QlaError):
            lat.set_index(bad)
        with pytest.raises(qla.QlaError) as e:
            qla.qla_set_tuning(lat.ctx, 24, 7, 0)            # unsupported prefetch depth
        assert e.value.status == qla.QLA_EINVAL
        with pytest.raises(qla.QlaError):
            qla.qla_set_tuning(lat.ctx, 24, 0, 3)            # unsupported steps per pass
        with pytest.raises(qla.QlaError):
            lat.advance(-1)
    with qla.Lattice(16, 16, 3.0) as lat:                    # delta/(4n) = 0.75 rad
        with pytest.raises(qla.QlaError) as e:
            lat.set_index(np.ones((16, 16)))
        assert e.value.status == qla.QLA_EINVAL
        assert "angle" in qla.qla_last_error()


def test_autotune_keeps_state_and_results(qla):
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    with qla.Lattice(w.nx, w.ny, w.delta) as ref:
        ref.set_index(n)
        ref.init_packet(w.packet)
        ref.advance(30)
        want = ref.fields()
    with qla.Lattice(w.nx, w.ny, w.delta) as lat:
        lat.set_index(n)
        lat.init_packet(w.packet)
        lat.advance(10)
        before = lat.fields()
        rows, pf, ts = qla.qla_autotune(lat.ctx)
        assert (rows, pf, ts) == qla.qla_get_tuning(lat.ctx)
        assert pf in (2, 3) and ts in (1, 2) and rows >= 1
        assert lat.steps == 10
        np.testing.assert_array_equal(lat.fields(), before)
        lat.advance(20)
        np.testing.assert_array_equal(lat.fields(), want)
