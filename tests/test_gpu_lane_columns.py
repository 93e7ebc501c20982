"""FP32 step kernel with two lattice columns per lane, against the oracle and against
the one-column kernel.

Each column goes through the same arithmetic in both layouts, so the two FP32
kernels must agree bit for bit; against the FP64 oracle the FP32 bar holds
(relative L2 <= 1e-5). Lattices are ragged (widths one pair past a strip of 112
or 120 columns, narrower than one wave, exact multiples), with random fields and
index, odd step counts (single steps after two-step passes), every potential mode
and both triples.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

BZ = [0, 1, 5]


@pytest.fixture(scope="module")
def qla():
    from paper_2604_21128_amd import qla as q
    q.load()
    return q


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(qla, n, q, delta, steps, cols, tuning, vmode=0, triple=0):
    ny, nx = n.shape
    with qla.Lattice(nx, ny, delta, precision=qla.QLA_F32, potential=vmode,
                     triple=triple) as lat:
        qla.qla_set_tuning(lat.ctx, *tuning)
        qla.qla_set_lane_columns(lat.ctx, cols)
        assert qla.qla_get_lane_columns(lat.ctx) == cols
        lat.set_index(n)
        lat.set_fields(q)
        lat.advance(steps)
        return lat.fields(), lat.energy()


@pytest.mark.parametrize("tuning", [(0, 3, 2), (1, 2, 2), (40, 3, 1), (16, 2, 1)])
@pytest.mark.parametrize("nx,ny,steps", [
    (8, 8, 5),        # one wave covers the row 16 times over
    (58, 121, 7),     # narrower than one wave
    (114, 77, 9),     # one pair past a two-step strip (112 columns)
    (122, 40, 6),     # one pair past a one-step strip (120 columns)
    (224, 36, 4),     # exact multiple of the two-step strip
    (200, 9, 5),      # short and wide
])
def test_pairs_match_oracle_and_single_columns(qla, nx, ny, steps, tuning):
    rng = np.random.default_rng(nx * 7 + ny)
    n = np.clip(rng.uniform(1.2, 2.8) + rng.uniform(-0.5, 0.5, size=(ny, nx)), 1.0, 3.0)
    q = rng.standard_normal((3, ny, nx))
    q32 = q.astype(np.float32).astype(np.float64)
    for vmode in (0, 1, 2, 3):
        want = np.zeros((6, ny, nx))
        want[2:5] = q32
        oracle.advance(want, n, 0.4, steps, vmode)
        one, e1 = _run(qla, n, q32, 0.4, steps, 1, tuning, vmode)
        two, e2 = _run(qla, n, q32, 0.4, steps, 2, tuning, vmode)
        err = rel_l2(two, want[2:5])
        print(f"{nx}x{ny} steps={steps} tuning={tuning} vmode={vmode} rel_l2={err:.3e}",
              flush=True)
        assert err <= 1e-5
        np.testing.assert_array_equal(two, one)
        assert e1 == e2


@pytest.mark.parametrize("vmode", [0, 2])
def test_pairs_bz_triple(qla, vmode):
    ny, nx, steps = 45, 130, 7
    rng = np.random.default_rng(77)
    n = rng.uniform(1.0, 2.5, size=(ny, nx))
    q = np.zeros((6, ny, nx))
    q[BZ] = rng.standard_normal((3, ny, nx)).astype(np.float32)
    one, _ = _run(qla, n, q[BZ], 0.25, steps, 1, (0, 3, 2), vmode, qla.QLA_TRIPLE_BZ)
    two, _ = _run(qla, n, q[BZ], 0.25, steps, 2, (0, 3, 2), vmode, qla.QLA_TRIPLE_BZ)
    oracle.advance(q, n, 0.25, steps, vmode)
    assert rel_l2(two, q[BZ]) <= 1e-5
    np.testing.assert_array_equal(two, one)


def test_pairs_large_angles(qla):
    # delta = 1.6: the long-series kernel variant
    ny, nx = 40, 70
    n = 1.0 + 0.5 * (1 + np.sin(2 * np.pi * np.arange(nx) / nx))[None, :] \
        * (1 + np.cos(2 * np.pi * np.arange(ny) / ny))[:, None] / 2
    q = np.random.default_rng(5).standard_normal((3, ny, nx)).astype(np.float32)
    for vmode in (0, 1, 3):
        want = np.zeros((6, ny, nx))
        want[2:5] = q
        oracle.advance(want, n, 1.6, 12, vmode)
        one, _ = _run(qla, n, q, 1.6, 12, 1, (0, 0, 0), vmode)
        two, _ = _run(qla, n, q, 1.6, 12, 2, (0, 0, 0), vmode)
        assert rel_l2(two, want[2:5]) <= 1e-5
        np.testing.assert_array_equal(two, one)


def test_pairs_full_size_4096(qla):
    """The 4096^2 ellipse workload's lattice with random fields, 20 steps: the whole
    field equals the one-column kernel's bit for bit, and windows whose centre the
    oracle computes exactly (4 cells of dependence per step and axis) match it."""
    w = workloads.plain_4096()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    q = np.random.default_rng(42).standard_normal((3, w.ny, w.nx)).astype(np.float32)
    steps = 20
    one, e1 = _run(qla, n, q, w.delta, steps, 1, (56, 3, 2))
    two, e2 = _run(qla, n, q, w.delta, steps, 2, (56, 3, 2))
    assert np.array_equal(two, one) and e1 == e2
    del one
    margin = 4 * steps + 2
    half = margin + 12
    e = w.ellipse
    for cx, cy in [(int(e.xc - e.a), int(e.yc)), (int(e.xc), int(e.yc + e.b)), (0, 0),
                   (w.nx - 1, 1234), (111, 3000)]:
        ys = np.arange(cy - half, cy + half + 1) % w.ny
        xs = np.arange(cx - half, cx + half + 1) % w.nx
        nw = np.ascontiguousarray(n[np.ix_(ys, xs)])
        qw = np.zeros((6,) + nw.shape)
        qw[2:5] = q[:, ys][:, :, xs]
        out = oracle.advance(qw, nw, w.delta, steps)[2:5]
        inner = slice(margin, 2 * half + 1 - margin)
        err = rel_l2(two[:, ys[inner]][:, :, xs[inner]], out[:, inner, inner])
        print(f"window centre=({cx},{cy}) rel_l2={err:.3e}", flush=True)
        assert err <= 1e-5


def test_lane_columns_errors_and_autotune(qla):
    with qla.Lattice(64, 32, 0.25, precision=qla.QLA_F64) as lat:
        assert qla.qla_get_lane_columns(lat.ctx) == 1
        with pytest.raises(qla.QlaError) as e:
            qla.qla_set_lane_columns(lat.ctx, 2)
        assert e.value.status == qla.QLA_EINVAL
    with qla.Lattice(63, 32, 0.25, precision=qla.QLA_F32) as lat:
        with pytest.raises(qla.QlaError):
            qla.qla_set_lane_columns(lat.ctx, 2)
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    with qla.Lattice(w.nx, w.ny, w.delta, precision=qla.QLA_F32) as lat:
        for bad in (-1, 3):
            with pytest.raises(qla.QlaError):
                qla.qla_set_lane_columns(lat.ctx, bad)
        qla.qla_set_lane_columns(lat.ctx, 2)
        qla.qla_set_lane_columns(lat.ctx, 0)
        assert qla.qla_get_lane_columns(lat.ctx) == 1
        lat.set_index(n)
        lat.init_packet(w.packet)
        lat.advance(10)
        before = lat.fields()
        qla.qla_autotune(lat.ctx)
        assert qla.qla_get_lane_columns(lat.ctx) in (1, 2)
        assert lat.steps == 10
        np.testing.assert_array_equal(lat.fields(), before)
        lat.advance(20)
        got = lat.fields()
    with qla.Lattice(w.nx, w.ny, w.delta, precision=qla.QLA_F32) as ref:
        ref.set_index(n)
        ref.init_packet(w.packet)
        ref.advance(30)
        np.testing.assert_array_equal(got, ref.fields())
