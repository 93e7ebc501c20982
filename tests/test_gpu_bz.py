"""The B_z triple (q0, q1, q5) and the divergence diagnostic on the GPU, against the oracle.

The oracle steps all six components with the printed operators, so a B_z state (only
q0, q1, q5 non-zero) checks the B_z path directly. Tolerances as for the E_z triple:
relative L2 <= 1e-12 (FP64) and <= 1e-5 (FP32). The divergence diagnostic is a
plain FP64 reduction; it must match the oracle's centred differences to 1e-12.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}
BZ = [0, 1, 5]          # ABI plane order of the B_z triple


@pytest.fixture(scope="module")
def qla():
    from paper_2604_21128_amd import qla as q
    q.load()
    return q


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _bz_packet(n, p):
    return oracle.packet_bz(n, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)


@pytest.mark.parametrize("prec", [0, 1])
def test_bz_packet_and_readout_match_oracle(qla, prec):
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    with qla.Lattice(w.nx, w.ny, w.delta, precision=prec, triple=qla.QLA_TRIPLE_BZ) as lat:
        lat.set_index(n)
        for p in (w.packet, workloads.Packet(x0=30.5, y0=200.0, sigma=9.0, lam=12.0, phi=0.7,
                                               amp=0.5, planar=False)):
            lat.init_packet(p)
            want = _bz_packet(n, p)
            tol = 1e-15 if prec == 0 else 6e-8
            assert np.abs(lat.fields() - want[BZ]).max() <= tol
            phys = lat.fields(physical=True)
            ex, ey, bz = oracle.physical_fields_bz(want, n)
            assert np.abs(phys - np.stack([ex, ey, bz])).max() <= tol


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("vmode", [0, 2])
def test_bz_parity_small_workload(qla, prec, vmode):
    w = workloads.parity_small()
    n = workloads.ellipse_index(w.nx, w.ny, w.ellipse)
    q = _bz_packet(n, w.packet)
    with qla.Lattice(w.nx, w.ny, w.delta, precision=prec, potential=vmode,
                     triple=qla.QLA_TRIPLE_BZ) as lat:
        lat.set_index(n)
        lat.init_packet(w.packet)
        lat.advance(w.steps)
        got = lat.fields()
        e = lat.energy()
    oracle.advance(q, n, w.delta, w.steps, vmode)
    assert not q[2:5].any()
    assert rel_l2(got, q[BZ]) <= TOL[prec]
    assert abs(e / oracle.energy(q) - 1) <= (1e-12 if prec == 0 else 1e-6)


@pytest.mark.parametrize("tuning", [(24, 2, 1), (40, 3, 2)])
def test_bz_parity_ragged_random_state(qla, tuning):
    # ragged lattice, random fields and index, odd step count (a single step after the
    # two-step passes), both temporal-blocking depths
    ny, nx, steps = 37, 70, 7
    rng = np.random.default_rng(5)
    n = np.clip(1.8 + rng.uniform(-0.6, 0.6, size=(ny, nx)), 1.0, 3.0)
    q = np.zeros((6, ny, nx))
    q[BZ] = rng.standard_normal((3, ny, nx))
    with qla.Lattice(nx, ny, 0.25, triple=qla.QLA_TRIPLE_BZ) as lat:
        lat.set_index(n)
        qla.qla_set_tuning(lat.ctx, *tuning)
        lat.set_fields(q[BZ])
        lat.advance(steps)
        got = lat.fields()
    oracle.advance(q, n, 0.25, steps)
    assert rel_l2(got, q[BZ]) <= 1e-12


def test_bz_and_ez_triples_evolve_independently(qla):
    # a state with both triples populated evolves as the two triples apart (oracle)
    ny, nx, steps = 40, 48, 6
    rng = np.random.default_rng(9)
    n = rng.uniform(1.0, 2.5, size=(ny, nx))
    q = rng.standard_normal((6, ny, nx))
    want = oracle.advance(q.copy(), n, 0.25, steps)
    got = {}
    for triple, planes in ((qla.QLA_TRIPLE_EZ, [2, 3, 4]), (qla.QLA_TRIPLE_BZ, BZ)):
        with qla.Lattice(nx, ny, 0.25, triple=triple) as lat:
            lat.set_index(n)
            lat.set_fields(q[planes])
            lat.advance(steps)
            got[triple] = lat.fields()
        assert rel_l2(got[triple], want[planes]) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("triple", [0, 1])
def test_divergence_matches_oracle(qla, prec, triple):
    ny, nx = 45, 66
    rng = np.random.default_rng(13 + triple)
    n = rng.uniform(1.0, 3.0, size=(ny, nx))
    planes = [2, 3, 4] if triple == 0 else BZ
    q = np.zeros((6, ny, nx))
    q[planes] = rng.standard_normal((3, ny, nx))
    if prec == 1:
        q = q.astype(np.float32).astype(np.float64)     # what the FP32 planes hold
    with qla.Lattice(nx, ny, 0.25, precision=prec, triple=triple) as lat:
        lat.set_index(n)
        lat.set_fields(q[planes])
        l2, mx, scale = lat.divergence()
    div_b, div_d = oracle.divergence(q, n, 0.25)
    div = div_b if triple == 0 else div_d
    if triple == 0:
        fx, fy = q[3], q[4]
    else:
        fx, fy = n * q[0], n * q[1]
    ddx = (np.roll(fx, -1, 1) - np.roll(fx, 1, 1)) / 0.5
    ddy = (np.roll(fy, -1, 0) - np.roll(fy, 1, 0)) / 0.5
    assert abs(l2 / np.sqrt((div ** 2).sum()) - 1) <= 1e-12
    assert abs(mx / np.abs(div).max() - 1) <= 1e-12
    assert abs(scale / np.sqrt((ddx ** 2 + ddy ** 2).sum()) - 1) <= 1e-12


def test_divergence_of_the_initial_planar_packets_vanishes(qla):
    # a planar packet moving along x in vacuum has B = (0, By(x)) or D = (0, Dy(x)):
    # every centred difference in the divergence is exactly zero
    w = workloads.parity_small()
    n = np.ones((w.ny, w.nx))
    for triple in (0, 1):
        with qla.Lattice(w.nx, w.ny, w.delta, triple=triple) as lat:
            lat.set_index(n)
            lat.init_packet(w.packet)
            l2, mx, scale = lat.divergence()
        assert mx == 0.0 and l2 == 0.0 and scale == 0.0


@pytest.mark.parametrize("ellipse", [
    workloads.Ellipse(128.0, 128.0, 40.0, 20.0, 0.0, 2.0, 1.0, 3.0),
    workloads.Ellipse(70.3, 150.0, 55.0, 17.5, 0.9, 1.0, 2.6, 2.0),     # rotated bubble
])
def test_set_index_ellipse_matches_the_input_generator(qla, ellipse):
    nx, ny = 256, 200
    want = workloads.ellipse_index(nx, ny, ellipse)
    with qla.Lattice(nx, ny, 0.25) as lat:
        qla.qla_set_index_ellipse(lat.ctx, ellipse.xc, ellipse.yc, ellipse.a, ellipse.b,
                                  ellipse.rot, ellipse.n_in, ellipse.n_out, ellipse.width)
        th, _, _ = lat.coefficients()
    # theta = delta / (4 n): n to a few ulps (cos, sin, tanh of the device libraries)
    np.testing.assert_allclose(0.25 / (4 * th), want, rtol=1e-14, atol=0)
    with qla.Lattice(nx, ny, 0.25) as lat:
        with pytest.raises(qla.QlaError):
            qla.qla_set_index_ellipse(lat.ctx, 1, 1, 0.0, 5, 0, 2, 1, 3)    # a = 0
