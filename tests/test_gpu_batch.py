"""Batched QLA (qla_batch_*): many uneven lattices advanced by one captured run.

Every lattice's result must equal, bit for bit, the single-lattice path on the same
inputs (the batched kernel applies the same per-site arithmetic), and one lattice
is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qla():
    from paper_2604_21128_amd import qla as q
    q.load()
    return q


SIZES = [(64, 64), (57, 90), (130, 40), (200, 200), (96, 128), (8, 8)]
STEPS = [12, 20, 8, 16, 10, 6]


def _instance(i, nx, ny):
    rng = np.random.default_rng(100 + i)
    e = workloads.Ellipse(nx / 2, ny / 2, rng.uniform(0.1, 0.3) * nx, rng.uniform(0.1, 0.3) * ny,
                          rng.uniform(0, np.pi), rng.uniform(1.5, 3.0), 1.0, 3.0)
    n = workloads.ellipse_index(nx, ny, e)
    p = workloads.Packet(x0=rng.uniform(0, nx), y0=ny / 2, sigma=rng.uniform(3, 6),
                         lam=rng.uniform(8, 16))
    return n, p


def _single(qla, n, p, steps, prec):
    ny, nx = n.shape
    with qla.Lattice(nx, ny, 0.25, precision=prec) as lat:
        lat.set_index(n)
        lat.init_packet(p)
        lat.advance(steps)
        return lat.fields()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [1, pytest.param(2, marks=pytest.mark.skip(
    reason="one cooperative launch per run (grid barrier between passes) hung in FP32 on "
           "the GPU; the cause is not shown, so the mode is switched off"))])
def test_batch_matches_single_lattice_bitwise(qla, prec, mode):
    b = qla.qla_batch_create([s[0] for s in SIZES], [s[1] for s in SIZES], [0.25] * len(SIZES),
                             precision=prec)
    try:
        inputs = []
        for i, (nx, ny) in enumerate(SIZES):
            n, p = _instance(i, nx, ny)
            inputs.append((n, p))
            ctx = qla.qla_batch_context(b, i)
            qla.qla_set_index(ctx, n)
            qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam)
        qla.qla_batch_plan(b, STEPS, mode)
        info = qla.qla_batch_plan_info(b)
        assert info["mode"] == mode and info["steps_per_pass"] in (1, 2)
        assert info["passes"] == max(STEPS) // info["steps_per_pass"]
        assert info["site_updates"] == sum(nx * ny * s for (nx, ny), s in zip(SIZES, STEPS))
        qla.qla_batch_run(b)
        for i, (nx, ny) in enumerate(SIZES):
            ctx = qla.qla_batch_context(b, i)
            assert qla.qla_step_count(ctx) == STEPS[i]
            got = qla.qla_get_fields(ctx, nx, ny)
            want = _single(qla, *inputs[i], STEPS[i], prec)
            np.testing.assert_array_equal(got, want, err_msg=f"instance {i} {nx}x{ny}")
        # a second run of the same graph continues from there (odd pass counts included)
        qla.qla_batch_run(b)
        ctx = qla.qla_batch_context(b, 3)
        np.testing.assert_array_equal(qla.qla_get_fields(ctx, 200, 200),
                                      _single(qla, *inputs[3], 2 * STEPS[3], prec))
    finally:
        qla.qla_batch_destroy(b)


def test_batch_against_oracle_and_energy(qla):
    nx, ny, steps = 96, 72, 24
    n, p = _instance(7, nx, ny)
    b = qla.qla_batch_create([nx, 40], [ny, 40], [0.25, 0.25], precision=0)
    try:
        ctx = qla.qla_batch_context(b, 0)
        qla.qla_set_index(ctx, n)
        qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam)
        ctx1 = qla.qla_batch_context(b, 1)
        qla.qla_set_index(ctx1, np.full((40, 40), 1.3))
        qla.qla_init_packet(ctx1, 10.0, 20.0, 4.0, 9.0)
        qla.qla_batch_plan(b, [steps, 10], 0)
        qla.qla_batch_run(b)
        got = qla.qla_get_fields(ctx, nx, ny)
        e = qla.qla_energy(ctx)
    finally:
        qla.qla_batch_destroy(b)
    want = oracle.advance(oracle.packet_from(n, p), n, 0.25, steps)
    assert np.linalg.norm(got - want[2:5]) / np.linalg.norm(want[2:5]) <= 1e-12
    assert abs(e / oracle.energy(want) - 1) < 1e-12


def test_batch_odd_steps_and_errors(qla):
    b = qla.qla_batch_create([32, 48], [40, 24], [0.25, 0.25], precision=1)
    try:
        ctx0 = qla.qla_batch_context(b, 0)
        with pytest.raises(qla.QlaError) as e:
            qla.qla_batch_plan(b, [4, 4], 2)               # cooperative mode is off
        assert e.value.status == qla.QLA_EINVAL
        with pytest.raises(qla.QlaError) as e:
            qla.qla_batch_plan(b, [4, 4], 0)               # no index yet
        assert e.value.status == qla.QLA_ESTATE
        with pytest.raises(qla.QlaError):
            qla.qla_destroy(ctx0)                           # owned by the batch
        with pytest.raises(qla.QlaError):
            qla.qla_batch_context(b, 2)
        ns = []
        for i, (nx, ny) in enumerate(((32, 40), (48, 24))):
            n, p = _instance(20 + i, nx, ny)
            ns.append((n, p))
            ctx = qla.qla_batch_context(b, i)
            qla.qla_set_index(ctx, n)
            qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam)
        qla.qla_batch_plan(b, [7, 4], 0)                    # odd: one step per pass
        assert qla.qla_batch_plan_info(b)["steps_per_pass"] == 1
        qla.qla_batch_run(b)
        for i, (nx, ny) in enumerate(((32, 40), (48, 24))):
            got = qla.qla_get_fields(qla.qla_batch_context(b, i), nx, ny)
            np.testing.assert_array_equal(got, _single(qla, *ns[i], (7, 4)[i], 1))
        qla.qla_batch_run(b)                                # 7 passes: parity flips
        for i, (nx, ny) in enumerate(((32, 40), (48, 24))):
            got = qla.qla_get_fields(qla.qla_batch_context(b, i), nx, ny)
            np.testing.assert_array_equal(got, _single(qla, *ns[i], 2 * (7, 4)[i], 1))
    finally:
        qla.qla_batch_destroy(b)


@pytest.mark.parametrize("fit", [False, True])
@pytest.mark.parametrize("rows,pf,ts", [(24, 2, 2), (56, 3, 2), (20, 3, 1)])
def test_batch_fixed_tuning_and_fitted_heights(qla, fit, rows, pf, ts):
    """Given tunings, with one segment height for all lattices or heights fitted to each
    lattice: results equal the single-lattice path bit for bit, and every height is one
    the kernel realises (whole loop trips of its register window)."""
    sizes = [(64, 300), (57, 90), (130, 40), (96, 128), (8, 8), (40, 161)]
    steps = [12, 20, 8, 10, 6, 14]
    b = qla.qla_batch_create([s[0] for s in sizes], [s[1] for s in sizes], [0.25] * len(sizes),
                             precision=1)
    try:
        inputs = []
        for i, (nx, ny) in enumerate(sizes):
            n, p = _instance(40 + i, nx, ny)
            inputs.append((n, p))
            ctx = qla.qla_batch_context(b, i)
            qla.qla_set_index(ctx, n)
            qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam)
        qla.qla_batch_plan_fixed(b, steps, rows, pf, ts, fit)
        info = qla.qla_batch_plan_info(b)
        assert (info["rows_per_segment"], info["prefetch_rows"], info["steps_per_pass"]) == \
            (rows, pf, ts)
        win, halo = pf + 4 * ts + 2, 4 * ts
        heights = [qla.qla_batch_segment_rows(b, i) for i in range(len(sizes))]
        realised = ((rows + 2 * halo + win - 1) // win) * win - 2 * halo
        for h in heights:
            assert h >= 1 and (h + 2 * halo) % win == 0
            assert 4 * h >= 3 * rows and (2 * h <= 3 * rows or h == realised)
        if not fit:
            assert len(set(heights)) == 1
        qla.qla_batch_run(b)
        for i, (nx, ny) in enumerate(sizes):
            got = qla.qla_get_fields(qla.qla_batch_context(b, i), nx, ny)
            np.testing.assert_array_equal(got, _single(qla, *inputs[i], steps[i], 1),
                                          err_msg=f"instance {i} {nx}x{ny} heights={heights}")
        with pytest.raises(qla.QlaError):
            qla.qla_batch_plan_fixed(b, steps, rows, 4, ts, fit)        # prefetch 4
        with pytest.raises(qla.QlaError):
            qla.qla_batch_plan_fixed(b, [7] + steps[1:], rows, pf, 2, fit)  # odd, 2 per pass
        with pytest.raises(qla.QlaError):
            qla.qla_batch_segment_rows(b, len(sizes))
    finally:
        qla.qla_batch_destroy(b)


def test_full_batched_workload_against_the_oracle(qla):
    """The 512-instance batched workload as the benchmark runs it: sides 256-1024, FP32,
    4 N steps each, autotuned plan captured in one graph. The two smallest instances are
    checked whole against the FP64 oracle (FP32 bar, relative L2 <= 1e-5), and every
    instance's energy stays at its initial value to FP32 rounding (the step is unitary)."""
    inst = workloads.sample_instances(512, seed=0)
    b = qla.qla_batch_create([i.n_side for i in inst], [i.n_side for i in inst],
                             [i.delta for i in inst], precision=1)
    try:
        ns, e0 = [], []
        for k, i in enumerate(inst):
            n = workloads.ellipse_index(i.n_side, i.n_side, i.ellipse)
            ns.append(n)
            ctx = qla.qla_batch_context(b, k)
            qla.qla_set_index(ctx, n)
            p = i.packet
            qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)
            e0.append(qla.qla_energy(ctx))
        qla.qla_batch_plan(b, [i.steps for i in inst], 0)
        print("plan", qla.qla_batch_plan_info(b), flush=True)
        qla.qla_batch_run(b)
        drift = max(abs(qla.qla_energy(qla.qla_batch_context(b, k)) / e0[k] - 1)
                    for k in range(len(inst)))
        print(f"max energy drift over 512 instances {drift:.2e}", flush=True)
        assert drift <= 2e-5
        smallest = sorted(range(len(inst)), key=lambda k: inst[k].n_side)[:2]
        for k in smallest:
            i = inst[k]
            got = qla.qla_get_fields(qla.qla_batch_context(b, k), i.n_side, i.n_side)
            want = oracle.advance(oracle.packet_from(ns[k], i.packet), ns[k], i.delta, i.steps)
            err = np.linalg.norm(got - want[2:5]) / np.linalg.norm(want[2:5])
            print(f"instance {k}: side {i.n_side}, {i.steps} steps, rel_l2 {err:.2e}",
                  flush=True)
            assert err <= 1e-5
    finally:
        qla.qla_batch_destroy(b)


def test_batch_degenerate_cases(qla):
    """A lattice with no steps is left as it was, a single-lattice batch equals the
    single-lattice path, and a batch whose step counts are all zero runs nothing."""
    sizes = [(40, 24), (33, 50), (64, 9)]
    b = qla.qla_batch_create([s[0] for s in sizes], [s[1] for s in sizes], [0.25] * 3,
                             precision=0)
    try:
        inputs = []
        for i, (nx, ny) in enumerate(sizes):
            n, p = _instance(60 + i, nx, ny)
            inputs.append((n, p))
            ctx = qla.qla_batch_context(b, i)
            qla.qla_set_index(ctx, n)
            qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam)
        before = qla.qla_get_fields(qla.qla_batch_context(b, 0), 40, 24)
        qla.qla_batch_plan(b, [0, 6, 3], 0)
        assert qla.qla_batch_plan_info(b)["passes"] == 6
        qla.qla_batch_run(b)
        np.testing.assert_array_equal(qla.qla_get_fields(qla.qla_batch_context(b, 0), 40, 24),
                                      before)
        assert qla.qla_step_count(qla.qla_batch_context(b, 0)) == 0
        for i, s in ((1, 6), (2, 3)):
            nx, ny = sizes[i]
            np.testing.assert_array_equal(qla.qla_get_fields(qla.qla_batch_context(b, i), nx, ny),
                                          _single(qla, *inputs[i], s, 0))
        qla.qla_batch_plan(b, [0, 0, 0], 0)
        info = qla.qla_batch_plan_info(b)
        assert info["passes"] == 0 and info["site_updates"] == 0
        qla.qla_batch_run(b)
        assert qla.qla_step_count(qla.qla_batch_context(b, 2)) == 3
    finally:
        qla.qla_batch_destroy(b)
    one = qla.qla_batch_create([72], [40], [0.25], precision=1)
    try:
        n, p = _instance(70, 72, 40)
        ctx = qla.qla_batch_context(one, 0)
        qla.qla_set_index(ctx, n)
        qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam)
        qla.qla_batch_plan(one, [10], 0)
        qla.qla_batch_run(one)
        np.testing.assert_array_equal(qla.qla_get_fields(ctx, 72, 40), _single(qla, n, p, 10, 1))
    finally:
        qla.qla_batch_destroy(one)


def test_run_refuses_an_index_set_after_planning_with_wider_angles(qla):
    # A run evaluates rotation angles with the series range fixed when it was planned
    # (here: every angle up to 1/16 rad). A sharp index set afterwards has potential
    # half-angles (delta/4)(n+ - n-)/n^2 = 0.125 rad: the run must refuse it (plan again)
    # rather than use the short series; after a new plan it runs and matches the
    # single-lattice path.
    sizes = [(64, 48), (40, 40)]
    b = qla.qla_batch_create([s[0] for s in sizes], [s[1] for s in sizes], [0.25, 0.25],
                             precision=1)
    try:
        smooth = []
        for i, (nx, ny) in enumerate(sizes):
            n, p = _instance(i, nx, ny)
            smooth.append((n, p))
            ctx = qla.qla_batch_context(b, i)
            qla.qla_set_index(ctx, n)
            qla.qla_init_packet(ctx, p.x0, p.y0, p.sigma, p.lam)
        steps = [8, 8]
        qla.qla_batch_plan_fixed(b, steps, 24, 2, 2, 0)
        sharp = np.ones((48, 64))
        sharp[:, 20:40] = 3.0
        ctx0 = qla.qla_batch_context(b, 0)
        qla.qla_set_index(ctx0, sharp)
        qla.qla_init_packet(ctx0, 10.0, 24.0, 4.0, 12.0)
        with pytest.raises(qla.QlaError) as err:
            qla.qla_batch_run(b)
        assert err.value.status == qla.QLA_ESTATE
        qla.qla_batch_plan_fixed(b, steps, 24, 2, 2, 0)
        qla.qla_batch_run(b)
        got = qla.qla_get_fields(ctx0, 64, 48)
        want = _single(qla, sharp, workloads.Packet(x0=10.0, y0=24.0, sigma=4.0, lam=12.0),
                       8, 1)
        assert np.array_equal(got, want)
    finally:
        qla.qla_batch_destroy(b)
