"""qla_energy_noalloc: the energy of Eq. (A13) of caller-owned planes, computed with the
library's file-scope scratch instead of any allocation. It must return the same bits as
qla_energy_device on a context holding the same state (same kernels, same summation
order), on two calls in a row with the second on a smaller lattice, so no partial sum
of the first call leaks into the second."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_energy_noalloc_matches_the_context_energy_on_two_calls(prec):
    import torch
    from paper_2604_21128_amd import qla
    qla.load()
    dt = torch.float64 if prec == qla.QLA_F64 else torch.float32
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(40 + prec)
    for nx, ny in ((300, 200), (37, 11)):
        q = rng.normal(size=(3, ny, nx))
        print(f"[noalloc] precision {prec}, {nx}x{ny}", flush=True)
        with torch.cuda.stream(stream):
            out = torch.zeros(2, dtype=torch.float64, device="cuda")
            pitch = nx + 5
            planes = torch.full((3, ny, pitch), float("nan"), dtype=dt, device="cuda")
            planes[:, :, :nx] = torch.from_numpy(q).to("cuda").to(dt)
            ctx = qla.qla_create(nx, ny, 0.25, prec, qla.QLA_V_SKEW_HALF, stream.cuda_stream)
            try:
                qla.qla_set_fields(ctx, q)
                qla.qla_energy_device(ctx, out[0:1])
                qla.qla_energy_noalloc(planes[0], planes[1], planes[2], nx, ny, pitch, prec,
                                       out[1:2], stream.cuda_stream)
                stream.synchronize()
            finally:
                qla.qla_destroy(ctx)
        e_ctx, e_na = out.cpu().numpy()
        assert e_na == e_ctx, (e_na, e_ctx)
        stored = q.astype(np.float32).astype(np.float64) if prec == qla.QLA_F32 else q
        want = float((stored ** 2).sum())
        assert abs(e_na / want - 1) < 1e-12


def test_energy_noalloc_rejects_bad_arguments():
    import torch
    from paper_2604_21128_amd import qla
    qla.load()
    a = torch.zeros((4, 8), dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for nx, ny, pitch, prec in ((0, 4, 8, 0), (8, 0, 8, 0), (8, 4, 7, 0), (8, 4, 8, 7)):
        with pytest.raises(qla.QlaError) as err:
            qla.qla_energy_noalloc(a, a, a, nx, ny, pitch, prec, out)
        assert err.value.status == qla.QLA_EINVAL
    with pytest.raises(qla.QlaError):
        qla.qla_energy_noalloc(a, a, 0, 8, 4, 8, 0, out)
