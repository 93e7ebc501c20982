"""The neural-operator surrogate's GPU kernels (qla_fno_*) against the FP64 CPU reference.

The library stores activations, the Fourier bases and the GEMM weights in BF16 and
accumulates in FP32, so it is compared with the FP64 reference on relative L2 error
with a tolerance set by BF16 rounding. Weights are set to BF16-representable values,
so only the rounding of stored activations and of the cosine/sine bases counts: each
stored value carries a relative error of at most u = 2^-9 ~ 2e-3, independent from
value to value, and a layer stores about six tensors on the way from v_l to v_{l+1}
(Z, T is FP32, S, U, z, v); adding those in quadrature over the depth gives a few u
on the output, and the tolerance is 5u ~ 1e-2 on the output and on each parameter
block of the gradient.

All work (torch allocations and copies, library calls) runs on one stream, so a
temporary tensor handed to an asynchronous call is never reused before the call ran.
"""
import numpy as np
import pytest
import torch

from oracle import fno

pytestmark = pytest.mark.gpu

FWD_TOL = 1e-2
GRAD_TOL = 1e-2


@pytest.fixture(scope="module")
def qla():
    from paper_2604_21128_amd import qla as q
    q.load()
    return q


@pytest.fixture(scope="module", autouse=True)
def stream():
    prev = torch.cuda.current_stream()
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    yield st
    torch.cuda.synchronize()
    torch.cuda.set_stream(prev)


def bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_round(x):
    return bf16_value(bf16_bits(x))


def to_device(bits):
    return torch.from_numpy(bits.view(np.int16).copy()).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def make_params(s, seed, spectral=1.0, pointwise=1.0):
    """Weights at initialisation-like scales, rounded to BF16-representable values."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in fno.param_shapes(s):
        n = int(np.prod(shape))
        if name == "P":
            v = rng.normal(0, 1 / np.sqrt(s.cin), n)
        elif name.startswith("W"):
            v = pointwise * rng.normal(0, 1 / np.sqrt(s.C), n)
        elif name.startswith("R"):
            v = spectral * rng.normal(0, 1 / np.sqrt(2 * s.C), n)
        elif name == "Q1":
            v = rng.normal(0, 1 / np.sqrt(s.C), n)
        elif name == "Q2":
            v = rng.normal(0, 1 / np.sqrt(s.C2), n)
        else:
            v = rng.normal(0, 0.1, n)
        parts.append(v)
    return bf16_round(np.concatenate(parts)).astype(np.float32)


class Net:
    def __init__(self, qla, s, batch, seed=0):
        self.qla, self.s = qla, s
        self.h = qla.qla_fno_create(s.H, s.W, s.cin, s.cout, s.C, s.m, s.L, s.C2, batch, seed,
                                    torch.cuda.current_stream().cuda_stream)

    def close(self):
        if self.h:
            self.qla.qla_fno_destroy(self.h)
            self.h = 0


@pytest.fixture
def net_factory(qla):
    nets = []

    def make(s, batch, seed=0):
        n = Net(qla, s, batch, seed)
        nets.append(n)
        return n
    yield make
    for n in nets:
        n.close()


def inputs(s, B, seed):
    rng = np.random.default_rng(seed)
    u = bf16_bits(rng.normal(size=(B, s.cin, s.H, s.W)))
    t = bf16_bits(rng.normal(size=(B, s.cout, s.H, s.W)))
    return u, t


def gpu_forward(qla, net, u_bits, B):
    out = torch.empty(B * net.s.cout * net.s.H * net.s.W, dtype=torch.float32, device="cuda")
    qla.qla_fno_forward(net.h, to_device(u_bits), B, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64).reshape(B, net.s.cout, net.s.H, net.s.W)


# "fused": rows a multiple of 64 cells, where the inverse x transform runs inside the
# channel-mixing GEMM; "small" and "ragged" take the separate path; "mix256" (width 64,
# rows of 256 cells) runs the dedicated layer kernel; "spectral" (a multiple of 32 rows
# of a multiple of 128 cells, 16 modes: every row and column of the tiles in use) runs
# the one-pass x and y transform kernel, as do "full" and the 512^2 and 64 x 256 band
# fraction cases. The weight gradients of the pointwise layers run the matrix-core
# weight-gradient kernel wherever the pixels per sample are a multiple of 64 (all but
# "ragged"), in each of its tile shapes: up to 64 x 64 output x input channels in these
# cases, 128 x 32 (projection 1) and 64 x 128 (projection 2 with 40 outputs) in "wide",
# and 128 x 64 (projection 1) and 32 x 128 (projection 2) in "full". Training's projection
# kernels (width 64, rows of a multiple of 256 cells) run with two groups of 64 projection
# channels in "proj" and "full" and with one in "proj64" (two outputs).
SPECS = {
    "small": fno.Spec(H=40, W=72, cin=4, cout=3, C=16, m=6, L=3, C2=24),
    "ragged": fno.Spec(H=33, W=70, cin=4, cout=3, C=10, m=5, L=2, C2=70),
    "fused": fno.Spec(H=24, W=128, cin=4, cout=3, C=16, m=7, L=3, C2=40),
    # width 64 on rows of 256 cells: the layers run the 256-pixel mixing kernel
    "mix256": fno.Spec(H=16, W=256, cin=4, cout=3, C=64, m=6, L=2, C2=40),
    "spectral": fno.Spec(H=96, W=384, cin=4, cout=3, C=16, m=16, L=2, C2=40),
    "wide": fno.Spec(H=16, W=128, cin=4, cout=40, C=32, m=4, L=1, C2=128),
    # width 64 on rows of 256 cells with 128 projection channels: training's first
    # projection runs its dedicated kernel (two groups of 64 outputs), as in "full"
    "proj": fno.Spec(H=8, W=256, cin=4, cout=3, C=64, m=4, L=1, C2=128),
    # the same with 64 projection channels: one group of 64 outputs in both projection kernels
    "proj64": fno.Spec(H=8, W=512, cin=4, cout=2, C=64, m=4, L=1, C2=64),
}


def test_param_count_matches_the_reference_layout(qla, net_factory):
    for s in SPECS.values():
        net = net_factory(s, 2)
        assert qla.qla_fno_param_count(net.h) == fno.param_count(s)


@pytest.mark.parametrize("name", list(SPECS))
@pytest.mark.parametrize("variant", ["both", "spectral_only", "pointwise_only"])
def test_forward_matches_fp64_reference(qla, net_factory, name, variant):
    s = SPECS[name]
    B = 3
    net = net_factory(s, B)
    p = make_params(s, 11, spectral=0.0 if variant == "pointwise_only" else 1.0,
                    pointwise=0.0 if variant == "spectral_only" else 1.0)
    qla.qla_fno_set_params(net.h, p)
    np.testing.assert_array_equal(qla.qla_fno_get_params(net.h), p)
    u, _ = inputs(s, B, 12)
    got = gpu_forward(qla, net, u, B)
    want = fno.predict(s, p.astype(np.float64), bf16_value(u))
    err = rel(got, want)
    print(f"forward {name} {variant}: rel L2 {err:.2e}")
    assert err <= FWD_TOL


@pytest.mark.parametrize("name", list(SPECS))
def test_gradient_matches_fp64_reference(qla, net_factory, name):
    s = SPECS[name]
    B = 2
    net = net_factory(s, B)
    p = make_params(s, 21)
    qla.qla_fno_set_params(net.h, p)
    u, t = inputs(s, B, 22)
    loss = qla.qla_fno_loss_grad(net.h, to_device(u), to_device(t), B)
    g = qla.qla_fno_get_grads(net.h).astype(np.float64)
    want_loss, want = fno.loss_and_grad(s, p.astype(np.float64), bf16_value(u), bf16_value(t))
    assert abs(loss / want_loss - 1) <= FWD_TOL
    off = 0
    for pname, shape in fno.param_shapes(s):
        n = int(np.prod(shape))
        err = rel(g[off:off + n], want[off:off + n])
        print(f"grad {name} {pname}: rel L2 {err:.2e}")
        assert err <= GRAD_TOL, pname
        off += n
    # directional derivative along a random direction against FP64 central differences
    d = np.random.default_rng(23).normal(size=p.size)
    eps = 1e-4
    pp = p.astype(np.float64)
    fd = (fno.loss_value(s, pp + eps * d, bf16_value(u), bf16_value(t))
          - fno.loss_value(s, pp - eps * d, bf16_value(u), bf16_value(t))) / (2 * eps)
    assert abs(g @ d - fd) <= GRAD_TOL * abs(fd)


@pytest.mark.parametrize("name", ["mix256", "wide", "full"])
def test_gradients_repeat_bit_for_bit(qla, net_factory, name):
    """No sum in the loss and its gradient depends on scheduling: the weight and bias
    gradients of the pointwise layers (lift, layer weights, both projections) come from the
    matrix-core weight-gradient kernel, whose per-block partial sums are added in a fixed
    order, the loss sums add their per-block shares in block order, and every other
    reduction has one writer per output. Two backward passes over the same batch give
    identical bits in every parameter block. "full" is the surrogate's 512^2, width-64
    shape (batch 1)."""
    s = SPECS.get(name) or fno.Spec(H=512, W=512, cin=4, cout=3, C=64, m=12, L=4, C2=128)
    B = 2 if name in SPECS else 1
    net = net_factory(s, B)
    qla.qla_fno_set_params(net.h, make_params(s, 91))
    u, t = inputs(s, B, 92)
    ud, td = to_device(u), to_device(t)
    grads = []
    for _ in range(2):
        qla.qla_fno_loss_grad(net.h, ud, td, B)
        grads.append(qla.qla_fno_get_grads(net.h))
    off = 0
    for pname, shape in fno.param_shapes(s):
        n = int(np.prod(shape))
        np.testing.assert_array_equal(grads[0][off:off + n], grads[1][off:off + n],
                                      err_msg=f"{name} {pname}")
        assert np.abs(grads[0][off:off + n]).max() > 0, pname
        off += n


def test_adam_step_matches_the_reference_update(qla, net_factory):
    s = SPECS["small"]
    net = net_factory(s, 2)
    p = make_params(s, 31)
    qla.qla_fno_set_params(net.h, p)
    u, t = inputs(s, 2, 32)
    pp = p.astype(np.float64)
    m1 = np.zeros_like(pp)
    m2 = np.zeros_like(pp)
    for step in (1, 2):
        qla.qla_fno_loss_grad(net.h, to_device(u), to_device(t), 2)
        g = qla.qla_fno_get_grads(net.h).astype(np.float64)
        qla.qla_fno_adam_step(net.h, 1e-3)
        pp, m1, m2 = fno.adam(pp, g, m1, m2, step, 1e-3)
        got = qla.qla_fno_get_params(net.h).astype(np.float64)
        np.testing.assert_allclose(got, pp, rtol=1e-5, atol=1e-7)


def test_training_learns_a_translation(qla, net_factory):
    """Learn u -> roll(u) (a pure spectral map): the loss must fall well below its start."""
    s = fno.Spec(H=32, W=32, cin=3, cout=3, C=16, m=8, L=2, C2=32)
    B = 8
    net = net_factory(s, B, seed=5)
    rng = np.random.default_rng(41)

    def smooth_batch():
        x = np.zeros((B, 3, 32, 32))
        for ky in range(-4, 5):
            for kx in range(0, 5):
                a = rng.normal(size=(B, 3, 1, 1)) / (1 + ky * ky + kx * kx)
                ph = rng.uniform(0, 2 * np.pi, size=(B, 3, 1, 1))
                y, xx = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
                x += a * np.cos(2 * np.pi * (ky * y + kx * xx) / 32 + ph)
        return x

    losses = []
    for it in range(300):
        x = smooth_batch()
        u = bf16_bits(x)
        t = bf16_bits(np.roll(x, (5, -7), axis=(2, 3)))
        loss_dev = torch.zeros(1, dtype=torch.float32, device="cuda")
        qla.qla_fno_train_step(net.h, to_device(u), to_device(t), B, 3e-3, loss_dev)
        losses.append(float(loss_dev.item()))
    first, last = np.mean(losses[:10]), np.mean(losses[-10:])
    print(f"translation task: loss {first:.3f} -> {last:.3f}")
    assert last < 0.25 * first and last < 0.2


def test_pack_and_output_energy(qla, net_factory):
    nx, ny = 48, 40
    rng = np.random.default_rng(51)
    q = rng.normal(size=(3, ny, nx))
    n = rng.uniform(1.0, 3.0, size=(ny, nx))
    qd = torch.tensor(q, device="cuda")
    nd = torch.tensor(n, device="cuda")
    inp = torch.zeros(4 * nx * ny, dtype=torch.int16, device="cuda")
    tgt = torch.zeros(3 * nx * ny, dtype=torch.int16, device="cuda")
    qla.qla_fno_pack(qd, nd, nx, ny, 2.0, inp, tgt, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    want_in = bf16_bits(np.concatenate([(n - 2.0)[None], q]).astype(np.float32))
    np.testing.assert_array_equal(inp.cpu().numpy().view(np.uint16).reshape(4, ny, nx), want_in)
    np.testing.assert_array_equal(tgt.cpu().numpy().view(np.uint16).reshape(3, ny, nx),
                                  bf16_bits(q.astype(np.float32)))
    s = fno.Spec(H=ny, W=nx, cin=4, cout=3, C=8, m=4, L=1, C2=8)
    net = net_factory(s, 2)
    u = np.stack([want_in, bf16_bits(rng.normal(size=(4, ny, nx)))])
    out = gpu_forward(qla, net, u, 2)
    e = torch.zeros(2, dtype=torch.float64, device="cuda")
    qla.qla_fno_output_energy(net.h, 2, e)
    np.testing.assert_allclose(e.cpu().numpy(), (out ** 2).reshape(2, -1).sum(axis=1), rtol=1e-12)


def test_batch_bounds_are_checked(qla, net_factory):
    s = SPECS["small"]
    net = net_factory(s, 2)
    u, _ = inputs(s, 3, 61)
    out = torch.empty(3 * s.cout * s.H * s.W, dtype=torch.float32, device="cuda")
    for b in (0, 3):
        with pytest.raises(qla.QlaError) as e:
            qla.qla_fno_forward(net.h, to_device(u), b, out)
        assert e.value.status == qla.QLA_EINVAL


def test_full_size_network_forward_and_gradient(qla, net_factory):
    """The surrogate's own shape: 512^2 grid, width 64, 12 modes, 4 layers."""
    s = fno.Spec(H=512, W=512, cin=4, cout=3, C=64, m=12, L=4, C2=128)
    B = 1
    net = net_factory(s, B)
    p = make_params(s, 71)
    qla.qla_fno_set_params(net.h, p)
    u, t = inputs(s, B, 72)
    got = gpu_forward(qla, net, u, B)
    loss = qla.qla_fno_loss_grad(net.h, to_device(u), to_device(t), B)
    g = qla.qla_fno_get_grads(net.h).astype(np.float64)
    want_loss, want = fno.loss_and_grad(s, p.astype(np.float64), bf16_value(u), bf16_value(t))
    want_out = fno.predict(s, p.astype(np.float64), bf16_value(u))
    err = rel(got, want_out)
    print(f"full size forward rel L2 {err:.2e}, loss {loss:.5f} vs {want_loss:.5f}")
    assert err <= FWD_TOL
    assert abs(loss / want_loss - 1) <= FWD_TOL
    off = 0
    for pname, shape in fno.param_shapes(s):
        n = int(np.prod(shape))
        e = rel(g[off:off + n], want[off:off + n])
        print(f"full size grad {pname}: rel L2 {e:.2e}")
        assert e <= GRAD_TOL, pname
        off += n


@pytest.mark.parametrize("name", list(SPECS) + ["full"])
def test_inference_forward_agrees_with_the_training_forward(qla, net_factory, name):
    """Inference runs the projection as one fused kernel (hidden layer on chip, GELU in
    FP32 with the Abramowitz & Stegun 7.1.26 erf); training runs it as two GEMMs with a
    BF16 hidden layer. Both are the same function to BF16 rounding: the output energies
    (the acceptance test's quantity) agree to 1e-3 and the outputs to 5e-3."""
    s = SPECS.get(name) or fno.Spec(H=128, W=128, cin=4, cout=3, C=64, m=12, L=2, C2=128)
    B = 2
    net = net_factory(s, B)
    qla.qla_fno_set_params(net.h, make_params(s, 81))
    u, t = inputs(s, B, 82)
    e_inf = torch.zeros(B, dtype=torch.float64, device="cuda")
    e_trn = torch.zeros(B, dtype=torch.float64, device="cuda")
    out_inf = gpu_forward(qla, net, u, B)
    qla.qla_fno_output_energy(net.h, B, e_inf)
    qla.qla_fno_loss_grad(net.h, to_device(u), to_device(t), B)   # training forward
    qla.qla_fno_output_energy(net.h, B, e_trn)
    torch.cuda.synchronize()
    ratio = e_inf.cpu().numpy() / e_trn.cpu().numpy()
    print(f"{name}: inference / training output energy {ratio}")
    assert np.abs(ratio - 1).max() <= 1e-3
    want = fno.predict(s, make_params(s, 81).astype(np.float64), bf16_value(u))
    assert rel(out_inf, want) <= FWD_TOL


def _band_inputs(H, W, cin, m, seed):
    """Samples whose band fractions span [0, 1]: plane waves inside and outside the kept
    modes, their mix, Gaussian packets of short and long wavelength along x, noise and
    a zero sample; channel 0 is an unrelated medium-like plane."""
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")

    def wave(ky, kx, ph=0.3):
        return np.cos(2 * np.pi * (ky * y / H + kx * x / W) + ph)

    def packet(lam, sigma):
        return np.exp(-0.5 * ((x - W / 3) / sigma) ** 2) * np.cos(2 * np.pi * (x - W / 3) / lam)

    fields = [
        [wave(1, 2), wave(H - 2, 1), wave(0, m - 1)],
        [wave(m + 1, 1), wave(2, m), wave(H // 2 - 1, W // 2 - 1)],
        [wave(1, 1) + 0.7 * wave(m + 2, m + 1), 0.2 * wave(m, 0), rng.normal(size=(H, W))],
        [packet(W / 3.0, W / 8.0), 0 * x, -packet(W / 3.0, W / 8.0)],
        [packet(W / (m + 6.0), W / 10.0), 0 * x, -packet(W / (m + 6.0), W / 10.0)],
        [rng.normal(size=(H, W)) for _ in range(3)],
        [np.zeros((H, W))] * 3,
    ]
    u = np.zeros((len(fields), cin, H, W))
    for b, f in enumerate(fields[:-1]):     # the last sample stays zero in every plane
        u[b, 0] = 1.0 + 0.5 * np.tanh(rng.normal(size=(H, W)))
        for c in range(min(3, cin - 1)):
            u[b, 1 + c] = f[c]
    return bf16_bits(u)


@pytest.mark.parametrize("H,W,m,first,channels", [
    (512, 512, 12, 1, 3),     # the surrogate's grid and the packet planes (q2, q3, q4)
    (64, 256, 9, 1, 3),       # the one-pass transform kernel at two row pieces per thread
    (40, 24, 5, 1, 3),        # ragged: rows and columns not multiples of the GEMM tiles
    (40, 24, 5, 0, 4),        # every input plane
])
def test_band_fraction_matches_the_reference(qla, stream, H, W, m, first, channels):
    """qla_fno_band_fraction against the FP64 DFT definition on the same BF16 inputs:
    the kept-mode energy goes through BF16-stored partial transforms (relative error a
    few 2^-9 on the kept part), so the fractions agree to 1e-2."""
    cin = 4
    bits = _band_inputs(H, W, cin, m, seed=H + first)
    B = bits.shape[0]
    h = qla.qla_fno_create(H, W, cin, 3, 8, m, 1, 8, B, 0, stream.cuda_stream)
    try:
        frac = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
        qla.qla_fno_band_fraction(h, to_device(bits), B, first, channels, frac)
        got = frac.cpu().numpy()
    finally:
        qla.qla_fno_destroy(h)
    want = fno.band_fraction(m, bf16_value(bits)[:, first:first + channels])
    print("band fractions", np.round(got, 4), np.round(want, 4))
    assert np.abs(got - want).max() <= 1e-2
    assert got[-1] == 0.0                       # zero sample
    assert want.min() < 0.05 and want.max() > 0.95  # the cases span the range


def test_band_fraction_rejects_bad_channels(qla, stream):
    h = qla.qla_fno_create(40, 24, 4, 3, 8, 5, 1, 8, 2, 0, stream.cuda_stream)
    try:
        x = torch.zeros((2, 4, 40, 24), dtype=torch.int16, device="cuda")
        f = torch.zeros(2, dtype=torch.float64, device="cuda")
        for first, ch, b in [(-1, 3, 2), (1, 4, 2), (0, 9, 2), (1, 0, 2), (1, 3, 3)]:
            with pytest.raises(qla.QlaError):
                qla.qla_fno_band_fraction(h, x, b, first, ch, f)
    finally:
        qla.qla_fno_destroy(h)
