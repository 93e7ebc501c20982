"""Pins of the FP64 CPU neural-operator reference (oracle/fno.py) against closed forms.

The spectral convolution is checked on single Fourier modes, where the kept-mode
product reduces to a complex scalar multiplication with a known answer, and on
band-limited fields, where keeping every mode with the identity mixing must return
the input. The network is checked for the symmetries it must have (periodic
translation equivariance; pixel-wise action when the spectral weights vanish), the
GELU at tabulated points of the normal CDF, the loss on a scaled target, the
gradient against central finite differences of the loss, and the first Adam step
against its closed form.
"""
import math

import numpy as np
import pytest
import torch

from oracle import fno

SMALL = fno.Spec(H=16, W=12, cin=3, cout=2, C=4, m=3, L=2, C2=6)


def _params(s, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, fno.param_count(s))


def _plane_wave(H, W, ky, kx, phase=0.0):
    y, x = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return np.cos(2 * np.pi * (kx * x / W + ky * y / H) + phase)


def _R(s, re, im):
    R = torch.zeros(2 * s.m, s.m, s.C, s.C, 2, dtype=torch.float64)
    for c in range(s.C):
        R[:, :, c, c, 0] = re
        R[:, :, c, c, 1] = im
    return R


@pytest.mark.parametrize("ky,kx", [(2, 1), (15, 2), (0, 2), (14, 1)])
def test_single_mode_is_multiplied_by_the_complex_weight(ky, kx):
    # for kx > 0: Re[(a + ib) e^{i theta}] = a cos(theta) - b sin(theta)
    s = fno.Spec(H=16, W=12, cin=1, cout=1, C=1, m=3, L=1, C2=1)
    a, b = 0.7, -1.3
    v = torch.tensor(_plane_wave(16, 12, ky, kx, 0.4))[None, None]
    got = fno.spectral_conv(s, v, _R(s, a, b)).numpy()[0, 0]
    # cos(theta + pi/2) = -sin(theta)
    want = a * _plane_wave(16, 12, ky, kx, 0.4) + b * _plane_wave(16, 12, ky, kx, 0.4 + np.pi / 2)
    np.testing.assert_allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("ky", [1, 2, 14])
def test_kx_zero_keeps_only_the_real_part_of_the_weight(ky):
    # at kx = 0 the inverse real transform keeps the real part of each column, so a
    # real field cos(2 pi ky y / H) picks up only Re(R)
    s = fno.Spec(H=16, W=12, cin=1, cout=1, C=1, m=3, L=1, C2=1)
    v = torch.tensor(_plane_wave(16, 12, ky, 0, 0.3))[None, None]
    got = fno.spectral_conv(s, v, _R(s, 0.7, -1.3)).numpy()[0, 0]
    np.testing.assert_allclose(got, 0.7 * _plane_wave(16, 12, ky, 0, 0.3), atol=1e-12)


@pytest.mark.parametrize("ky,kx", [(3, 1), (12, 0), (0, 3), (8, 5), (5, 4)])
def test_modes_outside_the_kept_set_are_removed(ky, kx):
    s = fno.Spec(H=16, W=12, cin=1, cout=1, C=1, m=3, L=1, C2=1)
    v = torch.tensor(_plane_wave(16, 12, ky, kx, 0.2))[None, None]
    got = fno.spectral_conv(s, v, _R(s, 1.0, 0.0)).numpy()
    np.testing.assert_allclose(got, 0.0, atol=1e-12)


def test_identity_mixing_with_every_mode_kept_returns_a_band_limited_field():
    # H = 2m keeps every row; kx < m = W/2 keeps every column but the x-Nyquist one
    s = fno.Spec(H=8, W=8, cin=1, cout=1, C=2, m=4, L=1, C2=1)
    rng = np.random.default_rng(3)
    v = np.zeros((1, 2, 8, 8))
    for c in range(2):
        for ky in range(8):
            for kx in range(4):
                v[0, c] += rng.normal() * _plane_wave(8, 8, ky, kx, rng.uniform(0, 2 * np.pi))
    got = fno.spectral_conv(s, torch.tensor(v), _R(s, 1.0, 0.0)).numpy()
    np.testing.assert_allclose(got, v, atol=1e-12)


def test_channels_are_mixed_by_the_c_in_to_c_out_matrix():
    s = fno.Spec(H=16, W=12, cin=1, cout=1, C=2, m=3, L=1, C2=1)
    R = torch.zeros(6, 3, 2, 2, 2, dtype=torch.float64)
    R[..., 0, 1, 0] = 2.0       # in channel 0 -> out channel 1, real weight 2
    R[..., 1, 0, 1] = 1.0       # in channel 1 -> out channel 0, weight i
    w0, w1 = _plane_wave(16, 12, 1, 2), _plane_wave(16, 12, 2, 1)
    v = torch.tensor(np.stack([w0, w1]))[None]
    got = fno.spectral_conv(s, v, R).numpy()[0]
    np.testing.assert_allclose(got[1], 2 * w0, atol=1e-12)
    np.testing.assert_allclose(got[0], _plane_wave(16, 12, 2, 1, np.pi / 2), atol=1e-12)  # Re(i e^{it})


def test_gelu_is_x_times_the_normal_cdf():
    x = torch.tensor([0.0, 1.0, -1.0, 2.0, -3.0], dtype=torch.float64)
    phi = np.array([0.5, 0.8413447460685429, 0.15865525393145707, 0.9772498680518208,
                    0.0013498980316301035])
    np.testing.assert_allclose(fno.gelu(x).numpy(), x.numpy() * phi, rtol=1e-14, atol=1e-16)


def test_network_commutes_with_periodic_translation():
    s = SMALL
    p = _params(s, 1)
    u = np.random.default_rng(2).normal(size=(2, s.cin, s.H, s.W))
    a = fno.predict(s, p, np.roll(u, (3, -5), axis=(2, 3)))
    b = np.roll(fno.predict(s, p, u), (3, -5), axis=(2, 3))
    np.testing.assert_allclose(a, b, atol=1e-11)


def test_without_spectral_weights_the_network_acts_pixel_by_pixel():
    s = SMALL
    p = _params(s, 4)
    view = fno.unflatten(s, torch.from_numpy(p))
    for l in range(s.L):
        view[f"R{l}"].zero_()                # writes through the view into p
    u = np.random.default_rng(5).normal(size=(1, s.cin, s.H, s.W))
    perm = np.random.default_rng(6).permutation(s.H * s.W)
    up = u.reshape(1, s.cin, -1)[:, :, perm].reshape(u.shape)
    a = fno.predict(s, p, up).reshape(1, s.cout, -1)
    b = fno.predict(s, p, u).reshape(1, s.cout, -1)[:, :, perm]
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_relative_l2_loss_of_a_scaled_target():
    t = torch.tensor(np.random.default_rng(7).normal(size=(3, 2, 4, 5)))
    scale = torch.tensor([2.0, 0.5, -1.0], dtype=torch.float64)[:, None, None, None]
    assert abs(float(fno.rel_l2_loss(scale * t, t)) - (1.0 + 0.5 + 2.0) / 3) < 1e-14


def test_gradient_matches_central_differences():
    s = SMALL
    p = _params(s, 8)
    rng = np.random.default_rng(9)
    u = rng.normal(size=(2, s.cin, s.H, s.W))
    t = rng.normal(size=(2, s.cout, s.H, s.W))
    _, g = fno.loss_and_grad(s, p, u, t)
    for trial in range(3):
        d = rng.normal(size=p.size)
        eps = 1e-5
        fd = (fno.loss_value(s, p + eps * d, u, t) - fno.loss_value(s, p - eps * d, u, t)) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-7 * max(1.0, abs(fd)), (trial, fd, g @ d)
    # and single coordinates in every parameter block
    off = 0
    for name, shape in fno.param_shapes(s):
        i = off + int(rng.integers(int(np.prod(shape))))
        off += int(np.prod(shape))
        e = np.zeros_like(p)
        e[i] = 1e-5
        fd = (fno.loss_value(s, p + e, u, t) - fno.loss_value(s, p - e, u, t)) / 2e-5
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), name


def test_first_adam_step_moves_each_weight_by_lr_against_its_gradient_sign():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m1, m2 = fno.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert math.isclose(m1[1], -0.2) and math.isclose(m2[1], 0.004)


# The band fraction: the share of a field's energy in the modes the spectral branch keeps.
@pytest.mark.parametrize("ky,kx,expect", [
    (0, 0, 1.0),            # constant
    (2, 0, 1.0),            # kept row, kx = 0
    (16 - 3, 2, 1.0),       # negative ky with positive kx: kept
    (3, 2, 0.0),            # ky = m is not kept for kx > 0 (its partner is ky = H - m, kx < 0)
    (0, 3, 0.0),            # kx = m
    (5, 1, 0.0),            # ky beyond the kept rows
    (3, 0, 0.5),            # kx = 0 keeps ky = H - m but not ky = m: half the energy of a cosine
])
def test_band_fraction_of_single_plane_waves(ky, kx, expect):
    H, W, m = 16, 12, 3
    u = _plane_wave(H, W, ky, kx, phase=0.4)[None, None]
    assert fno.band_fraction(m, u)[0] == pytest.approx(expect, abs=1e-12)


def test_band_fraction_of_a_mix_is_the_kept_share_of_the_energy():
    H, W, m = 16, 12, 3
    # equal-energy cosines (no mode at kx = 0 or the Nyquist lines): amplitudes set the shares
    inside, outside = _plane_wave(H, W, 1, 1), _plane_wave(H, W, 4, 5, 1.0)
    u = np.stack([(2.0 * inside + 1.0 * outside)[None], (0.5 * inside)[None],
                  np.zeros((1, H, W))])
    f = fno.band_fraction(m, u)
    assert f[0] == pytest.approx(4.0 / 5.0, abs=1e-12)
    assert f[1] == pytest.approx(1.0, abs=1e-12)
    assert f[2] == 0.0


def test_band_fraction_of_a_field_the_truncation_keeps_whole_is_one():
    """A field built from kept half-spectrum modes only (Hermitian completion, kx = 0
    column real and symmetric) survives rfft2 -> keep -> irfft2 unchanged and its band
    fraction is 1; adding a real field with no content on the mask or its mirror image
    lowers it by that field's energy share."""
    H, W, m = 16, 12, 3
    s = fno.Spec(H=H, W=W, cin=1, cout=1, C=1, m=m, L=1, C2=1)
    rng = np.random.default_rng(5)
    X = np.zeros((H, W // 2 + 1), dtype=complex)
    for ky in fno.kept_rows(s):
        for kx in range(1, m):
            X[ky, kx] = rng.normal() + 1j * rng.normal()
    for ky in range(1, m):          # kx = 0: rows ky and -ky both kept, conjugate pair
        X[ky, 0] = rng.normal() + 1j * rng.normal()
        X[H - ky, 0] = np.conj(X[ky, 0])
    X[0, 0] = rng.normal()
    u = np.fft.irfft2(X, s=(H, W))
    assert fno.band_fraction(m, u[None, None])[0] == pytest.approx(1.0, abs=1e-12)
    mask = fno.kept_mask(H, W, m)
    mirror = np.roll(mask[::-1, ::-1], (1, 1), axis=(0, 1))   # mirror[k] = mask[-k]
    v = np.real(np.fft.ifft2(np.where(mask | mirror, 0.0, np.fft.fft2(rng.normal(size=(H, W))))))
    e_u, e_v = (u ** 2).sum(), (v ** 2).sum()
    got = fno.band_fraction(m, (u + v)[None, None])[0]
    assert got == pytest.approx(e_u / (e_u + e_v), abs=1e-12)
