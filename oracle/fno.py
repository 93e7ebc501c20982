"""FP64 CPU reference of the Fourier neural operator surrogate (test infrastructure).

Only the test suite and the benchmark's checks use this module; it shares no code
with the GPU library. It is the plain definition of the network, written with
torch's CPU float64 operations: `torch.fft.rfft2` / `torch.fft.irfft2` for the
transforms (the retained modes are cut out of the full half spectrum and put back
into a zero spectrum), `einsum` for the channel contractions and the exact GELU,
x * Phi(x). Gradients come from torch's autograd on this float64 graph.

Network (sizes from a `Spec`):
    v0 = P u + p
    v_{l+1} = act(irfft2(R_l . rfft2(v_l)[kept]) + W_l v_l + b_l),  act = GELU except
              after the last layer
    out = Q2 GELU(Q1 v_L + q1) + q2
kept modes: ky in [0, m) U [H - m, H) (rows of the 2D spectrum), kx in [0, m) (the
half-spectrum axis). Loss: the mean over the batch of ||out_b - t_b|| / ||t_b||.

The flat parameter vector has the layout of the GPU library:
    P [C][Cin], p [C]; per layer W [C][C], b [C], R [2m][m][C_in][C_out][re, im];
    Q1 [C2][C], q1 [C2], Q2 [Cout][C2], q2 [Cout].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch


@dataclasses.dataclass(frozen=True)
class Spec:
    H: int
    W: int
    cin: int
    cout: int
    C: int
    m: int
    L: int
    C2: int


def param_shapes(s: Spec):
    """(name, shape) in the order of the flat vector."""
    out = [("P", (s.C, s.cin)), ("p", (s.C,))]
    for l in range(s.L):
        out += [(f"W{l}", (s.C, s.C)), (f"b{l}", (s.C,)), (f"R{l}", (2 * s.m, s.m, s.C, s.C, 2))]
    out += [("Q1", (s.C2, s.C)), ("q1", (s.C2,)), ("Q2", (s.cout, s.C2)), ("q2", (s.cout,))]
    return out


def param_count(s: Spec) -> int:
    return sum(int(np.prod(shape)) for _, shape in param_shapes(s))


def unflatten(s: Spec, flat):
    """Dict of named tensors viewing `flat` (a float64 torch tensor)."""
    out, off = {}, 0
    for name, shape in param_shapes(s):
        n = int(np.prod(shape))
        out[name] = flat[off:off + n].reshape(shape)
        off += n
    return out


def gelu(x):
    """Exact GELU: x times the standard normal CDF."""
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def kept_rows(s: Spec):
    return list(range(s.m)) + list(range(s.H - s.m, s.H))


def spectral_conv(s: Spec, v, R):
    """irfft2 of the retained modes of rfft2(v), mixed over channels by the complex R."""
    X = torch.fft.rfft2(v)                               # [B, C, H, W/2 + 1]
    rows = kept_rows(s)
    Xk = X[:, :, rows, :s.m]                             # [B, C, 2m, m]
    Rc = torch.complex(R[..., 0], R[..., 1])             # [2m, m, Cin, Cout]
    Y = torch.einsum("bcyx,yxco->boyx", Xk, Rc)
    out_ft = torch.zeros(v.shape[0], s.C, s.H, s.W // 2 + 1, dtype=X.dtype)
    out_ft[:, :, rows, :s.m] = Y
    return torch.fft.irfft2(out_ft, s=(s.H, s.W))


def forward(s: Spec, flat, u):
    """u: float64 [B, Cin, H, W] -> float64 [B, Cout, H, W]."""
    p = unflatten(s, flat)
    v = torch.einsum("oc,bchw->bohw", p["P"], u) + p["p"][None, :, None, None]
    for l in range(s.L):
        z = spectral_conv(s, v, p[f"R{l}"]) + torch.einsum("oc,bchw->bohw", p[f"W{l}"], v) \
            + p[f"b{l}"][None, :, None, None]
        v = gelu(z) if l + 1 < s.L else z
    h = gelu(torch.einsum("oc,bchw->bohw", p["Q1"], v) + p["q1"][None, :, None, None])
    return torch.einsum("oc,bchw->bohw", p["Q2"], h) + p["q2"][None, :, None, None]


def rel_l2_loss(out, target):
    B = out.shape[0]
    d = (out - target).reshape(B, -1).norm(dim=1)
    t = target.reshape(B, -1).norm(dim=1)
    return (d / t).mean()


def loss_and_grad(s: Spec, params: np.ndarray, u: np.ndarray, target: np.ndarray):
    """Loss (float) and its gradient (float64 numpy, flat layout) at `params`."""
    flat = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    out = forward(s, flat, torch.tensor(np.asarray(u, dtype=np.float64)))
    loss = rel_l2_loss(out, torch.tensor(np.asarray(target, dtype=np.float64)))
    loss.backward()
    return float(loss.detach()), flat.grad.detach().numpy().copy()


def loss_value(s: Spec, params: np.ndarray, u: np.ndarray, target: np.ndarray) -> float:
    with torch.no_grad():
        out = forward(s, torch.tensor(np.asarray(params, dtype=np.float64)),
                      torch.tensor(np.asarray(u, dtype=np.float64)))
        return float(rel_l2_loss(out, torch.tensor(np.asarray(target, dtype=np.float64))))


def predict(s: Spec, params: np.ndarray, u: np.ndarray) -> np.ndarray:
    with torch.no_grad():
        return forward(s, torch.tensor(np.asarray(params, dtype=np.float64)),
                       torch.tensor(np.asarray(u, dtype=np.float64))).numpy()


def adam(params, grad, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba, Algorithm 1); returns new arrays."""
    m1 = b1 * m1 + (1 - b1) * grad
    m2 = b2 * m2 + (1 - b2) * grad * grad
    mh = m1 / (1 - b1 ** t)
    vh = m2 / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2


def kept_mask(H: int, W: int, m: int) -> np.ndarray:
    """Boolean [H, W] mask of the full 2D spectrum that the truncation touches: the
    kept half-spectrum modes (ky in [0, m) U [H - m, H), kx in [0, m)) and, for
    kx > 0, their Hermitian partners (-ky, -kx), which a real field carries with the
    same magnitude."""
    mask = np.zeros((H, W), dtype=bool)
    for ky in kept_rows(Spec(H, W, 1, 1, 1, m, 1, 1)):
        for kx in range(m):
            mask[ky, kx] = True
            if kx > 0:
                mask[(-ky) % H, (-kx) % W] = True
    return mask


def band_fraction(m: int, u) -> np.ndarray:
    """Share of each sample's energy sum(u^2) (u: [B, c, H, W]) held by the modes the
    network's spectral branch keeps: by Parseval, sum over the masked modes of the
    full 2D DFT of |U|^2 / (H W), over sum u^2 (0 for a zero sample). A sample whose
    energy lies mostly outside these modes cannot be carried by the Fourier layers."""
    u = np.asarray(u, dtype=np.float64)
    B, _, H, W = u.shape
    X = np.fft.fft2(u)
    mask = kept_mask(H, W, m)
    kept = (np.abs(X) ** 2 * mask).reshape(B, -1).sum(axis=1) / (H * W)
    total = (u ** 2).reshape(B, -1).sum(axis=1)
    return np.where(total > 0, kept / np.where(total > 0, total, 1.0), 0.0)
