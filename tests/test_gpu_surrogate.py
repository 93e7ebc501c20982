"""What the trained surrogate gains over QLA alone (the surrogate workflow end to end).

Instances of the batched scattering family on a 512^2 grid, 1024 QLA steps, with
packet wavelengths 64-128 cells (inside the network's 12 kept modes): QLA generates
the training pairs, the network trains on the GPU, and the held-out lattices go
through the surrogate, the energy check (|E/E0 - 1| < 1e-2) and the QLA fallback.
The untrained network must have every prediction rejected (so its path is slower
than QLA alone), the trained one must have accepted predictions with small field
error, and its path must beat QLA alone in lattices per second. The band gate (inputs
with little energy in the kept modes skip the network) must pass every one of these
in-band packets and leave the results unchanged, and must send short-wavelength
packets (8-32 cells, beyond the kept modes) straight to QLA.
"""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

SIDE, STEPS = 512, 1024


@pytest.fixture(scope="module")
def stream():
    prev = torch.cuda.current_stream()
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    yield st
    torch.cuda.synchronize()
    torch.cuda.set_stream(prev)


def _family(count, seed):
    return workloads.sample_instances(count, seed=seed, fixed_side=SIDE, lam_min=64.0,
                                      lam_max=128.0, steps=STEPS)


def test_trained_surrogate_beats_plain_qla_at_the_acceptance_tolerance(stream):
    from paper_2604_21128_amd import qla, surrogate as S
    qla.load()
    train_i, test_i = _family(4000, 20), _family(256, 21)

    def index_fn(insts):
        return lambda c0, k: workloads.ellipse_index_batch(
            SIDE, SIDE, [i.ellipse for i in insts[c0:c0 + k]], device="cuda")

    def packets(insts):
        return [S.PacketSpec(i.packet.x0, i.packet.y0, i.packet.sigma, i.packet.lam)
                for i in insts]
    d = workloads.DELTA
    train = S.qla_pairs(index_fn(train_i), len(train_i), packets(train_i), d, STEPS)
    test = S.qla_pairs(index_fn(test_i), len(test_i), packets(test_i), d, STEPS, keep_f32=True)
    with S.Surrogate(SIDE, SIDE, max_batch=16, seed=3) as sur:
        _, e_untrained = S.predict_all(sur, test.inputs, 16)
        assert not bool(S.accept(e_untrained, test.e0).any())
        hist = S.train(sur, train.inputs, train.targets, 16, 6.0, 1e-3, log=print)
        assert np.mean(hist["losses"][-50:]) < 0.5 * np.mean(hist["losses"][:50])
        out, ok, t = S.run_with_fallback(sur, test.inputs, test.e0, index_fn(test_i),
                                         packets(test_i), d, STEPS, 16)
        # these packets lie inside the kept modes: the band gate lets every one through
        # and changes nothing
        frac = S.band_fractions(sur, test.inputs, 16).cpu().numpy()
        out_g, ok_g, t_g = S.run_with_fallback(sur, test.inputs, test.e0, index_fn(test_i),
                                               packets(test_i), d, STEPS, 16, band_min=0.5)
    assert frac.min() >= 0.5 and t_g["gated_out"] == 0
    assert torch.equal(ok_g, ok) and torch.equal(out_g, out)
    ok = ok.cpu().numpy()
    err = ((out - test.targets_f32).flatten(1).norm(dim=1)
           / test.targets_f32.flatten(1).norm(dim=1)).cpu().numpy()
    gain = test.qla_seconds / (t["surrogate_s"] + t["fallback_qla_s"])
    print(f"accepted {ok.sum()}/{ok.size}, accepted field rel L2 median "
          f"{np.median(err[ok]) if ok.any() else float('nan'):.3f}, gain {gain:.2f}x")
    # rejected lattices were advanced by QLA itself: their fields are QLA's
    assert float(err[~ok].max(initial=0.0)) < 1e-6
    assert ok.mean() >= 0.3
    assert np.median(err[ok]) < 0.12
    assert gain > 1.0


def test_band_gate_sends_short_wavelength_packets_to_qla(stream):
    """Packets of 8-32 cells put their carrier at 16-64 cycles per 512 cells, beyond the
    12 kept modes: their band fractions stay far below 1/2 while 64-128-cell packets sit
    above it (the fraction depends on the inputs only, so an untrained network does).
    On a mix of both, the gate sends the short ones straight to QLA and predicts the
    rest; every lattice that is not accepted ends with QLA's own fields."""
    from paper_2604_21128_amd import qla, surrogate as S
    qla.load()
    n_short = 40
    insts = (workloads.sample_instances(n_short, seed=31, fixed_side=SIDE, steps=STEPS)
             + _family(40, 32))

    def index_fn(c0, k):
        return workloads.ellipse_index_batch(SIDE, SIDE, [i.ellipse for i in insts[c0:c0 + k]],
                                             device="cuda")
    packets = [S.PacketSpec(i.packet.x0, i.packet.y0, i.packet.sigma, i.packet.lam)
               for i in insts]
    d = workloads.DELTA
    pairs = S.qla_pairs(index_fn, len(insts), packets, d, STEPS, keep_f32=True)
    with S.Surrogate(SIDE, SIDE, max_batch=16, seed=1) as sur:
        frac = S.band_fractions(sur, pairs.inputs, 16).cpu().numpy()
        out, ok, t = S.run_with_fallback(sur, pairs.inputs, pairs.e0, index_fn, packets, d,
                                         STEPS, 16, band_min=0.5)
    print(f"band fractions: short max {frac[:n_short].max():.3f}, "
          f"long min {frac[n_short:].min():.3f}; gated out {t['gated_out']}")
    assert frac[:n_short].max() < 0.5 <= frac[n_short:].min()
    assert t["gated_out"] == n_short
    ok = ok.cpu().numpy()
    assert not ok[:n_short].any()
    err = ((out - pairs.targets_f32).flatten(1).norm(dim=1)
           / pairs.targets_f32.flatten(1).norm(dim=1)).cpu().numpy()
    assert float(err[~ok].max(initial=0.0)) < 1e-6
