"""The seeded input generators: the batched torch index maps equal the numpy ones."""
import numpy as np

import workloads


def test_batched_index_maps_equal_the_single_ones():
    inst = workloads.sample_instances(8, seed=3, fixed_side=96)
    got = workloads.ellipse_index_batch(96, 96, [i.ellipse for i in inst]).numpy()
    for k, i in enumerate(inst):
        np.testing.assert_allclose(got[k], workloads.ellipse_index(96, 96, i.ellipse),
                                   rtol=0, atol=1e-14)


def test_instances_follow_the_stated_ranges():
    inst = workloads.sample_instances(200, seed=1, fixed_side=512)
    for i in inst:
        e = i.ellipse
        assert i.n_side == 512 and i.steps == 4 * 512
        assert 0.05 * 512 <= e.a <= 0.25 * 512 and 0.05 * 512 <= e.b <= 0.25 * 512
        assert 8.0 <= i.packet.lam <= 32.0
        assert {e.n_in, e.n_out} & {1.0} and 1.5 <= max(e.n_in, e.n_out) <= 3.0
    bubbles = sum(i.ellipse.n_in == 1.0 for i in inst)
    assert 60 <= bubbles <= 140
