"""Seeded input generators: determinism, shapes and value ranges."""
import math

import numpy as np

import synth


def test_generators_are_deterministic():
    a, b = synth.field_c2(3, 64, 48), synth.field_c2(3, 64, 48)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.w, b.w)
    c = synth.field_c2(4, 64, 48)
    assert not np.array_equal(a.X, c.X)


def test_observed_phase_range_and_congruence():
    f = synth.field_c3(0, 64, 64)
    assert np.all(f.X > -math.pi - 1e-15) and np.all(f.X <= math.pi + 1e-15)
    k = (f.phi - f.X) / (2 * math.pi)
    assert np.allclose(k, np.round(k), atol=1e-9)


def test_weights_and_shapes():
    f = synth.field_c2(0, 96, 80)
    assert f.X.shape == (96, 80) and f.w.shape == (96, 80)
    assert np.all(f.w > 0) and np.all(f.w < 1)
    assert np.any(f.w == 0.05)  # the decorrelated band
    g = synth.field_c5(1, 20, 17)
    assert g.Cv.shape == (19, 17) and g.Ch.shape == (20, 16)
    assert np.all((g.Cv > 0) & (g.Cv < 1))
    s = synth.tile_shapes_c4(0)
    assert s.shape == (64, 2) and s.min() >= 512 and s.max() <= 3072
    assert np.array_equal(s, synth.tile_shapes_c4(0))


def test_c5_truth_is_the_noise_free_phase():
    f = synth.field_c5(3, 64, 48)
    t = synth.field_c5_truth(3, 64, 48)
    d = f.phi - t
    # the difference is the N(0, 0.3^2) noise: no structure, the right spread
    assert abs(d.std() - 0.3) < 0.02 and abs(d.mean()) < 0.03
