"""The seeded input generators: determinism, ranges and record-length sanity."""
import numpy as np

import synth


def test_inputs_are_seeded_and_deterministic():
    a = synth.make_inputs(synth.TINY, seed=3)
    b = synth.make_inputs(synth.TINY, seed=3)
    np.testing.assert_array_equal(a.S, b.S)
    np.testing.assert_array_equal(a.sos_true, b.sos_true)
    c = synth.make_inputs(synth.TINY, seed=4)
    assert not np.array_equal(a.S, c.S)


def test_paper_scale_phantom_ranges():
    inp = synth.make_inputs(synth.PAPER, with_channels=False)
    assert inp.sos_true.shape == (140, 140)
    assert 1.480 - 1e-12 <= inp.sos_true.min() and inp.sos_true.max() <= 1.600 + 1e-12
    assert inp.mask.sum() > 0 and inp.mask.dtype == np.uint8
    assert len(inp.delays) == 11 and synth.PAPER.n_patches == 169
    assert synth.TINY.n_patches == 49 and synth.TINY.M == 5


def test_record_reaches_the_farthest_pixel():
    for s in (synth.TINY, synth.PAPER):
        far = s.radius + np.hypot(s.nx * s.px / 2, s.ny * s.px / 2) + max(abs(d) for d in s.delays)
        assert far / s.v0 * s.fs < s.n_t - 1


def test_travel_time_uniform_is_distance_over_v0():
    scan = synth.TINY.with_(phantom="uniform")
    ph = synth.make_sos_phantom(scan, np.random.default_rng(0))
    T = synth.travel_times(scan, ph, [1.0], [2.0])
    phi = 2 * np.pi * np.arange(scan.n_elem) / scan.n_elem
    dist = np.hypot(scan.radius * np.cos(phi) - 1.0, scan.radius * np.sin(phi) - 2.0)
    np.testing.assert_allclose(T[0], dist / scan.v0, rtol=1e-14)
