"""Checks of the seeded input generator (host side; no method arithmetic here)."""
import numpy as np

from paper_2405_04253_amd import synth


def test_numpy_generator_shapes_ranges_determinism():
    a = synth.gen_channel(1000, 75.0, 22.0, seed=5)
    b = synth.gen_channel(1000, 75.0, 22.0, seed=5)
    assert a.samples.shape == (2000, 4) and a.samples.dtype == np.int8
    assert a.samples.min() >= -16 and a.samples.max() <= 15
    assert np.array_equal(a.samples, b.samples) and np.array_equal(a.taps, b.taps)
    assert a.taps.shape == (32, 2) and a.taps.min() >= -32 and a.taps.max() <= 31
    assert 2.5 < a.samples.astype(float).std() < 5.5


def test_tap_count_follows_fibre_length():
    assert synth.cdc_tap_count(10.0) == 8
    assert synth.cdc_tap_count(75.0) == 32
    assert synth.cdc_tap_count(80.0) == 32
    taps, shift, gain = synth.design_cdc_taps(20.0)
    assert taps.shape[0] == synth.cdc_tap_count(20.0) and shift >= 0 and gain > 1


def test_batched_specs_distributions():
    specs = synth.batched_specs(400, 12, 20, tag="t")
    n = np.array([s.nsym for s in specs])
    km = np.array([s.fibre_km for s in specs])
    assert n.min() >= 2 ** 12 * 0.99 and n.max() <= 2 ** 20 * 1.01
    assert 10 <= km.min() and km.max() <= 80
    # log-uniform: about half the channels below the geometric midpoint 2^16
    assert 0.35 < np.mean(n < 2 ** 16) < 0.65


def test_torch_generator_on_cpu():
    import torch
    q, taps, shift, unit = synth.gen_channel_torch(3000, 40.0, 20.0, seed=9, device="cpu")
    q2, *_ = synth.gen_channel_torch(3000, 40.0, 20.0, seed=9, device="cpu")
    assert q.shape == (6000, 4) and q.dtype == torch.int8
    assert int(q.min()) >= -16 and int(q.max()) <= 15
    assert torch.equal(q, q2)
    ref_taps, ref_shift, _ = synth.design_cdc_taps(40.0)
    assert np.array_equal(taps, ref_taps) and shift == ref_shift and unit >= 1
