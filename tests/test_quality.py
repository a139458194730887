"""Receiver-quality tooling: the SER alignment and counting (pinned on
constructed cases), the float reference receiver, and the SER of the library's
integer path on a high-OSNR channel (GPU)."""
import numpy as np
import pytest

from paper_2405_04253_amd import quality as Q
from paper_2405_04253_amd import synth


def _symbols(n, seed):
    r = np.random.default_rng(seed)
    return (r.integers(0, 4, size=(n, 4)) * 2 - 3).astype(np.int8)


def test_alignment_recovers_swap_conjugation_delay_and_gain():
    sym = _symbols(4096, 1)
    s = Q.tx_complex(sym)
    y = np.zeros_like(s)
    # output 0 = conj(Y pol) delayed by 5, output 1 = X pol delayed by -3, rotated and scaled
    y[0] = 0.7 * np.exp(0.3j) * np.roll(np.conj(s[1]), 5)
    y[1] = 2.5 * np.exp(-1.1j) * np.roll(s[0], -3)
    r = Q.align_and_count(y, sym)
    assert r["ser"] == 0.0
    assert r["alignment"][0] == dict(out=0, tx=1, conj=True, delay=5)
    assert r["alignment"][1] == dict(out=1, tx=0, conj=False, delay=-3)


def test_counting_of_planted_errors():
    sym = _symbols(4096, 2)
    y = Q.tx_complex(sym).copy()
    m = y.shape[1]
    lo, hi = m // 2, m - 48
    bad = [lo + 3, lo + 100, hi - 1]
    for i in bad:
        y[0, i] += 2.0                      # moves the I component to the next level
    r = Q.align_and_count(y, sym)
    assert r["errors"] == len(bad)
    assert r["symbols"] == 2 * (hi - lo)


def test_bit_errors_follow_the_gray_map():
    # hand-written Gray table of the levels per dimension, and the planted decisions
    gray = {-3: (0, 0), -1: (0, 1), 1: (1, 1), 3: (1, 0)}
    sym = _symbols(4096, 4)
    y = Q.tx_complex(sym).copy()
    m = y.shape[1]
    lo = m // 2
    plant = {lo + 1: 3 + 3j, lo + 7: -3 - 1j, lo + 50: 1 - 1j, lo + 90: -1 + 3j}
    want_bits = want_syms = 0
    for i, v in plant.items():
        ref = complex(y[0, i])
        for a, b in ((ref.real, v.real), (ref.imag, v.imag)):
            want_bits += sum(x != z for x, z in zip(gray[int(a)], gray[int(b)]))
        want_syms += v != ref
        y[0, i] = v
    r = Q.align_and_count(y, sym)
    assert r["errors"] == want_syms
    assert r["bit_errors"] == want_bits
    assert r["ber"] == pytest.approx(want_bits / (4 * r["symbols"]))


def test_carrier_recovery_tracks_a_phase_walk():
    sym = _symbols(8192, 5)
    s = Q.tx_complex(sym)
    rng = np.random.default_rng(6)
    walk = np.cumsum(rng.standard_normal(s.shape) * 0.02, axis=1) + np.array([[0.5], [-2.0]])
    y = s * np.exp(1j * walk) + 0.05 * (rng.standard_normal(s.shape) + 1j * rng.standard_normal(s.shape))
    assert Q.align_and_count(y, sym)["ser"] > 0.1
    assert Q.align_and_count(Q.cpe_4th_power(y), sym)["ser"] == 0.0


def test_linewidth_changes_only_the_received_phase():
    a = synth.gen_channel(4096, 40.0, 24.0, 9)
    b = synth.gen_channel(4096, 40.0, 24.0, 9, linewidth_hz=1e6)
    assert np.array_equal(a.symbols, b.symbols) and np.array_equal(a.taps, b.taps)
    assert a.requant_shift == b.requant_shift
    assert not np.array_equal(a.samples, b.samples)
    pa = (a.samples.astype(np.float64) ** 2).sum()
    pb = (b.samples.astype(np.float64) ** 2).sum()
    assert abs(pa / pb - 1) < 0.02


def test_required_osnr_interpolation():
    assert Q.required_osnr([10, 12, 14], [1e-1, 1e-2, 1e-3], 1e-2) == pytest.approx(12.0)
    assert Q.required_osnr([10, 12], [1e-1, 1e-3], 1e-2) == pytest.approx(11.0)
    assert Q.required_osnr([10, 12], [1e-3, 1e-4], 1e-2) is None


def test_float_reference_receiver_high_osnr():
    nsym = 1 << 15
    ch = synth.gen_channel(nsym, 75.0, 30.0, 7, keep_float=True)
    r = Q.align_and_count(Q.float_receiver(ch.float_rx, 75.0, nsym, mu=2e-5, cma_blocks=256), ch.symbols)
    assert r["ser"] < 1e-3


@pytest.mark.gpu
def test_fnt_receiver_converges():
    """The integer receiver separates the polarisations and equalises within 2^16
    symbols: with the default RDE step (err_shift 16, mu_shift 4) its SER at
    OSNR 26 dB is ~1e-2 (the oracle gives 8.5e-3 on this channel), against ~0.75
    for an unconverged equaliser."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ch = synth.gen_channel(1 << 16, 75.0, 26.0, 11)
    r = Q.align_and_count(Q.fnt_receiver(ch), ch.symbols)
    print(f"[case] FNT receiver SER at OSNR 26 dB: {r['ser']:.2e} {r['alignment']}", flush=True)
    assert r["ser"] < 0.03
    assert {a["tx"] for a in r["alignment"]} == {0, 1}


@pytest.mark.gpu
def test_fnt_receiver_with_phase_noise_and_carrier_recovery():
    """With 100 kHz of laser linewidth the phase-blind RDE equaliser still
    converges, and the blind carrier recovery after it restores the SER."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ch = synth.gen_channel(1 << 16, 75.0, 26.0, 11, linewidth_hz=1e5)
    r = Q.align_and_count(Q.cpe_4th_power(Q.fnt_receiver(ch)), ch.symbols)
    print(f"[case] FNT receiver + carrier recovery, 100 kHz, OSNR 26 dB: SER {r['ser']:.2e} "
          f"BER {r['ber']:.2e}", flush=True)
    assert r["ser"] < 0.05
