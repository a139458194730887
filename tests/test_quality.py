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
    """The integer receiver separates the polarisations and equalises: with the
    default (fast, coarse) RDE step its SER floor at OSNR 26 dB is ~2e-2, against
    ~0.75 for an unconverged equaliser."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ch = synth.gen_channel(1 << 16, 75.0, 26.0, 11)
    r = Q.align_and_count(Q.fnt_receiver(ch), ch.symbols)
    print(f"[case] FNT receiver SER at OSNR 26 dB: {r['ser']:.2e} {r['alignment']}", flush=True)
    assert r["ser"] < 0.05
    assert {a["tx"] for a in r["alignment"]} == {0, 1}
