"""GPU parity of fnt_cdc_long: the CDC with a 128-point transform (64 new
instants per block) and 3-bit tap digits, for up to 65 taps, against the
oracle's direct convolution (exact z and the resampled 5-bit stream), element
by element: random lengths with ragged tails, both decimation phases, every
tap count class, the Eq. (5) worst cases that need the digit split, and the
range and argument errors."""
import numpy as np
import pytest

import oracle as O
from paper_2405_04253_amd import fnt, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fnt.lib()
    fnt.fnt_check()
    return torch, torch.device("cuda:0")


def note(msg):
    print(f"[case] {msg}", flush=True)


def check(torch, dev, x, h, shift, phase):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    z, a = fnt.fnt_cdc_long(xd, h, shift, phase)
    torch.cuda.synchronize()
    zr, ar = O.cdc(x, h, shift, phase)
    assert np.array_equal(z.cpu().numpy(), zr), (x.shape[0], h.shape[0], shift, phase)
    assert np.array_equal(a.cpu().numpy(), ar), (x.shape[0], h.shape[0], shift, phase)
    return zr


@pytest.mark.parametrize("n,L,shift,phase", [(1, 1, 0, 0), (63, 65, 3, 1), (64, 34, 5, 0), (65, 65, 7, 1),
                                              (1000, 50, 8, 0), (4113, 33, 6, 1), (100000, 65, 9, 0),
                                              (262144 + 40, 64, 11, 1)])
def test_cdc_long_random_vs_oracle(torch_dev, n, L, shift, phase):
    torch, dev = torch_dev
    x = synth.random_samples(n, seed=n + L)
    h = synth.random_taps(L, seed=7 * L + n)
    note(f"fnt_cdc_long n={n} L={L} shift={shift} phase={phase}")
    check(torch, dev, x, h, shift, phase)
    fnt.fnt_check()


def test_cdc_long_eq5_worst_cases(torch_dev):
    """65 taps of -32 - 32j (and mixed signs) on samples of -16: |z| up to
    65 * 1024 = 66560, twice the Eq. (5) bound, exact through the 3-bit digits."""
    torch, dev = torch_dev
    n = 64 * 40 + 5
    for hr, hi in ((-32, -32), (-32, 31), (31, -32), (31, 31)):
        x = np.full((n, 4), -16, dtype=np.int8)
        h = np.empty((65, 2), dtype=np.int8)
        h[:, 0], h[:, 1] = hr, hi
        note(f"fnt_cdc_long worst case taps ({hr}, {hi})")
        zr = check(torch, dev, x, h, 16, 0)
        assert np.abs(zr[100:]).max() > 32768            # beyond one transform's range
    fnt.fnt_check()


def test_cdc_long_range_and_argument_errors(torch_dev):
    torch, dev = torch_dev
    x = synth.random_samples(300, seed=3)
    x[123, 2] = 17                                      # outside 5 bit
    xd = torch.from_numpy(x).to(dev)
    h = synth.random_taps(40, seed=4)
    note("fnt_cdc_long range flag")
    fnt.fnt_cdc_long(xd, h, 4, 0)
    torch.cuda.synchronize()
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_check()
    assert e.value.code == fnt.FNT_E_RANGE
    fnt.fnt_check()                                     # the flag was cleared
    for bad in (np.zeros((0, 2), np.int8), np.zeros((66, 2), np.int8)):
        with pytest.raises(fnt.FntError) as e:
            fnt.fnt_cdc_long(xd, bad, 4, 0)
        assert e.value.code == fnt.FNT_E_INVAL
    hb = h.copy()
    hb[5, 1] = -33
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_cdc_long(xd, hb, 4, 0)
    assert e.value.code == fnt.FNT_E_RANGE
    with pytest.raises(fnt.FntError):
        fnt.fnt_cdc_long(xd, h, 17, 0)
    with pytest.raises(fnt.FntError):
        fnt.fnt_cdc_long(xd, h, 4, 2)
    z, a = fnt.fnt_cdc_long(xd[:0], h, 4, 0)            # empty input: nothing to do
    assert z.shape[0] == 0 and a.shape[0] == 0
