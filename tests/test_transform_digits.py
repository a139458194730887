"""The arithmetic the AEQ's matrix-core input spectra rely on, checked on the CPU.

The polarisation-split AEQ computes Eq. (1)'s forward transform (N = 32, radix 2,
F = 65537) of 8 blocks' windows as one matrix product on the int8 matrix cores.
Row p of the transform matrix holds bin bitrev5(p) (the position order of the
products), and every entry 2^(nk) mod F is a signed power of two written as
256 hi + lo with int8 digits hi, lo; the kernel accumulates the hi digits, scales
the 32-bit accumulator by 256, adds the lo digits and folds once.  These tests
restate that decomposition from its definition and pin it against the oracle's
transform: congruence of every entry, int8 range of every digit, the int32 and
fold bounds at the extreme 5-bit windows, and equality of the whole digit product
with the plain transform on random windows.
"""
import numpy as np

from oracle import fnt_ref as R

F = R.fermat(4)


def bitrev5(p):
    return int(f"{p:05b}"[::-1], 2)


def digits(k, n):
    """(hi, lo) of the entry 2^(k n) mod F as the matrix cores take it."""
    m = (k * n) % 32
    e, neg = m % 16, m >= 16            # 2^m = -2^(m-16) for m >= 16, since 2^16 = -1
    if e <= 6:
        return 0, -(1 << e) if neg else 1 << e
    if e == 7:
        return (0, -128) if neg else (1, -128)
    if e <= 14:
        return (-(1 << (e - 8)) if neg else 1 << (e - 8)), 0
    return (-128, 0) if neg else (-128, -1)      # 2^15 = -32769 (mod F)


def digit_matrices():
    hi = np.zeros((32, 32), np.int64)
    lo = np.zeros((32, 32), np.int64)
    for p in range(32):
        for n in range(32):
            hi[p, n], lo[p, n] = digits(bitrev5(p), n)
    return hi, lo


def test_every_entry_congruent_and_int8():
    hi, lo = digit_matrices()
    assert hi.min() >= -128 and hi.max() <= 127 and lo.min() >= -128 and lo.max() <= 127
    for p in range(32):
        for n in range(32):
            assert (256 * hi[p, n] + lo[p, n] - pow(2, bitrev5(p) * n, F)) % F == 0, (p, n)


def fold16(v):
    return (v & 0xFFFF) - (v >> 16)


def test_accumulator_and_fold_bounds():
    """The largest magnitude either digit sum can reach with 5-bit samples, the
    scaled accumulator within int32, and the folded value within the 24-bit
    operand range of the spectral products."""
    hi, lo = digit_matrices()
    worst_hi = int(np.abs(hi).sum(axis=1).max()) * 16
    worst_lo = int(np.abs(lo).sum(axis=1).max()) * 16
    acc = 256 * worst_hi + worst_lo
    assert acc < 2 ** 31 - 1
    for v in (acc, -acc, 0, 65535, -65536):
        assert abs(fold16(v)) < 2 ** 17


def test_digit_product_equals_transform():
    hi, lo = digit_matrices()
    rng = np.random.default_rng(11)
    windows = rng.integers(-16, 16, size=(32, 32), dtype=np.int64)     # 32 columns of 32 symbols
    windows[:, 0] = -16                                                # an extreme column
    windows[:, 1] = 15
    acc = 256 * (hi @ windows) + lo @ windows                          # as the matrix cores accumulate it
    assert np.abs(acc).max() < 2 ** 31
    folded = fold16(acc)
    for c in range(windows.shape[1]):
        X = R.fnt([int(v) % F for v in windows[:, c]], 2, F)
        for p in range(32):
            assert (int(folded[p, c]) - X[bitrev5(p)]) % F == 0, (c, p)
