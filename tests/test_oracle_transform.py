"""Pins for the oracle's number theory and transforms (Eqs. (1)-(5), (7), (8), Tab. 1).

Each check ties the oracle to something other than itself: hand-worked values,
closed forms, invariants, or brute-force integer convolution.
"""
import os
import random

import numpy as np
import pytest

from oracle import fnt_ref as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# The three (t, radix) pairs the paper uses: Fig. 1, the AEQ and the CDC.
CASES = [(2, "2", 8), (2, "sqrt2", 16), (3, "2", 16), (3, "sqrt2", 32), (4, "2", 32), (4, "sqrt2", 64)]


def is_prime(n):
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def horner(x, z, F):
    """Polynomial sum_n x[n] z^n evaluated by Horner's rule (a different route than Eq. (1))."""
    acc = 0
    for c in reversed(list(x)):
        acc = (acc * z + int(c)) % F
    return acc


def test_fermat_numbers_and_primality():
    # F_t = 2^(2^t) + 1 (FNT section); F_0..F_4 are the Fermat primes.
    assert [R.fermat(t) for t in range(5)] == [3, 5, 17, 257, 65537]
    assert all(is_prime(R.fermat(t)) for t in range(5))
    assert not is_prime(R.fermat(5))  # 641 * 6700417


def test_radix_sqrt2_is_4080_and_legal():
    # The CDC radix: alpha = sqrt(2) mod 65537 (Proposed structure); the shift-friendly
    # root 2^12 - 2^4.  Eq. (4) plus order exactly N (alpha^(N/2) = -1).
    F = 65537
    a = R.sqrt2(4)
    assert a == 4080 == (1 << 12) - (1 << 4)
    assert a * a % F == 2
    assert R.order(a, F) == 64
    assert pow(a, 32, F) == F - 1
    # the other root is -alpha = alpha^33
    assert (F - a) * (F - a) % F == 2 and pow(a, 33, F) == F - a
    # t = 2: sqrt(2) mod 17 = 6 (order 16), t = 3: 60 mod 257 (order 32)
    assert R.sqrt2(2) == 6 and 6 * 6 % 17 == 2 and R.order(6, 17) == 16
    assert R.sqrt2(3) == 60 and 60 * 60 % 257 == 2 and R.order(60, 257) == 32


@pytest.mark.parametrize("t,kind,N", CASES)
def test_transform_length_is_radix_order(t, kind, N):
    F = R.fermat(t)
    a = R.radix(t, kind)
    assert R.transform_length(t, kind) == N
    assert pow(a, N, F) == 1 and pow(a, N // 2, F) == F - 1  # Eq. (4), strengthened


def test_eq78_constants_are_inverses():
    # -2^(q-1) = 2^-1 and -2^(q/2-1) = (2 * 2^(q/2))^-1 mod F, q = 16 (Eqs. (7), (8)).
    F = 65537
    assert (-(1 << 15) * 2) % F == 1
    assert (-(1 << 7) * 512) % F == 1
    assert pow(256, 2, F) == F - 1          # j = 2^(q/2) is a square root of -1
    assert (64 * -1024) % F == 1            # N^-1 for N = 64
    assert (32 * -2048) % F == 1            # N^-1 for N = 32


def test_fig1_hand_worked_values():
    rows = []
    with open(os.path.join(GOLDEN, "fig1_fnt8_mod17.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            x, X = line.split("|")
            rows.append(([int(v) for v in x.split()], [int(v) for v in X.split()]))
    assert len(rows) == 5
    for x, X in rows:
        assert R.fnt(x, 2, 17) == X
        assert R.ifnt(X, 2, 17) == x


def test_fig1_unit_vectors_convolve_by_index_addition():
    # Exhaustive over pairs of unit vectors: delta_a (*) delta_b = delta_(a+b mod 8).
    F, N = 17, 8
    for a in range(N):
        for b in range(N):
            da = [1 if i == a else 0 for i in range(N)]
            db = [1 if i == b else 0 for i in range(N)]
            want = [1 if i == (a + b) % N else 0 for i in range(N)]
            assert R.cyclic_conv_fnt(da, db, 2, F) == want


@pytest.mark.parametrize("t,kind,N", CASES)
def test_fnt_is_polynomial_evaluation(t, kind, N):
    F = R.fermat(t)
    a = R.radix(t, kind)
    rng = random.Random(t * 100 + N)
    for _ in range(3):
        x = [rng.randrange(F) for _ in range(N)]
        X = R.fnt(x, a, F)
        assert X == [horner(x, pow(a, k, F), F) for k in range(N)]


@pytest.mark.parametrize("t,kind,N", CASES)
def test_fnt_special_bins_and_round_trip(t, kind, N):
    F = R.fermat(t)
    a = R.radix(t, kind)
    rng = random.Random(7 + N)
    for _ in range(3):
        x = [rng.randrange(F) for _ in range(N)]
        X = R.fnt(x, a, F)
        assert X[0] == sum(x) % F                                        # DC bin
        assert X[N // 2] == sum(v if n % 2 == 0 else -v for n, v in enumerate(x)) % F
        assert R.ifnt(X, a, F) == x
        assert R.fnt(R.ifnt(x, a, F), a, F) == x


@pytest.mark.parametrize("t,kind,N", CASES)
def test_convolution_theorem_vs_brute_force(t, kind, N):
    F = R.fermat(t)
    a = R.radix(t, kind)
    rng = random.Random(3 * N)
    for _ in range(3):
        x = [rng.randrange(F) for _ in range(N)]
        y = [rng.randrange(F) for _ in range(N)]
        brute = [sum(x[m] * y[(n - m) % N] for m in range(N)) % F for n in range(N)]
        assert R.cyclic_conv_fnt(x, y, a, F) == brute


def _linear_complex(xr, xi, hr, hi):
    """Brute-force complex linear convolution, numpy int64 (library routine)."""
    zr = np.convolve(xr, hr) - np.convolve(xi, hi)
    zi = np.convolve(xr, hi) + np.convolve(xi, hr)
    return zr, zi


def _cdc_window_check(xr, xi, hr, hi):
    N = 64
    L = len(hr)
    hpr = list(hr) + [0] * (N - L)
    hpi = list(hi) + [0] * (N - L)
    zr, zi = R.cdc_block_eq78(list(xr), list(xi), hpr, hpi)
    br, bi = _linear_complex(np.array(xr, np.int64), np.array(xi, np.int64),
                             np.array(hr, np.int64), np.array(hi, np.int64))
    # circular positions n >= L-1 are free of wrap-around and equal the linear conv
    return ([zr[n] for n in range(L - 1, N)] == [int(v) for v in br[L - 1:N]] and
            [zi[n] for n in range(L - 1, N)] == [int(v) for v in bi[L - 1:N]])


def test_eq78_complex_packing_random_blocks():
    rng = np.random.default_rng(1)
    for L in (1, 8, 17, 32):
        for _ in range(2):
            xr, xi = rng.integers(-16, 16, 64), rng.integers(-16, 16, 64)
            hr, hi = rng.integers(-32, 32, L), rng.integers(-32, 32, L)
            assert _cdc_window_check(xr, xi, hr, hi)


def test_eq5_worst_case_cdc_lifts_exactly():
    # Largest |Im z|: h = -32 - 32j against x = -16 - 16j on every tap -> 32 * 1024 = 32768
    # = (F-1)/2, exactly at the Eq. (5) bound.  Largest |Re z| (1008 per tap) likewise.
    L = 32
    hr, hi = [-32] * L, [-32] * L
    xr, xi = [-16] * 64, [-16] * 64
    assert _cdc_window_check(xr, xi, hr, hi)
    zr, zi = R.cdc_block_eq78(xr, xi, hr + [0] * 32, hi + [0] * 32)
    assert max(abs(v) for v in zi[31:]) == 32768
    hr2, hi2 = [-32] * L, [31] * L
    xr2, xi2 = [-16] * 64, [-16] * 64
    assert _cdc_window_check(xr2, xi2, hr2, hi2)


def test_eq5_violation_wraps():
    # Taps of 7 bit (outside the 6-bit width) break Eq. (5): the lift aliases.
    L = 32
    hr, hi = [-64] * L, [-64] * L
    xr, xi = [-16] * 64, [-16] * 64
    assert not _cdc_window_check(xr, xi, hr, hi)


def test_digit_split_exhaustive():
    for w in range(-8192, 8192):
        hi, lo = R.split_digits(w)
        assert 128 * hi + lo == w
        assert -64 <= lo <= 63 and -64 <= hi <= 64


def _aeq_brute(windows, w):
    """y[s2][n] for n = 16..31 by direct real convolution (numpy, int64)."""
    out = []
    for s2 in range(4):
        acc = np.zeros(47, np.int64)
        for s1 in range(4):
            acc += np.convolve(np.array(windows[s1], np.int64), np.array(w[s1][s2], np.int64))
        out.append([int(v) for v in acc[16:32]])
    return out


def test_aeq_digit_split_block_random():
    rng = np.random.default_rng(2)
    for _ in range(2):
        win = rng.integers(-16, 16, (4, 32))
        w = rng.integers(-8192, 8192, (4, 4, 16))
        y = R.aeq_block_digits(win.tolist(), w.tolist())
        assert [row[16:] for row in y] == _aeq_brute(win.tolist(), w.tolist())


def test_aeq_digit_split_block_worst_case():
    # Every digit at its extreme against -16 inputs: each pair sum hits 2*16*64*16 = 32768.
    win = [[-16] * 32 for _ in range(4)]
    for tap in (-8192, 8191, -8128, 8127, -64):
        w = [[[tap] * 16 for _ in range(4)] for _ in range(4)]
        y = R.aeq_block_digits(win, w)
        assert [row[16:] for row in y] == _aeq_brute(win, w)


def _gradient_direct(eps, win):
    # G[k] = sum_m eps[m] x[16 b + m - k], the block's symbols at window positions 16..31
    return [sum(eps[m] * win[16 + m - k] for m in range(16)) for k in range(16)]


def test_aeq_gradient_in_the_fermat_domain_is_exact():
    # The correlation through FNT32 equals the direct sum for random blocks and at the
    # Eq. (5) extreme (|eps| = 128 against |x| = 16 everywhere: 16 * 128 * 16 = 32768).
    rng = random.Random(17)
    for trial in range(200):
        eps = [rng.randint(-128, 127) for _ in range(16)]
        win = [rng.randint(-16, 15) for _ in range(32)]
        assert R.aeq_gradient_fnt(eps, win) == _gradient_direct(eps, win), trial
    for e0, x0 in ((-128, -16), (-128, 15), (127, -16)):
        eps, win = [e0] * 16, [x0] * 32
        assert R.aeq_gradient_fnt(eps, win) == _gradient_direct(eps, win)
    # past the bound (a 9-bit error, 16 * 256 * 16 = 65536) the lift wraps
    eps, win = [-256] * 16, [-16] * 32
    assert R.aeq_gradient_fnt(eps, win) != _gradient_direct(eps, win)


def test_table1_product_counts():
    # Tab. 1: FNT-CDC 8 and FNT-AEQ 64 real multiplications.  Per CDC block of one
    # polarisation: 2 spectra x 64 bins for 32 new instants; both polarisations -> 8
    # per dual-pol instant.  Per AEQ block: 16 filters x 2 digit groups x 32 bins for
    # 16 new symbols -> 64 per symbol.
    cnt = {}
    z = [0] * 64
    R.cdc_block_eq78(z, z, z, z, counter=cnt)
    assert cnt["products"] * 2 / 32 == 8
    cnt = {}
    R.aeq_block_digits([[0] * 32] * 4, [[[0] * 16] * 4] * 4, counter=cnt)
    assert cnt["products"] / 16 == 64


# ---- longer CDC transform (N = 128) with 3-bit tap digits ------------------------
def _long_window_check(xr, xi, hr, hi, model):
    N = 128
    L = len(hr)
    hpr = list(hr) + [0] * (N - L)
    hpi = list(hi) + [0] * (N - L)
    zr, zi = model(list(xr), list(xi), hpr, hpi)
    br, bi = _linear_complex(np.array(xr, np.int64), np.array(xi, np.int64),
                             np.array(hr, np.int64), np.array(hi, np.int64))
    return ([zr[n] for n in range(L - 1, N)] == [int(v) for v in br[L - 1:N]] and
            [zi[n] for n in range(L - 1, N)] == [int(v) for v in bi[L - 1:N]])


def test_long_radix_order_128():
    F = 65537
    a = R.sqrt_sqrt2(4)
    assert a == 4938
    assert a * a % F == R.sqrt2(4) == 4080
    assert R.order(a, F) == 128 and pow(a, 64, F) == F - 1


def test_long_constants_fold_n_inverse():
    # With N = 128 (N^-1 = -512 = -2^9) the constants of Eqs. (7)-(8) times N^-1
    # become -256 for z and -1 for z^ (2^32 = 1 and 2^16 = -1 mod F)
    F = 65537
    assert (128 * -512) % F == 1
    assert (-(1 << 15) * -512 - -256) % F == 0
    assert (-(1 << 7) * -512 - -1) % F == 0
    # they are the inverses of 2 N and of 2 N j (j = 2^8)
    assert (-256 * 256) % F == 1 and (-1 * 256 * 256) % F == 1


def test_digit3_split_exhaustive():
    for h in range(-32, 32):
        hi, lo = R.split_digits3(h)
        assert 8 * hi + lo == h
        assert -4 <= lo <= 3 and -4 <= hi <= 4


def test_long_block_random_vs_numpy():
    rng = np.random.default_rng(11)
    for L in (1, 33, 34, 50, 65):
        xr, xi = rng.integers(-16, 16, 128), rng.integers(-16, 16, 128)
        hr, hi = rng.integers(-32, 32, L), rng.integers(-32, 32, L)
        assert _long_window_check(xr, xi, hr, hi, R.cdc_block_long)


def test_long_eq5_worst_case_needs_the_digits():
    # 65 taps of -32 - 32j against x = -16 - 16j: |Im z| = 65 * 1024 = 66560, far
    # beyond (F - 1) / 2.  One transform per component wraps; the 3-bit digits keep
    # each partial convolution within 65 * 128 = 8320 (Eq. (5)) and recombine exactly.
    L = 65
    for hr, hi in (([-32] * L, [-32] * L), ([-32] * L, [31] * L), ([31] * L, [-32] * L)):
        xr, xi = [-16] * 128, [-16] * 128
        assert _long_window_check(xr, xi, hr, hi, R.cdc_block_long)
        undigitised = lambda a, b, c, d: R.cdc_block_eq78(a, b, c, d, alpha=R.sqrt_sqrt2(4))
        assert not _long_window_check(xr, xi, hr, hi, undigitised)
    # the per-digit bound itself: hi digits of -4 (h = -32) and lo digits of -4 (h = -4)
    hi_d = [R.split_digits3(-32)[0]] * L
    zr, zi = R.cdc_block_eq78([-16] * 128, [-16] * 128, hi_d + [0] * 63, hi_d + [0] * 63,
                              alpha=R.sqrt_sqrt2(4))
    assert max(abs(v) for v in zi[64:]) == 65 * 4 * 16 * 2 == 8320


def test_long_block_product_count():
    cnt = {}
    z = [0] * 128
    R.cdc_block_long(z, z, z, z, counter=cnt)
    assert cnt["products"] == 2 * 2 * 128       # two digits x (P, Q) x 128 bins per polarisation block
