"""Plain number-theoretic definitions of the Fermat number transform.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may use this module; the product path never does.

Everything here is Python integers, evaluated straight from the paper's
equations with no fast algorithm:

* ``fermat``               F_t = 2^(2^t) + 1            (FNT section, after Eq. (4))
* ``sqrt2``                a square root of 2 in Z_F    (radix of the FNT-CDC, Proposed structure)
* ``fnt`` / ``ifnt``       Eqs. (1) and (2) as O(N^2) sums
* ``cdc_block_eq78``       one overlap-save CDC block through Eqs. (7)-(8)
* ``cdc_block_long``       the same with N = 128 (radix of order 128) and the
                           6-bit taps split into two balanced 3-bit digits
* ``aeq_block_digits``     one AEQ filtering block through the 7+7-bit tap split

Both block models take an optional ``counter`` dict that tallies the true
Z_F multiplications (the pointwise products), the quantity of Tab. 1.

The two block models follow the method's steps (transform, pointwise product,
inverse transform, centred lift) on one block so that the tests can pin the
algebra of Eqs. (5), (7), (8) and of the digit split against brute-force
integer convolution.  The block-streaming results that the GPU must match are
the direct definitions in ``oracle.c``.
"""
from __future__ import annotations


def fermat(t: int) -> int:
    """Fermat number F_t = 2^(2^t) + 1."""
    return (1 << (1 << t)) + 1


def sqrt2(t: int) -> int:
    """The square root of 2 modulo F_t (t >= 2) made of two powers of two.

    With q = 2^t: (2^(3q/4) - 2^(q/4))^2 = 2^(3q/2) - 2^(q+1) + 2^(q/2), and
    2^q = -1 (mod F_t) turns this into 2.  For t = 4 it is 2^12 - 2^4 = 4080.
    """
    q = 1 << t
    return (pow(2, 3 * q // 4) - pow(2, q // 4)) % fermat(t)


def sqrt_sqrt2(t: int) -> int:
    """A radix of order 2^(t+3) modulo F_t: the smaller square root of sqrt2(t),
    by exhaustive search (4938 for t = 4).  Its square is sqrt2(t), so its
    order is twice that of sqrt2(t)."""
    F = fermat(t)
    s = sqrt2(t)
    return min(x for x in range(F) if x * x % F == s)


def radix(t: int, kind: str) -> int:
    if kind == "2":
        return 2
    if kind == "sqrt2":
        return sqrt2(t)
    raise ValueError(kind)


def order(a: int, F: int) -> int:
    """Multiplicative order of a modulo F by brute force."""
    x, k = a % F, 1
    while x != 1:
        x = x * a % F
        k += 1
        if k > F:
            raise ValueError("not a unit")
    return k


def transform_length(t: int, kind: str) -> int:
    """N = order of the radix: 2^(t+1) for alpha = 2, 2^(t+2) for alpha = sqrt(2)."""
    return order(radix(t, kind), fermat(t))


def fnt(x, alpha: int, F: int):
    """Eq. (1): X(k) = sum_n x(n) alpha^(n k) mod F."""
    N = len(x)
    return [sum(int(x[n]) * pow(alpha, n * k, F) for n in range(N)) % F for k in range(N)]


def ifnt(X, alpha: int, F: int):
    """Eq. (2): x(n) = N^-1 sum_k X(k) alpha^(-n k) mod F."""
    N = len(X)
    ninv = pow(N, -1, F)
    ainv = pow(alpha, -1, F)
    return [ninv * sum(int(X[k]) * pow(ainv, n * k, F) for k in range(N)) % F for n in range(N)]


def lift(r: int, F: int) -> int:
    """Centred representative of r mod F in [-(F-1)/2, (F-1)/2]."""
    r %= F
    return r - F if r > (F - 1) // 2 else r


def cyclic_conv_fnt(x, y, alpha: int, F: int):
    """Cyclic convolution through the transform: IFNT(FNT(x) . FNT(y))."""
    X, Y = fnt(x, alpha, F), fnt(y, alpha, F)
    return ifnt([a * b % F for a, b in zip(X, Y)], alpha, F)


def cdc_block_eq78(win_r, win_i, h_r, h_i, t: int = 4, counter=None, alpha=None):
    """One overlap-save CDC block by the complex packing of Eqs. (7)-(8).

    ``win_*``: the N-sample input window (oldest first) of one polarisation,
    ``h_*``: the taps zero-padded to N.  With q = 2^t and j = 2^(q/2) (j^2 = -1
    mod F), the method transforms x_r + j x_i and x_r - j x_i (equivalently
    FNT(x_r) +/- j FNT(x_i)), multiplies bin by bin with the matching tap
    spectra, and recovers

        z  = -2^(q-1)   IFNT(P + Q)      (Eq. 7)
        z^ = -2^(q/2-1) IFNT(P - Q)      (Eq. 8)

    then lifts to the centred range.  Returns the N circular outputs
    (re, im) as lists; positions >= L-1 equal the linear convolution.
    """
    q = 1 << t
    F = fermat(t)
    alpha = sqrt2(t) if alpha is None else alpha
    j = pow(2, q // 2, F)
    N = len(win_r)
    Xr, Xi = fnt(win_r, alpha, F), fnt(win_i, alpha, F)
    Hr, Hi = fnt(h_r, alpha, F), fnt(h_i, alpha, F)
    P = [(Xr[k] + j * Xi[k]) * (Hr[k] + j * Hi[k]) % F for k in range(N)]
    Q = [(Xr[k] - j * Xi[k]) * (Hr[k] - j * Hi[k]) % F for k in range(N)]
    if counter is not None:
        counter["products"] = counter.get("products", 0) + 2 * N
    zs = ifnt([(a + b) % F for a, b in zip(P, Q)], alpha, F)
    zd = ifnt([(a - b) % F for a, b in zip(P, Q)], alpha, F)
    c7 = -pow(2, q - 1)
    c8 = -pow(2, q // 2 - 1)
    return [lift(c7 * v, F) for v in zs], [lift(c8 * v, F) for v in zd]


def split_digits3(h: int):
    """6-bit tap -> (hi, lo) with h = 8 hi + lo, lo = ((h + 4) mod 8) - 4 in
    [-4, 3] and hi = (h - lo) / 8 in [-4, 4]."""
    lo = ((h + 4) % 8) - 4
    return (h - lo) // 8, lo


def cdc_block_long(win_r, win_i, h_r, h_i, t: int = 4, counter=None):
    """One overlap-save CDC block of N = len(win_r) = 128 samples (64 new) for
    up to 65 taps: longer than the N = 64 block of the paper allows (33 taps).

    A 65-tap convolution of 5-bit samples with 6-bit taps reaches
    65 * (32 * 16 + 31 * 16) = 65520 > (F - 1) / 2, outside Eq. (5), so the taps
    are split into two balanced 3-bit digits, h = 8 hi + lo; each digit's
    convolution stays within 65 * (4 * 16 + 4 * 16) = 8320 and goes through
    Eqs. (7)-(8) with the radix of order 128 (sqrt_sqrt2); the two centred
    results are combined as z = 8 z_hi + z_lo.  Returns the N circular outputs
    (re, im); positions >= L - 1 equal the linear convolution."""
    alpha = sqrt_sqrt2(t)
    dr = [split_digits3(int(v)) for v in h_r]
    di = [split_digits3(int(v)) for v in h_i]
    zh = cdc_block_eq78(win_r, win_i, [d[0] for d in dr], [d[0] for d in di], t, counter, alpha)
    zl = cdc_block_eq78(win_r, win_i, [d[1] for d in dr], [d[1] for d in di], t, counter, alpha)
    return ([8 * a + b for a, b in zip(zh[0], zl[0])], [8 * a + b for a, b in zip(zh[1], zl[1])])


def split_digits(w: int):
    """14-bit tap -> (hi, lo) with w = 2^7 hi + lo, lo the low 7 bits (balanced).

    lo = ((w + 64) mod 128) - 64 in [-64, 63], hi = (w - lo) / 128 in [-64, 64].
    """
    lo = ((w + 64) % 128) - 64
    return (w - lo) // 128, lo


def aeq_block_digits(windows, w, t: int = 4, counter=None):
    """One AEQ filtering block (4x4 real MIMO) through the 7+7-bit split.

    ``windows[s1]``: the 32-symbol input window of stream s1 (oldest first);
    ``w[s1][s2]``: 16 taps of 14 bit.  Each tap set is split into two 7-bit
    digit groups; every group is convolved through the N = 32, alpha = 2
    transform, the two streams of a polarisation are summed in the transform
    domain (Eq. (5) still holds for the sum), and the result is recombined as
    2^7 * hi + lo.  Returns y[s2][n] for the 32 circular positions; positions
    16..31 are the block's linear outputs.
    """
    F = fermat(t)
    alpha = 2
    N = 32
    A = [fnt(list(windows[s]), alpha, F) for s in range(4)]
    y = [[0] * N for _ in range(4)]
    for s2 in range(4):
        for pair in ((0, 1), (2, 3)):
            for d in (0, 1):
                acc = [0] * N
                for s1 in pair:
                    dig = [split_digits(int(v))[d] for v in w[s1][s2]] + [0] * (N - len(w[s1][s2]))
                    W = fnt(dig, alpha, F)
                    acc = [(acc[k] + A[s1][k] * W[k]) % F for k in range(N)]
                    if counter is not None:
                        counter["products"] = counter.get("products", 0) + N
                part = [lift(v, F) for v in ifnt(acc, alpha, F)]
                scale = 128 if d == 0 else 1
                y[s2] = [y[s2][n] + scale * part[n] for n in range(N)]
    return y


def aeq_gradient_fnt(eps, window, t: int = 4):
    """The RDE gradient of one AEQ block in the Fermat domain (a variant the
    block update of Eq. (6) admits; the kernels compute it directly).

    ``eps``: the 16 error terms of output stream S2 in the block (8-bit);
    ``window``: the 32-symbol input window of stream S1 (oldest first, the block's
    own symbols at 16..31).  G[k] = sum_m eps[m] x[16 b + m - k] for k < 16 is a
    correlation: with the reversed, zero-padded error e'[n] = eps[15 - n], the
    cyclic convolution c = IFNT(FNT(window) FNT(e')) (N = 32, alpha = 2) holds
    c[31 - k] = G[k] with no wrap-around (the largest index used is 31).  Every
    true value is at most 16 * 128 * 16 = 32768 = (F - 1) / 2 (Eq. (5)), so the
    centred lift is exact.  Returns G[0..15]."""
    F = fermat(t)
    N = 32
    e = [eps[15 - n] for n in range(16)] + [0] * 16
    X = fnt([v % F for v in window], 2, F)
    E = fnt([v % F for v in e], 2, F)
    c = [lift(v, F) for v in ifnt([X[k] * E[k] % F for k in range(N)], 2, F)]
    return [c[N - 1 - k] for k in range(16)]

