"""Pins for the oracle's CDC, resampling/requantisation and AEQ definitions.

CDC is pinned to numpy's convolution (library routine) and to the FNT block
model of Eqs. (7)-(8); requantisation to hand-worked rounding values and the
round-to-nearest property; the AEQ filter bank to numpy's convolution, and the
RDE update (Eq. (6)) to a hand-worked two-block example and to invariants.
"""
import numpy as np
import pytest

import oracle as O
from oracle import fnt_ref as R
from paper_2405_04253_amd import synth


def np_cdc(x, h):
    """Exact complex causal convolution by numpy (int64), both polarisations."""
    x = x.astype(np.int64)
    hr, hi = h[:, 0].astype(np.int64), h[:, 1].astype(np.int64)
    n = x.shape[0]
    z = np.zeros((n, 4), np.int64)
    if n == 0:
        return z
    for p in range(2):
        xr, xi = x[:, 2 * p], x[:, 2 * p + 1]
        z[:, 2 * p] = (np.convolve(xr, hr) - np.convolve(xi, hi))[:n]
        z[:, 2 * p + 1] = (np.convolve(xi, hr) + np.convolve(xr, hi))[:n]
    return z


def test_rounding_hand_values():
    # rs(v, s): round half up then drop s bits; sat_b: clamp to b-bit two's complement.
    cases = [(3, 1, 2), (-3, 1, -1), (5, 2, 1), (6, 2, 2), (-5, 2, -1), (-6, 2, -1),
             (-7, 2, -2), (7, 0, 7), (-1, 1, 0), (1, 1, 1), (-32768, 15, -1), (32767, 15, 1)]
    for v, s, want in cases:
        assert O.rs(v, s) == want, (v, s)
    assert O.sat(100, 5) == 15 and O.sat(-100, 5) == -16 and O.sat(15, 5) == 15
    assert O.sat(40000, 16) == 32767 and O.sat(-9000, 14) == -8192 and O.sat(8191, 14) == 8191


def _check_requant(z, a, shift):
    """Round-to-nearest property (ties up), with saturation to 5 bit."""
    z = z.astype(np.int64)
    a = a.astype(np.int64)
    sat_hi = a == 15
    sat_lo = a == -16
    mid = ~(sat_hi | sat_lo)
    if shift == 0:
        assert np.array_equal(a[mid], z[mid])
    else:
        d = z - a * (1 << shift)           # remainder after rounding
        half = 1 << (shift - 1)
        assert np.all((d[mid] >= -half) & (d[mid] < half))
    assert np.all(z[sat_hi] >= 15 * (1 << shift) - (1 << shift) // 2)
    assert np.all(z[sat_lo] < -16 * (1 << shift) + (1 << shift) // 2)


@pytest.mark.parametrize("n,L,shift,phase", [(0, 32, 7, 0), (1, 5, 0, 0), (2, 32, 7, 1),
                                             (97, 17, 6, 0), (1000, 32, 7, 1), (333, 8, 3, 1)])
def test_cdc_matches_numpy_convolve(n, L, shift, phase):
    x = synth.random_samples(n, seed=n + L)
    h = synth.random_taps(L, seed=L)
    z, a = O.cdc(x, h, shift, phase)
    assert np.array_equal(z.astype(np.int64), np_cdc(x, h))
    assert a.shape[0] == O.n_symbols(n, phase) == len(range(phase, n, 2))
    _check_requant(z[phase::2], a, shift)


def test_cdc_generated_channel_and_bound():
    ch = synth.single_channel(1 << 12)
    z, a = O.cdc(ch.samples, ch.taps, ch.requant_shift)
    assert np.array_equal(z.astype(np.int64), np_cdc(ch.samples, ch.taps))
    assert np.abs(z).max() <= 32768          # Eq. (5) holds for 5-bit data, 32 taps of 6 bit
    _check_requant(z[0::2], a, ch.requant_shift)


def test_cdc_matches_eq78_block_model():
    # Two independent formulations of the oracle side agree: direct convolution and
    # the overlap-save FNT block with the complex packing (64-point window, 32 new).
    ch = synth.single_channel(256)
    z, _ = O.cdc(ch.samples, ch.taps, ch.requant_shift)
    L = ch.ntaps
    hr = [int(v) for v in ch.taps[:, 0]] + [0] * (64 - L)
    hi = [int(v) for v in ch.taps[:, 1]] + [0] * (64 - L)
    x = np.concatenate([np.zeros((32, 4), np.int8), ch.samples])
    for b in (0, 3, 7):
        for p in range(2):
            win = x[32 * b: 32 * b + 64]
            zr, zi = R.cdc_block_eq78([int(v) for v in win[:, 2 * p]],
                                      [int(v) for v in win[:, 2 * p + 1]], hr, hi)
            assert zr[32:] == [int(v) for v in z[32 * b: 32 * b + 32, 2 * p]]
            assert zi[32:] == [int(v) for v in z[32 * b: 32 * b + 32, 2 * p + 1]]


def test_cdc_history_streaming():
    x = synth.random_samples(640, seed=5)
    h = synth.random_taps(32, seed=6)
    z, a = O.cdc(x, h, 7)
    k = 320
    z2, a2 = O.cdc(x[k:], h, 7, hist=x[k - 32:k])
    assert np.array_equal(z2, z[k:])
    assert np.array_equal(a2, a[k // 2:])


def np_fir_bank(a, w):
    a = a.astype(np.int64)
    M = a.shape[0]
    y = np.zeros((M, 4), np.int64)
    if M == 0:
        return y
    for s2 in range(4):
        for s1 in range(4):
            y[:, s2] += np.convolve(a[:, s1], w[s1, s2].astype(np.int64))[:M]
    return y


def test_aeq_fixed_bank_matches_numpy(aeq_defaults):
    rng = np.random.default_rng(9)
    for M in (0, 1, 15, 16, 17, 100):
        a = rng.integers(-16, 16, (M, 4)).astype(np.int8)
        w = synth.random_aeq_taps(seed=M)
        prm = O.params(**dict(aeq_defaults, update_enable=0))
        out, wf = O.aeq(a, w, prm)
        assert np.array_equal(wf, w)
        y = np_fir_bank(a, w)
        s = aeq_defaults["out_shift"]
        half = 1 << (s - 1)
        yh = out.astype(np.int64)
        d = y - yh * (1 << s)
        ok = (yh == 32767) | (yh == -32768) | ((d >= -half) & (d < half))
        assert ok.all()


def test_aeq_hand_worked_two_blocks():
    # Block 0: a[0].XI = 8, w[XI][XI][0] = w[XQ][XQ][0] = 4096, s_o = 7, c_y = 64
    # (c^2 = 4096: thresholds 6c^2 = 24576, 14c^2 = 57344), s_e = 16, s_mu = 0.
    #   y_XI[0] = 4096*8 = 32768 -> yhat = rs(32768, 7) = 256, all other yhat = 0.
    #   r2 = 65536 >= 57344 -> R2 = 18c^2 = 73728, e = 8192,
    #   eps_XI[0] = rs(8192*256, 16) = 32; all other eps are 0 (yhat = 0).
    #   G[XI][XI][0] = 32 * a[0].XI = 256, every other G entry is 0
    #   -> w[XI][XI][0] = 4096 + 256 = 4352.
    # Block 1: a[16].XQ = -4.
    #   y_XQ[16] = w[XQ][XQ][0] * -4 = -16384 -> yhat = -128; pol X r2 = 16384 < 24576
    #   -> R2 = 2c^2 = 8192, e = -8192, eps_XQ[16] = rs(-8192*-128, 16) = 16.
    #   G[XQ][XQ][0] = 16 * -4 = -64 -> w[XQ][XQ][0] = 4032.  a[0] is 16 symbols back,
    #   outside the 16 taps, so nothing else moves.
    a = np.zeros((32, 4), np.int8)
    a[0, 0] = 8
    a[16, 1] = -4
    w = np.zeros((4, 4, 16), np.int16)
    w[0, 0, 0] = 4096
    w[1, 1, 0] = 4096
    prm = O.params(out_shift=7, err_shift=16, mu_shift=0, const_unit=64, update_enable=1)
    out, wf = O.aeq(a, w, prm)
    want_out = np.zeros((32, 4), np.int16)
    want_out[0, 0] = 256
    want_out[16, 1] = -128
    assert np.array_equal(out, want_out)
    want_w = w.copy()
    want_w[0, 0, 0] = 4352
    want_w[1, 1, 0] = 4032
    assert np.array_equal(wf, want_w)


def test_aeq_hand_worked_rings_lags_cross_pol():
    # One block of 16 symbols, two of them nonzero, with c_y = 64 (c^2 = 4096):
    # thresholds 6c^2 = 24576 and 14c^2 = 57344, radii R2 = 2c^2 = 8192,
    # 10c^2 = 40960, 18c^2 = 73728.  Neither threshold is a sum of two integer
    # squares (3 and 7 appear to an odd power), so r2 never ties with one; the
    # symbols below sit 31 below / 4 and 13 above them.  s_o = 0 (yhat = y),
    # s_e = 15, s_mu = 0 (w += G).  Lag-0 taps only: t = (16, 11, 39, 17) on
    # S1 == S2, so yhat_S[m] = t_S a_S[m].
    #   a[0] = (4, 13, -2, -8)   a[1] = (12, 13, -6, -3)
    #   m=0 X: yhat (64, 143)    r2 = 4096 + 20449  = 24545 < 6c^2    -> R2 =  8192, e_X = -16353
    #   m=0 Y: yhat (-78, -136)  r2 = 6084 + 18496  = 24580 >= 6c^2   -> R2 = 40960, e_Y = +16380
    #   m=1 X: yhat (192, 143)   r2 = 36864 + 20449 = 57313 < 14c^2   -> R2 = 40960, e_X = -16353
    #   m=1 Y: yhat (-234, -51)  r2 = 54756 + 2601  = 57357 >= 14c^2  -> R2 = 73728, e_Y = +16371
    # eps_S2 = sat8(rs(e_pol(S2) yhat_S2, 15)), e.g. rs(-16353 * 64, 15) = floor(-31.94 + 0.5) = -32:
    #   eps[0] = (-32, -71, -39, -68)    eps[1] = (-96, -71, -117, -25)
    # G[S1][S2][0] = eps_S2[0] a_S1[0] + eps_S2[1] a_S1[1];  G[S1][S2][1] = eps_S2[1] a_S1[0]
    # (lag 1 reaches a_S1[0] from m = 1; a[-1] is zero history), e.g.
    #   G[XI][XI][0] = -32*4 + -96*12 = -1280 -> w = 16 - 1280 = -1264;  G[XI][XI][1] = -96*4 = -384
    #   G[YI][XQ][0] = -71*-2 + -71*-6 = 568 (cross-polarisation: S2 = XQ uses e_X);  G[YI][XQ][1] = 142
    #   G[XQ][YI][0] = -39*13 + -117*13 = -2028 (S2 = YI uses e_Y);  G[XQ][YI][1] = -117*13 = -1521
    a = np.zeros((16, 4), np.int8)
    a[0] = (4, 13, -2, -8)
    a[1] = (12, 13, -6, -3)
    w = np.zeros((4, 4, 16), np.int16)
    for s, t in enumerate((16, 11, 39, 17)):
        w[s, s, 0] = t
    prm = O.params(out_shift=0, err_shift=15, mu_shift=0, const_unit=64, update_enable=1)
    out, wf = O.aeq(a, w, prm)
    want_out = np.zeros((16, 4), np.int16)
    want_out[0] = (64, 143, -78, -136)
    want_out[1] = (192, 143, -234, -51)
    assert np.array_equal(out, want_out)
    # final taps (lag 0, lag 1) for S1 (rows) x S2 = XI, XQ, YI, YQ (columns)
    want = {0: [(-1264, -384), (-1136, -284), (-1560, -468), (-572, -100)],
            1: [(-1664, -1248), (-1835, -923), (-2028, -1521), (-1209, -325)],
            2: [(640, 192), (568, 142), (819, 234), (286, 50)],
            3: [(544, 768), (781, 568), (663, 936), (636, 200)]}
    want_w = np.zeros((4, 4, 16), np.int16)
    for s1, row in want.items():
        for s2, (k0, k1) in enumerate(row):
            want_w[s1, s2, 0], want_w[s1, s2, 1] = k0, k1
    assert np.array_equal(wf, want_w)


def test_aeq_hand_worked_saturation_and_long_lags():
    # s_o = 10, s_e = 0, s_mu = 0, c_y = 64.  Taps: w[YI][XI][3] = 8150 (near the
    # 14-bit top), w[XQ][XQ][0] = -8000 (near the bottom), all others 0.
    # Input: a_YI[0] = 1, a_XQ[1] = 2, every other sample 0.
    #   y_XQ[1] = -8000 * 2 = -16000 -> yhat = rs(-16000, 10) = floor(-15.625 + 0.5) = -16
    #   y_XI[3] = 8150 * a_YI[0] = 8150 -> yhat = rs(8150, 10) = floor(7.959 + 0.5) = 8
    #   m=1 X: r2 = 256 < 6c^2 -> e = 8192 - 256 = 7936, eps_XQ = sat8(7936 * -16 = -126976) = -128
    #   m=3 X: r2 = 64         -> e = 8192 - 64 = 8128,  eps_XI = sat8(8128 * 8 = 65024) = 127
    #   every other yhat is 0, so every other eps is 0.
    # G[S1][XI][k] = 127 a_S1[3 - k]: G[YI][XI][3] = 127, G[XQ][XI][2] = 254
    # G[S1][XQ][k] = -128 a_S1[1 - k]: G[XQ][XQ][0] = -256, G[YI][XQ][1] = -128
    # w[YI][XI][3] = sat14(8150 + 127 = 8277) = 8191; w[XQ][XQ][0] = sat14(-8256) = -8192.
    a = np.zeros((16, 4), np.int8)
    a[0, 2] = 1
    a[1, 1] = 2
    w = np.zeros((4, 4, 16), np.int16)
    w[2, 0, 3] = 8150
    w[1, 1, 0] = -8000
    prm = O.params(out_shift=10, err_shift=0, mu_shift=0, const_unit=64, update_enable=1)
    out, wf = O.aeq(a, w, prm)
    want_out = np.zeros((16, 4), np.int16)
    want_out[1, 1] = -16
    want_out[3, 0] = 8
    assert np.array_equal(out, want_out)
    want_w = np.zeros((4, 4, 16), np.int16)
    want_w[2, 0, 3] = 8191
    want_w[1, 0, 2] = 254
    want_w[1, 1, 0] = -8192
    want_w[2, 1, 1] = -128
    assert np.array_equal(wf, want_w)


def test_aeq_update_invariants(aeq_defaults):
    ch = synth.single_channel(1 << 10)
    _, a = O.cdc(ch.samples, ch.taps, ch.requant_shift)
    w0 = synth.centre_spike_taps()
    # a step size too small to move any tap leaves the filter fixed
    out1, wf1 = O.aeq(a, w0, O.params(**dict(aeq_defaults, mu_shift=40)))
    out0, wf0 = O.aeq(a, w0, O.params(**dict(aeq_defaults, update_enable=0)))
    assert np.array_equal(wf1, w0) and np.array_equal(out1, out0)
    # zero error terms (err_shift huge) leave the taps fixed too
    _, wf2 = O.aeq(a, w0, O.params(**dict(aeq_defaults, err_shift=60)))
    assert np.array_equal(wf2, w0)
    # with the default step the taps move and stay within 14 bit
    _, wf3 = O.aeq(a, w0, O.params(**aeq_defaults))
    assert not np.array_equal(wf3, w0)
    assert wf3.min() >= -8192 and wf3.max() <= 8191


def test_aeq_history_streaming(aeq_defaults):
    rng = np.random.default_rng(11)
    a = rng.integers(-16, 16, (160, 4)).astype(np.int8)
    w0 = synth.centre_spike_taps()
    prm = O.params(**aeq_defaults)
    out, wf = O.aeq(a, w0, prm)
    k = 64
    o1, w1 = O.aeq(a[:k], w0, prm)
    o2, w2 = O.aeq(a[k:], w1, prm, hist=a[k - 16:k])
    assert np.array_equal(np.concatenate([o1, o2]), out)
    assert np.array_equal(w2, wf)


def test_rde_reduces_radius_error():
    # Sanity of the chosen constants (not parity): on the 75 km channel the RDE
    # pulls the outputs onto the 16QAM rings as the taps adapt.
    ch = synth.single_channel(1 << 14)
    prm = synth.aeq_params_for(ch)
    out, wf, a = O.cdc_aeq(ch.samples, ch.taps, ch.requant_shift, synth.centre_spike_taps(),
                           O.params(**prm))
    c2 = prm["const_unit"] ** 2
    y = out.astype(np.float64)

    def ring_err(seg):
        errs = []
        for p in range(2):
            r2 = seg[:, 2 * p] ** 2 + seg[:, 2 * p + 1] ** 2
            R2 = np.where(r2 < 6 * c2, 2 * c2, np.where(r2 < 14 * c2, 10 * c2, 18 * c2))
            errs.append(np.mean(np.abs(R2 - r2)) / c2)
        return float(np.mean(errs))

    early, late = ring_err(y[16:1024]), ring_err(y[-4096:])
    assert late < 0.7 * early, (early, late)


def test_chain_equals_parts_and_batch(aeq_defaults):
    prm = O.params(**aeq_defaults)
    chs = [synth.gen_channel(n, km, 20.0, seed=s) for n, km, s in ((300, 75, 1), (17, 12, 2), (0, 40, 3))]
    ref = []
    for ch in chs:
        _, a = O.cdc(ch.samples, ch.taps, ch.requant_shift)
        out, wf = O.aeq(a, synth.centre_spike_taps(), prm)
        o2, w2, a2 = O.cdc_aeq(ch.samples, ch.taps, ch.requant_shift, synth.centre_spike_taps(), prm)
        assert np.array_equal(out, o2) and np.array_equal(wf, w2) and np.array_equal(a, a2)
        ref.append((out, wf))
    outs, finals, used = O.batch([dict(samples=c.samples, taps=c.taps, shift=c.requant_shift,
                                       w=synth.centre_spike_taps(), params=prm) for c in chs],
                                 threads=2)
    assert used >= 1
    for (o, w), o2, w2 in zip(ref, outs, finals):
        assert np.array_equal(o, o2) and np.array_equal(w, w2)


# ---- RDE step schedule (mu_shift, then mu_shift_late from stream block gear_blocks) ----
def test_aeq_step_schedule_hand_worked():
    # The two-block example above with s_mu = 0 for stream block 0 and s_mu = 3 from
    # block 1 on (gear_blocks = 1):
    #   block 0: G[XI][XI][0] = 256 -> w = 4096 + rs(256, 0) = 4352 (as before);
    #   block 1: G[XQ][XQ][0] = -64 -> w = 4096 + rs(-64, 3) = 4096 + floor(-7.5) = 4088.
    # With the call starting at stream block 1 (block0 = 1) both blocks are late:
    #   block 0: rs(256, 3) = floor(32.5) = 32 -> 4128; block 1 as above -> 4088.
    # The outputs do not depend on the step (each block's outputs precede its update
    # and the two blocks use different filters).
    a = np.zeros((32, 4), np.int8)
    a[0, 0] = 8
    a[16, 1] = -4
    w = np.zeros((4, 4, 16), np.int16)
    w[0, 0, 0] = 4096
    w[1, 1, 0] = 4096
    want_out = np.zeros((32, 4), np.int16)
    want_out[0, 0] = 256
    want_out[16, 1] = -128
    base = dict(out_shift=7, err_shift=16, mu_shift=0, const_unit=64, update_enable=1, mu_shift_late=3)
    for block0, w00, w11 in ((0, 4352, 4088), (1, 4128, 4088)):
        out, wf = O.aeq(a, w, O.params(**base, gear_blocks=1, block0=block0))
        assert np.array_equal(out, want_out)
        want_w = w.copy()
        want_w[0, 0, 0] = w00
        want_w[1, 1, 0] = w11
        assert np.array_equal(wf, want_w), block0


def test_aeq_step_schedule_reductions():
    # gear_blocks = 0, a gear beyond the stream, or mu_shift_late = mu_shift: the
    # plain update; a late step of 40 freezes the taps at gear_blocks, after which
    # the outputs are the fixed FIR bank of those taps (numpy, update disabled).
    ch = synth.gen_channel(16 * 300, 40.0, 24.0, seed=42)
    _, a = O.cdc(ch.samples, ch.taps, ch.requant_shift)
    w0 = synth.centre_spike_taps()
    p = dict(out_shift=7, err_shift=16, mu_shift=3, const_unit=synth.aeq_params_for(ch)["const_unit"])
    ref_out, ref_w = O.aeq(a, w0, O.params(**p))
    for extra in (dict(gear_blocks=0, mu_shift_late=9), dict(gear_blocks=10 ** 6, mu_shift_late=9),
                  dict(gear_blocks=5, mu_shift_late=3), dict(gear_blocks=5, mu_shift_late=3, block0=77)):
        out, wf = O.aeq(a, w0, O.params(**p, **extra))
        assert np.array_equal(out, ref_out) and np.array_equal(wf, ref_w), extra
    G = 40
    frozen_out, frozen_w = O.aeq(a, w0, O.params(**p, gear_blocks=G, mu_shift_late=40))
    head_out, head_w = O.aeq(a[:16 * G], w0, O.params(**p))
    assert np.array_equal(frozen_w, head_w)
    assert np.array_equal(frozen_out[:16 * G], head_out)
    y = np.zeros((a.shape[0], 4), np.int64)
    x = a.astype(np.int64)
    for s2 in range(4):
        for s1 in range(4):
            y[:, s2] += np.convolve(x[:, s1], head_w[s1, s2].astype(np.int64))[: a.shape[0]]
    yh = np.clip(np.floor((y + 64) / 128), -32768, 32767).astype(np.int16)   # rs(y, 7), sat16
    assert np.array_equal(frozen_out[16 * G:], yh[16 * G:])


def test_aeq_step_schedule_changes_the_result():
    # a step that does change after gear_blocks gives other taps than either step alone
    ch = synth.gen_channel(16 * 200, 60.0, 24.0, seed=43)
    _, a = O.cdc(ch.samples, ch.taps, ch.requant_shift)
    w0 = synth.centre_spike_taps()
    p = dict(out_shift=7, err_shift=16, const_unit=synth.aeq_params_for(ch)["const_unit"])
    _, w_a = O.aeq(a, w0, O.params(**p, mu_shift=3))
    _, w_b = O.aeq(a, w0, O.params(**p, mu_shift=6))
    _, w_g = O.aeq(a, w0, O.params(**p, mu_shift=3, mu_shift_late=6, gear_blocks=50))
    assert not np.array_equal(w_g, w_a) and not np.array_equal(w_g, w_b)
