"""Equaliser quality on synthetic PDM-16QAM: symbol error rate (SER) of the
integer FNT receiver against float64 reference receivers on the same channels.

The experimental section of the paper compares the FNT-based CDC and AEQ with
conventional floating-point processing by the OSNR each needs for a given error
rate.  The lab captures are not available; this module reproduces the shape of
that comparison on the synthetic channels of ``synth``:

* ``float_ideal``: the received signal before the 5-bit rounding, CD removed in
  the frequency domain (the exact inverse of the channel's dispersion over the
  circular stream), then a float64 4x4 real-valued MIMO equaliser with the
  structure of the FNT-AEQ (16 taps, blocks of 16 symbols, one block-LMS update
  per block with the radius-directed error of Eq. (6) and the same ring
  decisions), sampled at one sample per symbol;
* ``float_5bit``: the same float receiver on the 5-bit samples;
* ``fnt_<err_shift>_<mu_shift>[_<mu_shift_late>_<gear_blocks>]``: the integer
  path of this library on the GPU (FNT-CDC with 6-bit taps and 5-bit
  requantisation, FNT-AEQ with 14-bit taps in two 7-bit digits), with the given
  RDE step shifts (and step schedule).

Every output stream first passes a blind carrier-phase recovery (the fourth-power
estimator of Viterbi and Viterbi over a sliding window, unwrapped), which only
matters when the channel carries laser phase noise (``--linewidth``); it is then
aligned to the transmitted symbols by a data-aided search (delay, polarisation,
a complex gain, and conjugation, which a real-valued 4x4 MIMO may converge to),
decided to the nearest 16QAM point, and the SER and the BER (Gray-mapped levels,
two bits per dimension) count the second half of the stream (after convergence).

``python -m paper_2405_04253_amd.quality --osnr 14,16,18,20,22,24`` prints one
JSON line per OSNR and the OSNR each receiver needs for a target SER.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import synth

LEVELS = np.array([-3.0, -1.0, 1.0, 3.0])
BLOCK = 16
NTAPS = 16


# ------------------------------------------------------------ float receiver --
def fd_cdc(rx: np.ndarray, fibre_km: float) -> np.ndarray:
    """Frequency-domain CD compensation of a 2-sps dual-pol stream float [n][4]
    (circular over n) -> complex [2][n]."""
    n = rx.shape[0]
    f = np.fft.fftfreq(n) * synth.BAUD * synth.SPS
    h = np.exp(1j * synth.dispersion_beta(fibre_km) * f * f)
    out = np.empty((2, n), np.complex128)
    for p in range(2):
        z = rx[:, 2 * p].astype(np.float64) + 1j * rx[:, 2 * p + 1].astype(np.float64)
        out[p] = np.fft.ifft(np.fft.fft(z) * h)
    return out


def float_aeq(z1: np.ndarray, mu: float = 1e-5, centre: int = 8, cma_blocks: int = 2048) -> np.ndarray:
    """Float64 4x4 real MIMO block-LMS equaliser on a 1-sps complex [2][m] stream
    normalised to the 16QAM grid (levels +-1, +-3): the constant-modulus error
    (radius^2 = E|s|^4 / E|s|^2 = 13.2) for the first `cma_blocks` blocks, as a
    conventional receiver pre-converges, then the radius-directed error of
    Eq. (6).  Returns complex [2][m]."""
    m = z1.shape[1]
    x = np.stack([z1[0].real, z1[0].imag, z1[1].real, z1[1].imag])           # [4][m]
    nb = (m + BLOCK - 1) // BLOCK
    xp = np.zeros((4, NTAPS - 1 + nb * BLOCK))
    xp[:, NTAPS - 1:NTAPS - 1 + m] = x
    # win[b][s][j][k] = x_s[16 b + j - k]
    idx = (np.arange(nb)[:, None, None] * BLOCK + np.arange(BLOCK)[None, :, None]
           - np.arange(NTAPS)[None, None, :] + NTAPS - 1)
    w = np.zeros((4, 4, NTAPS))
    for s in range(4):
        w[s, s, centre] = 1.0
    y_all = np.empty((4, nb * BLOCK))
    for b in range(nb):
        win = xp[:, idx[b]]                                                  # [4][16][16]
        y = np.einsum("sjk,stk->tj", win, w)                                 # [4 S2][16]
        y_all[:, b * BLOCK:(b + 1) * BLOCK] = y
        r2 = y[0::2] ** 2 + y[1::2] ** 2                                     # [2 pol][16]
        if b < cma_blocks:
            R2 = np.full_like(r2, 13.2)
        else:
            R2 = np.where(r2 < 6, 2.0, np.where(r2 < 14, 10.0, 18.0))
        e = np.repeat(R2 - r2, 2, axis=0) * y                                # [4 S2][16]
        valid = (b * BLOCK + np.arange(BLOCK)) < m
        e[:, ~valid] = 0.0
        w += mu * np.einsum("tj,sjk->stk", e, win)
    y_all = y_all[:, :m]
    return np.stack([y_all[0] + 1j * y_all[1], y_all[2] + 1j * y_all[3]])


def _normalise(z1: np.ndarray) -> np.ndarray:
    """Scale each polarisation to the 16QAM grid's mean power (10)."""
    return z1 * np.sqrt(10.0 / np.mean(np.abs(z1) ** 2, axis=1, keepdims=True))


def float_receiver(rx: np.ndarray, fibre_km: float, nsym: int, mu: float = 1e-5,
                   cma_blocks: int = 2048) -> np.ndarray:
    z = fd_cdc(rx, fibre_km)[:, 0:2 * nsym:2]                                # 1 sps, phase 0
    return float_aeq(_normalise(z), mu, cma_blocks=cma_blocks)


# ------------------------------------------------------ carrier recovery --
def cpe_4th_power(y: np.ndarray, window: int = 128) -> np.ndarray:
    """Blind carrier-phase recovery of complex [2][m]: per symbol, the phase of the
    window's sum of y^4 (for square 16QAM E[s^4] is a negative real number, so
    arg(-sum y^4) = 4 theta), unwrapped over the stream; returns y e^{-j theta}.
    The estimate is ambiguous by multiples of pi/2, which the alignment's complex
    gain absorbs."""
    out = np.empty_like(y)
    k = np.ones(window)
    for q in range(y.shape[0]):
        acc = np.convolve(y[q] ** 4, k, mode="same")
        theta = np.unwrap(np.angle(-acc)) / 4
        out[q] = y[q] * np.exp(-1j * theta)
    return out


# ---------------------------------------------------------------------- SER --
def gray_bits(levels: np.ndarray) -> np.ndarray:
    """Gray code of the 16QAM levels -3, -1, 1, 3 per dimension: 00, 01, 11, 10."""
    idx = np.rint((np.asarray(levels, np.float64) + 3) / 2).astype(np.int64)
    return idx ^ (idx >> 1)


def tx_complex(symbols: np.ndarray) -> np.ndarray:
    s = symbols.astype(np.float64)
    return np.stack([s[:, 0] + 1j * s[:, 1], s[:, 2] + 1j * s[:, 3]])


def align_and_count(y: np.ndarray, symbols: np.ndarray, max_delay: int = 48) -> dict:
    """SER and BER of equalised complex [2][m] against the transmitted levels
    int8 [n][4] over the second half of the stream, after a data-aided search for
    delay, polarisation, complex gain and conjugation per output."""
    s = tx_complex(symbols)
    m = min(y.shape[1], s.shape[1])
    lo, hi = m // 2, m - max_delay
    errors, bit_errors, count, picks = 0, 0, 0, []
    for q in range(2):
        yq = y[q, lo:hi]
        best = None
        for p in range(2):
            for conj in (False, True):
                sp = np.conj(s[p]) if conj else s[p]
                for d in range(-max_delay, max_delay + 1):
                    ref = sp[lo - d:hi - d]
                    c = np.vdot(ref, yq)
                    score = abs(c)
                    if best is None or score > best[0]:
                        best = (score, p, conj, d, c / np.vdot(ref, ref))
        _, p, conj, d, g = best
        ref = (np.conj(s[p]) if conj else s[p])[lo - d:hi - d]
        yn = yq / g
        dec = LEVELS[np.abs(yn.real[:, None] - LEVELS[None, :]).argmin(1)] + \
            1j * LEVELS[np.abs(yn.imag[:, None] - LEVELS[None, :]).argmin(1)]
        errors += int(np.count_nonzero(dec != ref))
        for part in (np.real, np.imag):
            diff = gray_bits(part(dec)) ^ gray_bits(part(ref))
            bit_errors += int(np.sum((diff & 1) + (diff >> 1)))
        count += ref.shape[0]
        picks.append(dict(out=q, tx=p, conj=conj, delay=d))
    return dict(ser=errors / max(count, 1), ber=bit_errors / max(4 * count, 1), errors=errors,
                bit_errors=bit_errors, symbols=count, alignment=picks)


# -------------------------------------------------------------- FNT receiver --
def fnt_receiver(ch: synth.Channel, **aeq_overrides) -> np.ndarray:
    """The library's integer path on the GPU -> complex [2][m] (int16 outputs).
    aeq_overrides replace fields of the channel's default AEQ parameters."""
    import torch
    from . import fnt
    dev = torch.device("cuda:0")
    x = torch.from_numpy(ch.samples).to(dev)
    taps = torch.from_numpy(synth.centre_spike_taps()).to(dev)
    prm = dict(synth.aeq_params_for(ch), **aeq_overrides)
    out = fnt.fnt_cdc_aeq(x, fnt.cdc_params(ch.taps, ch.requant_shift), taps, fnt.aeq_params(**prm))
    torch.cuda.synchronize()
    fnt.fnt_check()
    o = out.cpu().numpy().astype(np.float64)
    return np.stack([o[:, 0] + 1j * o[:, 1], o[:, 2] + 1j * o[:, 3]])


def required_osnr(osnrs, sers, target: float) -> float | None:
    """OSNR (dB) where the SER curve crosses `target`, by log-linear interpolation."""
    pts = [(o, s) for o, s in zip(osnrs, sers) if s > 0]
    for (o0, s0), (o1, s1) in zip(pts, pts[1:]):
        if s0 >= target >= s1:
            t = (math.log10(s0) - math.log10(target)) / max(math.log10(s0) - math.log10(s1), 1e-12)
            return o0 + t * (o1 - o0)
    return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--osnr", default="14,16,18,20,22,24")
    ap.add_argument("--nsym", type=int, default=1 << 18)
    ap.add_argument("--aeq", default="16:4:6:2048,16:4,16:5,16:3",
                    help="AEQ settings of the integer receiver, comma separated: err_shift:mu_shift "
                         "(one step) or err_shift:mu_shift:mu_shift_late:gear_blocks (step schedule)")
    ap.add_argument("--km", type=float, default=75.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--target", type=float, default=1e-2)
    ap.add_argument("--linewidth", type=float, default=0.0, help="combined laser linewidth, Hz")
    ap.add_argument("--cpe-window", type=int, default=128)
    ap.add_argument("--no-gpu", action="store_true", help="float receivers only")
    args = ap.parse_args(argv)
    osnrs = [float(v) for v in args.osnr.split(",")]
    settings = []
    for a in args.aeq.split(","):
        v = [int(x) for x in a.split(":")] if a else []
        if len(v) == 2:
            settings.append((f"fnt_{v[0]}_{v[1]}", dict(err_shift=v[0], mu_shift=v[1], gear_blocks=0)))
        elif len(v) == 4:
            settings.append((f"fnt_{v[0]}_{v[1]}_{v[2]}_{v[3]}",
                             dict(err_shift=v[0], mu_shift=v[1], mu_shift_late=v[2], gear_blocks=v[3])))
    curves = {"float_ideal": [], "float_5bit": []}
    for name, _ in settings:
        curves[name] = []
    for o in osnrs:
        ch = synth.gen_channel(args.nsym, args.km, o, synth.seed_for(args.seed, "quality", o), keep_float=True,
                               linewidth_hz=args.linewidth)
        row = {"osnr_db": o, "fibre_km": args.km, "nsym": args.nsym, "linewidth_hz": args.linewidth,
               "ser": {}, "ber": {}}
        outs = {"float_ideal": lambda: float_receiver(ch.float_rx, args.km, args.nsym),
                "float_5bit": lambda: float_receiver(ch.samples, args.km, args.nsym)}
        if not args.no_gpu:
            for name, ov in settings:
                outs[name] = (lambda ov=ov: fnt_receiver(ch, **ov))
        for name, run in outs.items():
            r = align_and_count(cpe_4th_power(run(), args.cpe_window), ch.symbols)
            row["ser"][name], row["ber"][name] = r["ser"], r["ber"]
            curves[name].append(r["ser"])
        print(json.dumps(row), flush=True)
    need = {k: required_osnr(osnrs, v, args.target) for k, v in curves.items() if v}
    print(json.dumps({"target_ser": args.target, "required_osnr_db": need}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
