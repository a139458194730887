"""CPU oracle for the FNT-CDC + FNT-AEQ receiver path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and never imports it.

* ``fnt_ref``  -- Eqs. (1)-(2), the radix and modulus, and single-block models
  of Eqs. (7)-(8) and of the 7+7-bit tap split, in Python integers.
* ``_oracle.so`` (built from ``oracle.c`` with gcc) -- the exact integer
  CDC, resampling/requantisation and AEQ with its block RDE update, by their
  plain definitions, used through the numpy wrappers below.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import fnt_ref  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

AEQ_TAPS = 16
AEQ_BLOCK = 16
CDC_HIST = 32


class AeqParams(ctypes.Structure):
    _fields_ = [("out_shift", ctypes.c_int32), ("err_shift", ctypes.c_int32),
                ("mu_shift", ctypes.c_int32), ("const_unit", ctypes.c_int32),
                ("update_enable", ctypes.c_int32), ("mu_shift_late", ctypes.c_int32),
                ("gear_blocks", ctypes.c_int32), ("block0", ctypes.c_int64)]


class _Channel(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("n", ctypes.c_int64), ("taps", ctypes.c_void_p),
                ("ntaps", ctypes.c_int32), ("shift", ctypes.c_int32), ("phase", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("w", ctypes.c_void_p), ("a_buf", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("aeq", AeqParams)]


def lib():
    global _LIB
    if _LIB is None:
        from . import build as _b
        path = _b.build(force=False)
        L = ctypes.CDLL(path)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.orc_cdc.argtypes = [vp, i64, vp, i32, i32, i32, vp, vp, vp]
        L.orc_cdc.restype = None
        L.orc_aeq.argtypes = [vp, i64, vp, ctypes.POINTER(AeqParams), vp, vp]
        L.orc_aeq.restype = None
        L.orc_cdc_aeq.argtypes = [vp, i64, vp, i32, i32, i32, vp, vp,
                                  ctypes.POINTER(AeqParams), vp, vp, vp]
        L.orc_cdc_aeq.restype = None
        L.orc_batch.argtypes = [ctypes.POINTER(_Channel), i64, i32]
        L.orc_batch.restype = i32
        L.orc_rs.argtypes = [i64, i32]
        L.orc_rs.restype = i64
        L.orc_sat.argtypes = [i64, i32]
        L.orc_sat.restype = i64
        _LIB = L
    return _LIB


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c8(a, shape_tail):
    a = np.ascontiguousarray(a, dtype=np.int8)
    assert a.shape[1:] == shape_tail, a.shape
    return a


def params(out_shift, err_shift, mu_shift, const_unit, update_enable=1, mu_shift_late=None, gear_blocks=0,
           block0=0) -> AeqParams:
    """AEQ constants.  Step schedule: blocks with stream index block0 + b <
    gear_blocks update with mu_shift, later ones with mu_shift_late (gear_blocks
    = 0: mu_shift throughout)."""
    late = mu_shift if mu_shift_late is None else mu_shift_late
    return AeqParams(int(out_shift), int(err_shift), int(mu_shift), int(const_unit),
                     int(update_enable), int(late), int(gear_blocks), int(block0))


def n_symbols(n: int, phase: int = 0) -> int:
    """Number of 1 sample/symbol outputs for n instants: indices 2m + phase < n."""
    return max(0, (int(n) + 1 - int(phase)) // 2)


def rs(v: int, s: int) -> int:
    return int(lib().orc_rs(int(v), int(s)))


def sat(v: int, bits: int) -> int:
    return int(lib().orc_sat(int(v), int(bits)))


def cdc(samples, taps, shift: int, phase: int = 0, hist=None):
    """Exact CDC z (int32 [n][4]) and the resampled 5-bit stream a (int8 [M][4])."""
    x = _c8(samples, (4,))
    h = _c8(taps, (2,))
    n = x.shape[0]
    z = np.zeros((n, 4), np.int32)
    a = np.zeros((n_symbols(n, phase), 4), np.int8)
    hs = None if hist is None else _c8(hist, (4,))
    if hs is not None:
        assert hs.shape[0] == CDC_HIST
    lib().orc_cdc(_ptr(x), n, _ptr(h), h.shape[0], int(shift), int(phase), _ptr(hs), _ptr(z), _ptr(a))
    return z, a


def aeq(a, w, prm: AeqParams, hist=None):
    """AEQ over a (int8 [M][4]) from taps w (int16 [4][4][16]).  Returns (out, w_final)."""
    x = _c8(a, (4,))
    wf = np.ascontiguousarray(np.array(w, dtype=np.int16).reshape(4, 4, AEQ_TAPS)).copy()
    out = np.zeros((x.shape[0], 4), np.int16)
    hs = None if hist is None else _c8(hist, (4,))
    if hs is not None:
        assert hs.shape[0] == AEQ_TAPS
    p = prm
    lib().orc_aeq(_ptr(x), x.shape[0], _ptr(wf), ctypes.byref(p), _ptr(hs), _ptr(out))
    return out, wf


def cdc_aeq(samples, taps, shift: int, w, prm: AeqParams, phase: int = 0,
            cdc_hist=None, aeq_hist=None):
    """The whole chain on one channel.  Returns (out int16 [M][4], w_final, a int8 [M][4])."""
    x = _c8(samples, (4,))
    h = _c8(taps, (2,))
    n = x.shape[0]
    M = n_symbols(n, phase)
    wf = np.ascontiguousarray(np.array(w, dtype=np.int16).reshape(4, 4, AEQ_TAPS)).copy()
    a = np.zeros((M, 4), np.int8)
    out = np.zeros((M, 4), np.int16)
    ch = None if cdc_hist is None else _c8(cdc_hist, (4,))
    ah = None if aeq_hist is None else _c8(aeq_hist, (4,))
    p = prm
    lib().orc_cdc_aeq(_ptr(x), n, _ptr(h), h.shape[0], int(shift), int(phase), _ptr(ch),
                      _ptr(wf), ctypes.byref(p), _ptr(ah), _ptr(a), _ptr(out))
    return out, wf, a


def batch(channels, threads: int = 1):
    """Run many independent channels.  ``channels``: list of dicts with keys
    samples, taps, shift, phase, w, params.  Returns (outs, finals, threads_used)."""
    n = len(channels)
    arr = (_Channel * max(n, 1))()
    keep, outs, finals = [], [], []
    for i, c in enumerate(channels):
        x = _c8(c["samples"], (4,))
        h = _c8(c["taps"], (2,))
        ph = int(c.get("phase", 0))
        M = n_symbols(x.shape[0], ph)
        wf = np.ascontiguousarray(np.array(c["w"], dtype=np.int16).reshape(4, 4, AEQ_TAPS)).copy()
        ab = np.zeros((M, 4), np.int8)
        out = np.zeros((M, 4), np.int16)
        keep += [x, h, ab]
        outs.append(out)
        finals.append(wf)
        p = c["params"]
        arr[i] = _Channel(_ptr(x), x.shape[0], _ptr(h), h.shape[0], int(c["shift"]), ph, 0,
                          _ptr(wf), _ptr(ab), _ptr(out), p)
    used = lib().orc_batch(arr, n, int(threads))
    return outs, finals, int(used)
