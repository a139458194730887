"""Python binding of libfnt (include/fnt.h): argument marshalling only.

Every step of the receiver path runs in the HIP kernels of ``libfnt.so``;
PyTorch only provides device memory (tensors) and streams.  There is no CPU
fallback: if the library is missing, :func:`lib` raises.

Names follow the C ABI: ``fnt_forward``, ``fnt_inverse``, ``fnt_cdc``,
``fnt_aeq``, ``fnt_cdc_aeq``, ``fnt_check``, ``Plan`` (fnt_plan_*) and
``Session`` (fnt_session_*).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfnt.so")
_LIB = None

FNT_OK, FNT_E_INVAL, FNT_E_RANGE, FNT_E_NOMEM, FNT_E_DEVICE, FNT_E_BUSY, FNT_E_STATE = range(7)
FNT_ALPHA_2, FNT_ALPHA_SQRT2 = 0, 1
FNT_SUBMIT_HOST = 1
FNT_STATE_BYTES = 768
FNT_STAGE_CDC, FNT_STAGE_AEQ, FNT_STAGE_ALL = 1, 2, 3
FNT_NOALLOC_MAX_CHANNELS = 4096
_ERR_NAMES = {1: "FNT_E_INVAL", 2: "FNT_E_RANGE", 3: "FNT_E_NOMEM", 4: "FNT_E_DEVICE",
              5: "FNT_E_BUSY", 6: "FNT_E_STATE"}


class FntError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class CdcParams(ctypes.Structure):
    _fields_ = [("taps", (ctypes.c_int8 * 2) * 32), ("ntaps", ctypes.c_int32),
                ("requant_shift", ctypes.c_int32), ("decim_phase", ctypes.c_int32)]


class AeqParams(ctypes.Structure):
    _fields_ = [("out_shift", ctypes.c_int32), ("err_shift", ctypes.c_int32),
                ("mu_shift", ctypes.c_int32), ("const_unit", ctypes.c_int32),
                ("update_enable", ctypes.c_int32), ("mu_shift_late", ctypes.c_int32),
                ("gear_blocks", ctypes.c_uint32)]


class ChannelDesc(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("taps", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("cdc", CdcParams), ("aeq", AeqParams)]


class PlanConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tune_quick", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_uint64), ("instants", ctypes.c_uint64),
                ("symbols", ctypes.c_uint64), ("cdc_blocks", ctypes.c_uint64),
                ("aeq_blocks_max", ctypes.c_uint64), ("cdc_waves_per_group", ctypes.c_int32),
                ("cdc_blocks_per_wave", ctypes.c_int32), ("aeq_variant", ctypes.c_int32),
                ("aeq_waves_per_pol", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("aeq_waves_long", ctypes.c_int32), ("tune_ms", ctypes.c_double),
                ("aeq_long_channels", ctypes.c_uint64), ("cdc_variant", ctypes.c_int32),
                ("lead_channels", ctypes.c_int32), ("lead_form", ctypes.c_int32),
                ("top_channels", ctypes.c_int32), ("top_form", ctypes.c_int32),
                ("tune_run_ms", ctypes.c_double), ("fused_lpt", ctypes.c_int32),
                ("fused_grid", ctypes.c_int32), ("fused_prio_channels", ctypes.c_uint64),
                ("fused_split", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class PlanTiming(ctypes.Structure):
    _fields_ = [("step_ms", ctypes.c_float), ("cdc_ms", ctypes.c_float), ("aeq_ms", ctypes.c_float),
                ("aeq_lead_ms", ctypes.c_float), ("aeq_blocks", ctypes.c_uint64),
                ("aeq_lead_blocks", ctypes.c_uint64), ("aeq_top_ms", ctypes.c_float),
                ("fused", ctypes.c_int32), ("aeq_top_blocks", ctypes.c_uint64)]


class SessionConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_channels", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("chunk_blocks", ctypes.c_uint32),
                ("max_active", ctypes.c_uint32), ("aeq_form", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SessionStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("instants_done", ctypes.c_uint64), ("ticks", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("first_arrival_s", ctypes.c_double), ("last_completion_s", ctypes.c_double),
                ("gsamples_per_s", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("ch", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("n", ctypes.c_uint64), ("at_ns", ctypes.c_uint64)]


# every symbol declared in include/fnt.h, with (restype, argtypes)
_vp, _u64, _i32, _u32, _sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t
SIGNATURES = {
    "fnt_last_error": (ctypes.c_char_p, []),
    "fnt_version": (_i32, []),
    "fnt_check": (_i32, [_vp]),
    "fnt_forward": (_i32, [_vp, _vp, _sz, _i32, _i32, _i32, _vp]),
    "fnt_inverse": (_i32, [_vp, _vp, _sz, _i32, _i32, _i32, _vp]),
    "fnt_cdc": (_i32, [_vp, _u64, ctypes.POINTER(CdcParams), _vp, _vp, _vp]),
    "fnt_cdc_long": (_i32, [_vp, _u64, _vp, _i32, _i32, _i32, _vp, _vp, _vp]),
    "fnt_aeq": (_i32, [_vp, _u64, _vp, ctypes.POINTER(AeqParams), _vp, _vp]),
    "fnt_cdc_aeq": (_i32, [_vp, _u64, ctypes.POINTER(CdcParams), _vp, ctypes.POINTER(AeqParams), _vp, _vp]),
    "fnt_plan_create": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(ChannelDesc), _sz,
                               ctypes.POINTER(PlanConfig), _vp]),
    "fnt_plan_run": (_i32, [_vp, _vp]),
    "fnt_plan_run_graph": (_i32, [_vp, _vp]),
    "fnt_plan_run_stage": (_i32, [_vp, _i32, _vp]),
    "fnt_plan_get_info": (_i32, [_vp, ctypes.POINTER(PlanInfo)]),
    "fnt_plan_set_aeq_variant": (_i32, [_vp, _i32]),
    "fnt_plan_set_cdc_variant": (_i32, [_vp, _i32]),
    "fnt_plan_set_aeq_waves": (_i32, [_vp, _i32]),
    "fnt_plan_set_cdc_schedule": (_i32, [_vp, _i32, _i32]),
    "fnt_plan_set_aeq_split": (_i32, [_vp, _u64, _i32, _i32]),
    "fnt_plan_set_lead": (_i32, [_vp, _u64, _i32, _u64, _i32]),
    "fnt_plan_set_fused": (_i32, [_vp, _i32, _u64, _i32]),
    "fnt_plan_run_timed": (_i32, [_vp, ctypes.POINTER(PlanTiming), _vp]),
    "fnt_plan_destroy": (_i32, [_vp]),
    "fnt_cdc_aeq_batch_noalloc": (_i32, [_vp, _u32, _vp]),
    "fnt_now_ns": (_u64, []),
    "fnt_session_create": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(SessionConfig)]),
    "fnt_session_add_channel": (_i32, [_vp, _u32, ctypes.POINTER(CdcParams), ctypes.POINTER(AeqParams), _vp]),
    "fnt_session_submit": (_i32, [_vp, _u32, _vp, _u64, _vp, _u32, _u64, ctypes.POINTER(_u64)]),
    "fnt_session_replay": (_i32, [_vp, ctypes.POINTER(Request), _sz, ctypes.POINTER(_u64)]),
    "fnt_session_poll": (_i32, [_vp, _u64, ctypes.POINTER(ctypes.c_int)]),
    "fnt_session_wait": (_i32, [_vp, _u64]),
    "fnt_session_drain": (_i32, [_vp]),
    "fnt_session_cancel": (_i32, [_vp, _u64]),
    "fnt_session_get_state": (_i32, [_vp, _u32, _vp, ctypes.POINTER(_sz)]),
    "fnt_session_set_state": (_i32, [_vp, _u32, _vp, _sz]),
    "fnt_session_get_stats": (_i32, [_vp, ctypes.POINTER(SessionStats)]),
    "fnt_session_destroy": (_i32, [_vp]),
}


def lib():
    """Load libfnt.so (raises if it has not been built: there is no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2405_04253_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _ok(rc):
    if rc != FNT_OK:
        raise FntError(rc, lib().fnt_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def cdc_params(taps, requant_shift: int, decim_phase: int = 0) -> CdcParams:
    taps = np.asarray(taps, dtype=np.int64)
    p = CdcParams()
    for k in range(taps.shape[0]):
        p.taps[k][0] = int(taps[k, 0])
        p.taps[k][1] = int(taps[k, 1])
    p.ntaps = int(taps.shape[0])
    p.requant_shift = int(requant_shift)
    p.decim_phase = int(decim_phase)
    return p


def aeq_params(out_shift, err_shift, mu_shift, const_unit, update_enable=1, mu_shift_late=None,
               gear_blocks=0) -> AeqParams:
    """fnt_aeq_params; the step schedule uses mu_shift_late from stream block
    gear_blocks on (gear_blocks = 0: mu_shift throughout)."""
    late = mu_shift if mu_shift_late is None else mu_shift_late
    return AeqParams(int(out_shift), int(err_shift), int(mu_shift), int(const_unit), int(update_enable),
                     int(late), int(gear_blocks))


def n_symbols(n: int, phase: int = 0) -> int:
    return max(0, (int(n) + 1 - int(phase)) // 2)


def _need(t, dtype, tail, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA/HIP tensor")
    if t.dtype != dtype or tuple(t.shape[1:]) != tail or not t.is_contiguous():
        raise TypeError(f"{name}: expected contiguous {dtype} [*, {tail}], got {t.dtype} {tuple(t.shape)}")


# ----------------------------------------------------------------- transforms --
def fnt_forward(x, t: int, log2n: int, alpha_kind: int, out=None, stream=None):
    """Eq. (1) on a batch: x int32 [batch, N] (canonical residues) on the GPU."""
    import torch
    _need(x, torch.int32, (1 << log2n,), "x")
    out = torch.empty_like(x) if out is None else out
    _ok(lib().fnt_forward(_ptr(x), _ptr(out), x.shape[0], t, log2n, alpha_kind, _stream(stream)))
    return out


def fnt_inverse(X, t: int, log2n: int, alpha_kind: int, out=None, stream=None):
    """Eq. (2) (with N^-1) on a batch: X int32 [batch, N] on the GPU."""
    import torch
    _need(X, torch.int32, (1 << log2n,), "X")
    out = torch.empty_like(X) if out is None else out
    _ok(lib().fnt_inverse(_ptr(X), _ptr(out), X.shape[0], t, log2n, alpha_kind, _stream(stream)))
    return out


def fnt_check(stream=None):
    """Synchronise and raise FntError(FNT_E_RANGE) if a kernel saw an out-of-range input."""
    _ok(lib().fnt_check(_stream(stream)))


# ---------------------------------------------------------------------- path --
def fnt_cdc(samples, params: CdcParams, exact: bool = True, one_sps: bool = True,
            z_out=None, a_out=None, stream=None):
    """FNT-CDC: samples int8 [n, 4] -> (z int32 [n, 4] or None, a int8 [M, 4] or None).
    Preallocated outputs may be passed as z_out / a_out."""
    import torch
    _need(samples, torch.int8, (4,), "samples")
    n = samples.shape[0]
    M = n_symbols(n, params.decim_phase)
    z = z_out if z_out is not None else (
        torch.empty((n, 4), dtype=torch.int32, device=samples.device) if exact else None)
    a = a_out if a_out is not None else (
        torch.empty((M, 4), dtype=torch.int8, device=samples.device) if one_sps else None)
    if z is not None:
        _need(z, torch.int32, (4,), "z_out")
        assert z.shape[0] == n
    if a is not None:
        _need(a, torch.int8, (4,), "a_out")
        assert a.shape[0] == M
    _ok(lib().fnt_cdc(_ptr(samples), n, ctypes.byref(params), _ptr(z), _ptr(a), _stream(stream)))
    return z, a


def fnt_cdc_long(samples, taps, requant_shift: int, decim_phase: int = 0, exact: bool = True,
                 one_sps: bool = True, stream=None):
    """fnt_cdc_long (N = 128, up to 65 taps): samples int8 [n, 4] on the GPU, taps
    int8 [L, 2] (host array) -> (z int32 [n, 4] or None, a int8 [M, 4] or None)."""
    import numpy as np
    import torch
    _need(samples, torch.int8, (4,), "samples")
    n = samples.shape[0]
    h = np.ascontiguousarray(np.asarray(taps, dtype=np.int8).reshape(-1, 2))
    z = torch.empty((n, 4), dtype=torch.int32, device=samples.device) if exact else None
    a = torch.empty((n_symbols(n, decim_phase), 4), dtype=torch.int8, device=samples.device) if one_sps else None
    _ok(lib().fnt_cdc_long(_ptr(samples), n, h.ctypes.data, h.shape[0], int(requant_shift), int(decim_phase),
                           _ptr(z), _ptr(a), _stream(stream)))
    return z, a


def fnt_aeq(a, taps, params: AeqParams, out=None, stream=None):
    """FNT-AEQ: a int8 [M, 4], taps int16 [4, 4, 16] (updated in place) -> out int16 [M, 4]."""
    import torch
    _need(a, torch.int8, (4,), "a")
    _need(taps, torch.int16, (4, 16), "taps")
    out = torch.empty((a.shape[0], 4), dtype=torch.int16, device=a.device) if out is None else out
    _need(out, torch.int16, (4,), "out")
    assert out.shape[0] == a.shape[0]
    _ok(lib().fnt_aeq(_ptr(a), a.shape[0], _ptr(taps), ctypes.byref(params), _ptr(out), _stream(stream)))
    return out


def fnt_cdc_aeq(samples, cdc: CdcParams, taps, aeq: AeqParams, out=None, stream=None):
    """The whole chain on one channel: samples int8 [n, 4] -> int16 [M, 4]; taps updated."""
    import torch
    _need(samples, torch.int8, (4,), "samples")
    _need(taps, torch.int16, (4, 16), "taps")
    M = n_symbols(samples.shape[0], cdc.decim_phase)
    out = torch.empty((M, 4), dtype=torch.int16, device=samples.device) if out is None else out
    _need(out, torch.int16, (4,), "out")
    assert out.shape[0] == M
    _ok(lib().fnt_cdc_aeq(_ptr(samples), samples.shape[0], ctypes.byref(cdc), _ptr(taps),
                          ctypes.byref(aeq), _ptr(out), _stream(stream)))
    return out


# --------------------------------------------------------------------- plans --
class Plan:
    """fnt_plan_*: many independent channels, one launch sequence (optionally a hipGraph)."""

    def __init__(self, channels, autotune=False, use_graph=True, tune_cache=None, stream=None, tune_quick=False):
        """channels: list of (samples int8 [n,4], out int16 [M,4], taps int16 [4,4,16],
        CdcParams, AeqParams) with all tensors on the GPU."""
        import torch
        self._keep = channels
        arr = (ChannelDesc * max(1, len(channels)))()
        for i, (x, out, taps, cp, ap) in enumerate(channels):
            _need(x, torch.int8, (4,), "samples")
            _need(out, torch.int16, (4,), "out")
            _need(taps, torch.int16, (4, 16), "taps")
            arr[i] = ChannelDesc(x.data_ptr(), out.data_ptr(), taps.data_ptr(), x.shape[0], cp, ap)
        dev = channels[0][0].device.index if channels else torch.cuda.current_device()
        cfg = PlanConfig(dev or 0, int(autotune), int(use_graph), int(tune_quick),
                         tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        _ok(lib().fnt_plan_create(ctypes.byref(h), arr, len(channels), ctypes.byref(cfg), _stream(stream)))
        self._h = h

    def run(self, stream=None):
        _ok(lib().fnt_plan_run(self._h, _stream(stream)))

    def run_graph(self, stream=None):
        """Replay the captured hipGraph whatever the schedule (fnt_plan_run_graph)."""
        _ok(lib().fnt_plan_run_graph(self._h, _stream(stream)))

    def run_stage(self, stages: int, stream=None):
        """Launch FNT_STAGE_CDC and/or FNT_STAGE_AEQ directly (outside the graph)."""
        _ok(lib().fnt_plan_run_stage(self._h, int(stages), _stream(stream)))

    def info(self) -> dict:
        inf = PlanInfo()
        _ok(lib().fnt_plan_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in PlanInfo._fields_}

    def set_aeq_variant(self, variant: int):
        _ok(lib().fnt_plan_set_aeq_variant(self._h, int(variant)))

    def set_cdc_variant(self, variant: int):
        _ok(lib().fnt_plan_set_cdc_variant(self._h, int(variant)))

    def set_aeq_waves(self, waves_per_pol: int):
        _ok(lib().fnt_plan_set_aeq_waves(self._h, int(waves_per_pol)))

    def set_aeq_split(self, long_channels: int, waves_long: int, waves: int):
        _ok(lib().fnt_plan_set_aeq_split(self._h, int(long_channels), int(waves_long), int(waves)))

    def set_cdc_schedule(self, waves_per_group: int, blocks_per_wave: int):
        _ok(lib().fnt_plan_set_cdc_schedule(self._h, int(waves_per_group), int(blocks_per_wave)))

    def set_lead(self, lead_channels: int, lead_form: int = -1, top_channels: int = 0, top_form: int = -1):
        _ok(lib().fnt_plan_set_lead(self._h, int(lead_channels), int(lead_form), int(top_channels),
                                    int(top_form)))

    def set_fused(self, lanes_per_transform: int, prio_channels: int = 0, split_halves: bool = False):
        """Every run as one launch of the fused CDC + AEQ kernel (0: off)."""
        _ok(lib().fnt_plan_set_fused(self._h, int(lanes_per_transform), int(prio_channels), int(split_halves)))

    def run_timed(self, stream=None) -> dict:
        """One run launched directly with events around every launch; blocks
        until it ends and returns the durations (ms) and block counts."""
        t = PlanTiming()
        _ok(lib().fnt_plan_run_timed(self._h, ctypes.byref(t), _stream(stream)))
        return {k: getattr(t, k) for k, _ in PlanTiming._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().fnt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def channel_table(channels) -> bytes:
    """fnt_channel_desc[] bytes for channels given as (samples, out, taps,
    CdcParams, AeqParams) tensors, as Plan takes them."""
    arr = (ChannelDesc * max(1, len(channels)))()
    for i, (x, out, taps, cp, ap) in enumerate(channels):
        arr[i] = ChannelDesc(x.data_ptr(), out.data_ptr(), taps.data_ptr(), x.shape[0], cp, ap)
    return bytes(arr)[: ctypes.sizeof(ChannelDesc) * len(channels)]


def fnt_cdc_aeq_batch_noalloc(dev_table, nch: int, stream=None):
    """dev_table: uint8 device tensor holding fnt_channel_desc[nch] (channel_table)."""
    _ok(lib().fnt_cdc_aeq_batch_noalloc(ctypes.c_void_p(dev_table.data_ptr() if nch else 0), int(nch),
                                       _stream(stream)))


# ------------------------------------------------------------------ sessions --
class Session:
    """fnt_session_*: continuing channel streams with HBM-resident state."""

    def __init__(self, max_channels: int, hbm_budget_bytes: int, chunk_blocks: int = 0,
                 max_active: int = 0, device: int = 0, aeq_form: int = -1):
        cfg = SessionConfig(int(device), int(max_channels), int(hbm_budget_bytes),
                            int(chunk_blocks), int(max_active), int(aeq_form), 0)
        h = ctypes.c_void_p()
        _ok(lib().fnt_session_create(ctypes.byref(h), ctypes.byref(cfg)))
        self._h = h

    def add_channel(self, ch: int, cdc: CdcParams, aeq: AeqParams, init_taps=None):
        buf = None
        if init_taps is not None:
            t = np.ascontiguousarray(np.asarray(init_taps, dtype=np.int16).reshape(256))
            buf = t.ctypes.data_as(ctypes.c_void_p)
            self._tmp = t
        _ok(lib().fnt_session_add_channel(self._h, ch, ctypes.byref(cdc), ctypes.byref(aeq), buf))

    def submit(self, ch: int, samples, out, host: bool = False, arrival_ns: int = 0) -> int:
        """samples: int8 [n, 4] (n a multiple of 32), out: int16 [n/2, 4]; GPU tensors, or
        C-contiguous numpy arrays with host=True (kept alive until completion by the caller)."""
        tk = ctypes.c_uint64()
        if host:
            pin, pout = samples.ctypes.data, out.ctypes.data
            n = samples.shape[0]
            flags = FNT_SUBMIT_HOST
        else:
            pin, pout, n, flags = samples.data_ptr(), out.data_ptr(), samples.shape[0], 0
        _ok(lib().fnt_session_submit(self._h, ch, pin, n, pout, flags, arrival_ns, ctypes.byref(tk)))
        return tk.value

    def replay(self, reqs, host: bool = False):
        """reqs: list of (ch, samples, out, at_ns) with GPU tensors, or with host
        (preferably pinned) CPU tensors when host=True; returns tickets."""
        arr = (Request * max(1, len(reqs)))()
        flags = FNT_SUBMIT_HOST if host else 0
        for i, (ch, x, o, at) in enumerate(reqs):
            arr[i] = Request(ch, flags, x.data_ptr(), o.data_ptr(), x.shape[0], int(at))
        tks = (ctypes.c_uint64 * max(1, len(reqs)))()
        _ok(lib().fnt_session_replay(self._h, arr, len(reqs), tks))
        return list(tks)[: len(reqs)]

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _ok(lib().fnt_session_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        _ok(lib().fnt_session_wait(self._h, ticket))

    def drain(self):
        _ok(lib().fnt_session_drain(self._h))

    def cancel(self, ticket: int):
        _ok(lib().fnt_session_cancel(self._h, ticket))

    def get_state(self, ch: int) -> bytes:
        buf = ctypes.create_string_buffer(FNT_STATE_BYTES)
        sz = ctypes.c_size_t(FNT_STATE_BYTES)
        _ok(lib().fnt_session_get_state(self._h, ch, buf, ctypes.byref(sz)))
        return buf.raw[: sz.value]

    def set_state(self, ch: int, state: bytes):
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        _ok(lib().fnt_session_set_state(self._h, ch, buf, len(state)))

    def stats(self) -> dict:
        st = SessionStats()
        _ok(lib().fnt_session_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in SessionStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            rc = lib().fnt_session_destroy(self._h)
            self._h = None
            _ok(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now_ns() -> int:
    return int(lib().fnt_now_ns())
