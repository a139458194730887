"""The measurement probe library (libfntprobe.so) that supplies bench.py's
measured ceilings: it exports its two calls, and on a GPU both report rates in
a plausible range (bounded above by the published peaks with a margin)."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_04253_amd", "libfntprobe.so")


def test_probe_library_exports():
    if not os.path.exists(LIB):
        pytest.skip("probe library not built")
    lib = ctypes.CDLL(LIB)
    for name in ("fntprobe_alu", "fntprobe_copy"):
        assert hasattr(lib, name), name


@pytest.mark.gpu
def test_probe_rates():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = ctypes.CDLL(LIB)
    dev = torch.device("cuda:0")
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sink = torch.empty(1024 * 256, dtype=torch.int32, device=dev)
    rates = []
    for form in (0, 1):
        r = ctypes.c_double(0)
        assert lib.fntprobe_alu(form, ctypes.c_void_p(sink.data_ptr()), 1024, 64, ctypes.byref(r), sp) == 0
        rates.append(r.value)
    assert lib.fntprobe_alu(2, ctypes.c_void_p(sink.data_ptr()), 1, 1, ctypes.byref(ctypes.c_double()), sp) == -1
    src = torch.zeros(1 << 26, dtype=torch.uint8, device=dev)
    dst = torch.ones_like(src)
    bw = ctypes.c_double(0)
    assert lib.fntprobe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                             ctypes.c_size_t(1 << 26), ctypes.byref(bw), sp) == 0
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    print(f"[case] probe: add {rates[0] / 1e12:.1f} T, sdwa {rates[1] / 1e12:.1f} T lane-ops/s, "
          f"copy {bw.value / 1e12:.2f} TB/s", flush=True)
    assert 1e12 < rates[1] <= rates[0] < 1.2 * 78.6e12
    assert 1e11 < bw.value < 1.2 * 8e12
