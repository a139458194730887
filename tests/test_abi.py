"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/fnt.h declares, and the binding's structs match the C layouts."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2405_04253_amd import fnt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fnt.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fnt_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("fnt_forward", "fnt_inverse", "fnt_cdc", "fnt_aeq", "fnt_cdc_aeq", "fnt_check",
                 "fnt_plan_create", "fnt_plan_run", "fnt_session_create", "fnt_session_submit",
                 "fnt_session_get_state", "fnt_session_set_state", "fnt_session_destroy"):
        assert want in names


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(fnt.LIB_PATH):
        from paper_2405_04253_amd import build
        build.build(force=False)
    L = ctypes.CDLL(fnt.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(fnt.SIGNATURES), "binding and header disagree"
    lib = fnt.lib()
    assert lib.fnt_version() >= 10000
    assert lib.fnt_last_error() is not None


def test_struct_layouts_match_c():
    code = r'''
#include <stdio.h>
#include <stddef.h>
#include "fnt.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(fnt_cdc_params), sizeof(fnt_aeq_params),
         sizeof(fnt_channel_desc), sizeof(fnt_plan_config), sizeof(fnt_plan_info),
         sizeof(fnt_session_config), sizeof(fnt_session_stats), sizeof(fnt_request));
  printf("%zu %zu %zu\n", offsetof(fnt_channel_desc, cdc), offsetof(fnt_channel_desc, aeq),
         offsetof(fnt_plan_info, tune_ms));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "sz.c")
        exe = os.path.join(d, "sz")
        open(c, "w").write(code)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(v) for v in out]
    py = [ctypes.sizeof(t) for t in (fnt.CdcParams, fnt.AeqParams, fnt.ChannelDesc, fnt.PlanConfig,
                                     fnt.PlanInfo, fnt.SessionConfig, fnt.SessionStats, fnt.Request)]
    assert sizes[:8] == py
    assert sizes[8:] == [fnt.ChannelDesc.cdc.offset, fnt.ChannelDesc.aeq.offset, fnt.PlanInfo.tune_ms.offset]


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(fnt, "_LIB", None)
    monkeypatch.setattr(fnt, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        fnt.lib()


def test_cdc_params_marshalling():
    import numpy as np
    taps = np.array([[1, -2], [31, -32], [0, 5]], np.int8)
    p = fnt.cdc_params(taps, 7, 1)
    assert p.ntaps == 3 and p.requant_shift == 7 and p.decim_phase == 1
    assert [p.taps[k][c] for k in range(3) for c in range(2)] == [1, -2, 31, -32, 0, 5]
    assert fnt.n_symbols(33, 0) == 17 and fnt.n_symbols(33, 1) == 16 and fnt.n_symbols(0, 1) == 0
