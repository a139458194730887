"""GPU: fnt_cdc_aeq_batch_noalloc (no allocation; tables and work counter in the
library's fixed device array) against fnt_plan_run with the fused schedule on
the same channels, bit-exactly, on two calls in a row, the second smaller."""
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


def make_channels(torch, dev, rng, nch, nlong):
    """nlong channels of 2-5 chunks of CDC (long chains) and short ragged ones."""
    chans = []
    for k in range(nch):
        n = int(rng.integers(2 * 2048, 5 * 2048)) if k < nlong else int(rng.integers(0, 600))
        phase = int(rng.integers(0, 2))
        ntaps = int(rng.integers(1, 33))
        x = rng.integers(-16, 16, size=(n, 4)).astype(np.int8)
        taps = rng.integers(-32, 32, size=(ntaps, 2)).astype(np.int8)
        w0 = (synth.centre_spike_taps() if k % 2 else
              rng.integers(-500, 500, size=(4, 4, 16)).astype(np.int16))
        prm = dict(out_shift=int(rng.integers(4, 10)), err_shift=int(rng.integers(10, 20)),
                   mu_shift=int(rng.integers(1, 6)), const_unit=int(rng.integers(20, 90)), update_enable=1)
        M = O.n_symbols(n, phase)
        chans.append(dict(x=torch.from_numpy(x).to(dev), xs=x, taps=taps, shift=int(rng.integers(4, 10)),
                          phase=phase, w0=w0, prm=prm,
                          out=torch.full((M, 4), 777, dtype=torch.int16, device=dev),
                          t=torch.from_numpy(w0).to(dev)))
    return chans


def entries(chans, out_key="out", taps_key="t"):
    return [(c["x"], c[out_key], c[taps_key], fnt.cdc_params(c["taps"], c["shift"], c["phase"]),
             fnt.aeq_params(**c["prm"])) for c in chans]


def plan_reference(torch, dev, chans):
    """The existing entry point: fnt_plan_run with the fused schedule."""
    for c in chans:
        c["ref_out"] = torch.full_like(c["out"], 555)
        c["ref_t"] = torch.from_numpy(c["w0"]).to(dev)
    plan = fnt.Plan(entries(chans, "ref_out", "ref_t"), autotune=False, use_graph=False)
    plan.set_fused(4, 512)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    fnt.fnt_check()


def test_noalloc_two_calls_vs_fused_plan(torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(2024)
    big = make_channels(torch, dev, rng, 1300, 20)      # more than the fused kernel keeps resident
    small = make_channels(torch, dev, rng, 90, 4)
    note("noalloc: fused plan references")
    plan_reference(torch, dev, big)
    plan_reference(torch, dev, small)
    tab_big = torch.frombuffer(bytearray(fnt.channel_table(entries(big))), dtype=torch.uint8).to(dev)
    tab_small = torch.frombuffer(bytearray(fnt.channel_table(entries(small))), dtype=torch.uint8).to(dev)
    stream = torch.cuda.current_stream()
    note(f"noalloc: call 1 ({len(big)} channels) then call 2 ({len(small)} channels)")
    fnt.fnt_cdc_aeq_batch_noalloc(tab_big, len(big), stream)
    fnt.fnt_cdc_aeq_batch_noalloc(tab_small, len(small), stream)
    torch.cuda.synchronize()
    fnt.fnt_check()
    for name, chans in (("call 1", big), ("call 2", small)):
        for i, c in enumerate(chans):
            assert torch.equal(c["out"], c["ref_out"]), (name, i, c["xs"].shape[0])
            assert torch.equal(c["t"], c["ref_t"]), (name, i, c["xs"].shape[0])
    # and the oracle on a few channels of each call, the longest first
    for chans in (big, small):
        for c in chans[:3] + chans[-2:]:
            outr, wr, _ = O.cdc_aeq(c["xs"], c["taps"], c["shift"], c["w0"], O.params(**c["prm"]), phase=c["phase"])
            assert np.array_equal(c["out"].cpu().numpy(), outr)
            assert np.array_equal(c["t"].cpu().numpy(), wr)


def test_noalloc_limits_and_invalid_descriptor(torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(7)
    chans = make_channels(torch, dev, rng, 12, 2)
    tab = torch.frombuffer(bytearray(fnt.channel_table(entries(chans))), dtype=torch.uint8).to(dev)
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_cdc_aeq_batch_noalloc(tab, fnt.FNT_NOALLOC_MAX_CHANNELS + 1)
    assert e.value.code == fnt.FNT_E_INVAL
    # channel 5 gets ntaps = 0: reported, skipped (its output untouched), the others right
    bad = fnt.channel_table(entries(chans))
    raw = bytearray(bad)
    desc = fnt.ChannelDesc.from_buffer(raw, 5 * fnt.ctypes.sizeof(fnt.ChannelDesc))
    desc.cdc.ntaps = 0
    tab_bad = torch.frombuffer(raw, dtype=torch.uint8).to(dev)
    note("noalloc: an invalid descriptor")
    fnt.fnt_cdc_aeq_batch_noalloc(tab_bad, len(chans))
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_check()
    assert e.value.code == fnt.FNT_E_INVAL
    assert (chans[5]["out"] == 777).all() and torch.equal(chans[5]["t"], torch.from_numpy(chans[5]["w0"]).to(dev))
    for i, c in enumerate(chans):
        if i == 5:
            continue
        outr, wr, _ = O.cdc_aeq(c["xs"], c["taps"], c["shift"], c["w0"], O.params(**c["prm"]), phase=c["phase"])
        assert np.array_equal(c["out"].cpu().numpy(), outr), i
        assert np.array_equal(c["t"].cpu().numpy(), wr), i
    fnt.fnt_check()
