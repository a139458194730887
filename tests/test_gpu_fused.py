"""GPU parity of the fused persistent CDC + AEQ kernel: one launch runs the CDC
into a ring in LDS and the AEQ chain from it (single-stream fnt_cdc_aeq and
fused plans), compared with the CPU oracle bit-exactly."""
import numpy as np
import pytest

import oracle as O
from paper_2405_04253_amd import fnt, synth

pytestmark = pytest.mark.gpu

# AEQ parameter sets from the everyday defaults to both ends of every range
AEQ_SETS = [dict(synth.AEQ_DEFAULTS, const_unit=60),
            dict(out_shift=24, err_shift=62, mu_shift=40, const_unit=4096, update_enable=1),
            dict(out_shift=0, err_shift=0, mu_shift=0, const_unit=1, update_enable=1),
            dict(out_shift=3, err_shift=20, mu_shift=17, const_unit=700, update_enable=1),
            dict(out_shift=9, err_shift=12, mu_shift=1, const_unit=33, update_enable=0)]


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


def to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rand_channel(rng, n, phase, k):
    """Random 5-bit samples and 6-bit taps (parity does not need a physical
    channel), a tap count in [1, 32], AEQ parameters from AEQ_SETS."""
    ntaps = int(rng.integers(1, 33))
    return dict(samples=rng.integers(-16, 16, size=(n, 4)).astype(np.int8),
                taps=rng.integers(-32, 32, size=(ntaps, 2)).astype(np.int8),
                shift=int(rng.integers(4, 10)), phase=phase,
                w0=(synth.centre_spike_taps() if k % 2 == 0
                    else rng.integers(-400, 400, size=(4, 4, 16)).astype(np.int16)),
                prm=AEQ_SETS[k % len(AEQ_SETS)])


def oracle_of(c):
    return O.cdc_aeq(c["samples"], c["taps"], c["shift"], c["w0"], O.params(**c["prm"]), phase=c["phase"])


def plan_entries(torch, dev, chans):
    ents = []
    for c in chans:
        M = O.n_symbols(c["samples"].shape[0], c["phase"])
        c["x"] = to_dev(torch, dev, c["samples"])
        c["out"] = torch.full((M, 4), 12345, dtype=torch.int16, device=dev)
        c["t"] = to_dev(torch, dev, c["w0"])
        ents.append((c["x"], c["out"], c["t"], fnt.cdc_params(c["taps"], c["shift"], c["phase"]),
                     fnt.aeq_params(**c["prm"])))
    return ents


def reset(torch, dev, chans):
    for c in chans:
        c["t"].copy_(to_dev(torch, dev, c["w0"]))
        c["out"].fill_(-1)


def check(chans, refs, what):
    for i, (c, (outr, wr, _)) in enumerate(zip(chans, refs)):
        assert np.array_equal(c["out"].cpu().numpy(), outr), (what, i, c["samples"].shape[0])
        assert np.array_equal(c["t"].cpu().numpy(), wr), (what, i, c["samples"].shape[0])


# instants: empty, shorter than a block, ragged, one chunk (64 blocks = 2048
# instants) and around it, the ring's four chunks and past them (wrap-around)
SINGLE_N = [0, 1, 2, 31, 33, 64, 2047, 2048, 2049, 8191, 8192, 8193, 4 * 2048 + 37, 9 * 2048 + 1001]


@pytest.mark.parametrize("lpt,split", [(4, False), (8, False), (16, False), (4, True), (8, True), (16, True)])
def test_fused_single_channel_lengths(torch_dev, lpt, split):
    """One channel per plan, fused with 1, 2 or 4 waves per polarisation half,
    both halves in one workgroup or one workgroup per half."""
    torch, dev = torch_dev
    rng = np.random.default_rng(lpt + 100 * split)
    for k, n in enumerate(SINGLE_N):
        c = rand_channel(rng, n, k % 2, k)
        ref = oracle_of(c)
        plan = fnt.Plan(plan_entries(torch, dev, [c]), autotune=False, use_graph=True)
        plan.set_fused(lpt, k % 2, split)
        info = plan.info()
        assert info["fused_lpt"] == lpt and info["graph"] == 1 and info["fused_split"] == int(split)
        assert info["fused_grid"] == (16 if split else 1)
        for rep in range(2):
            reset(torch, dev, [c])
            note(f"fused single lpt={lpt} split={split} n={n} phase={c['phase']} rep={rep}")
            plan.run()
            torch.cuda.synchronize()
            check([c], [ref], f"lpt={lpt} rep={rep}")
        plan.close()
    fnt.fnt_check()


def test_fnt_cdc_aeq_single_launch(torch_dev):
    """fnt_cdc_aeq (one fused launch, nothing allocated) on ragged lengths and both phases."""
    torch, dev = torch_dev
    rng = np.random.default_rng(77)
    for k, n in enumerate(SINGLE_N):
        c = rand_channel(rng, n, k % 2, k + 1)
        outr, wr, _ = oracle_of(c)
        taps = to_dev(torch, dev, c["w0"])
        note(f"fnt_cdc_aeq n={n} phase={c['phase']}")
        out = fnt.fnt_cdc_aeq(to_dev(torch, dev, c["samples"]), fnt.cdc_params(c["taps"], c["shift"], c["phase"]),
                              taps, fnt.aeq_params(**c["prm"]))
        assert np.array_equal(out.cpu().numpy(), outr), n
        assert np.array_equal(taps.cpu().numpy(), wr), n
    fnt.fnt_check()
    # an out-of-range sample is latched by the fused producer and reported
    bad = rng.integers(-16, 16, size=(4096, 4)).astype(np.int8)
    bad[3000, 2] = 16
    taps = to_dev(torch, dev, synth.centre_spike_taps())
    note("fnt_cdc_aeq range flag")
    fnt.fnt_cdc_aeq(to_dev(torch, dev, bad), fnt.cdc_params(np.ones((8, 2), np.int8), 6), taps,
                    fnt.aeq_params(**AEQ_SETS[0]))
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_check()
    assert e.value.code == fnt.FNT_E_RANGE
    fnt.fnt_check()


@pytest.mark.parametrize("prio", [0, 7, 1500])
def test_fused_batch_persistent(torch_dev, prio):
    """1500 channels (more than the fused kernel keeps resident, so workgroups
    take several channels from the work counter), a few long ones first in the
    longest-first order and many short, ragged or empty ones; graph replays with
    eager work between them, then a directly launched timed run; every channel
    bit-exact every time, so the counter is reset after each launch."""
    torch, dev = torch_dev
    rng = np.random.default_rng(1000 + prio)
    chans = []
    for k in range(1500):
        if k < 12:
            n = int(rng.integers(3 * 2048, 7 * 2048))
        else:
            n = int(rng.integers(0, 400)) if k % 7 else 0
        chans.append(rand_channel(rng, n, int(rng.integers(0, 2)), k))
    refs = [oracle_of(c) for c in chans]
    plan = fnt.Plan(plan_entries(torch, dev, chans), autotune=False, use_graph=True)
    plan.set_fused(4, prio)
    info = plan.info()
    assert info["fused_lpt"] == 4 and info["graph"] == 1
    assert 0 < info["fused_grid"] <= len(chans)
    note(f"fused batch grid={info['fused_grid']} prio={prio}")
    for rep in range(3):
        reset(torch, dev, chans)
        note(f"fused batch replay {rep}")
        plan.run()
        torch.cuda.synchronize()
        check(chans, refs, f"replay {rep}")
    reset(torch, dev, chans)
    note("fused batch timed run")
    t = plan.run_timed()
    assert t["fused"] == 1 and t["aeq_ms"] > 0
    check(chans, refs, "timed")
    # one workgroup per half for every channel (no work counter)
    plan.set_fused(8, prio, True)
    assert plan.info()["fused_grid"] == 16 * ((len(chans) + 7) // 8)
    reset(torch, dev, chans)
    note("fused batch, a workgroup per half")
    plan.run()
    torch.cuda.synchronize()
    check(chans, refs, "split halves")
    # switching the fused schedule off brings back the staged schedule, same results
    plan.set_fused(0)
    assert plan.info()["fused_lpt"] == 0
    reset(torch, dev, chans)
    note("staged after fused")
    plan.run()
    torch.cuda.synchronize()
    check(chans, refs, "staged")
    # a fused lead (lead form 6): the longest channels in the fused kernel on the
    # side stream, the others staged on the launch stream; more lead channels
    # than the kernel keeps resident, and a lead with a split after it
    for lead, nl, q in [(12, 0, 0), (1100, 0, 3), (300, 600, 0)]:
        plan.set_aeq_split(nl, 1, q)
        plan.set_lead(lead, 6)
        inf = plan.info()
        assert inf["lead_channels"] == lead and inf["lead_form"] == 6 and inf["top_channels"] == 0
        reset(torch, dev, chans)
        note(f"fused lead {lead} split {nl} rest form {q}")
        t = plan.run_timed()
        assert t["aeq_lead_ms"] > 0
        check(chans, refs, f"fused lead {lead}")
    plan.close()
    fnt.fnt_check()


def test_fused_plan_set_errors(torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(3)
    chans = [rand_channel(rng, 100, 0, 0)]
    plan = fnt.Plan(plan_entries(torch, dev, chans), autotune=False, use_graph=False)
    with pytest.raises(fnt.FntError) as e:
        plan.set_fused(5)
    assert e.value.code == fnt.FNT_E_INVAL
    plan.set_fused(16, 1)
    plan.set_aeq_waves(1)              # another schedule switches the fused kernel off
    assert plan.info()["fused_lpt"] == 0
    plan.close()
