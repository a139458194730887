"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Every result of the path is integer, so the tolerance is zero everywhere.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import fnt_ref as R
from paper_2405_04253_amd import fnt, synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


# ---------------------------------------------------------------- transforms --
TRANSFORMS = [(2, 3, fnt.FNT_ALPHA_2, 17, 2), (4, 5, fnt.FNT_ALPHA_2, 65537, 2),
              (4, 6, fnt.FNT_ALPHA_SQRT2, 65537, 4080), (2, 4, fnt.FNT_ALPHA_SQRT2, 17, 6),
              (3, 4, fnt.FNT_ALPHA_2, 257, 2), (3, 5, fnt.FNT_ALPHA_SQRT2, 257, 60)]


def test_transform_fig1_golden(torch_dev):
    torch, dev = torch_dev
    rows = []
    for line in open(os.path.join(GOLDEN, "fig1_fnt8_mod17.txt")):
        if line.startswith("#") or not line.strip():
            continue
        x, X = line.split("|")
        rows.append(([int(v) for v in x.split()], [int(v) for v in X.split()]))
    xs = to_dev(torch, dev, np.array([r[0] for r in rows], np.int32))
    note("fnt_forward t=2 N=8 golden")
    got = fnt.fnt_forward(xs, 2, 3, fnt.FNT_ALPHA_2).cpu().numpy()
    assert got.tolist() == [r[1] for r in rows]
    back = fnt.fnt_inverse(to_dev(torch, dev, got), 2, 3, fnt.FNT_ALPHA_2).cpu().numpy()
    assert back.tolist() == [r[0] for r in rows]
    fnt.fnt_check()


@pytest.mark.parametrize("t,log2n,kind,F,alpha", TRANSFORMS)
def test_transform_random_vs_definition(torch_dev, t, log2n, kind, F, alpha):
    torch, dev = torch_dev
    N = 1 << log2n
    rng = np.random.default_rng(N + t)
    batch = 37
    x = rng.integers(0, F, (batch, N)).astype(np.int64)
    x[0, :] = F - 1
    x[1, :] = 0
    x[2, :] = np.arange(N) % F
    xd = to_dev(torch, dev, x.astype(np.int32))
    note(f"fnt_forward t={t} N={N} batch={batch}")
    X = fnt.fnt_forward(xd, t, log2n, kind).cpu().numpy().astype(np.int64)
    for b in range(batch):
        assert X[b].tolist() == R.fnt(x[b].tolist(), alpha, F), b
    note(f"fnt_inverse t={t} N={N}")
    xi = fnt.fnt_inverse(to_dev(torch, dev, X.astype(np.int32)), t, log2n, kind).cpu().numpy()
    assert np.array_equal(xi.astype(np.int64), x)
    y = fnt.fnt_inverse(xd, t, log2n, kind).cpu().numpy().astype(np.int64)
    for b in range(3, 6):
        assert y[b].tolist() == R.ifnt(x[b].tolist(), alpha, F)
    # in place
    fnt.fnt_forward(xd, t, log2n, kind, out=xd)
    assert np.array_equal(xd.cpu().numpy().astype(np.int64), X)
    fnt.fnt_check()


def test_transform_range_and_shape_errors(torch_dev):
    torch, dev = torch_dev
    x = torch.zeros((2, 64), dtype=torch.int32, device=dev)
    x[1, 5] = 65537
    note("fnt_forward out-of-range residue")
    fnt.fnt_forward(x, 4, 6, fnt.FNT_ALPHA_SQRT2)
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_check()
    assert e.value.code == fnt.FNT_E_RANGE
    fnt.fnt_check()  # cleared
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_forward(torch.zeros((2, 64), dtype=torch.int32, device=dev), 4, 6, fnt.FNT_ALPHA_2)
    assert e.value.code == fnt.FNT_E_INVAL
    # lengths other than the radix's order, and moduli outside F_2..F_4
    for t, log2n, kind in [(3, 6, fnt.FNT_ALPHA_SQRT2), (3, 5, fnt.FNT_ALPHA_2), (2, 5, fnt.FNT_ALPHA_SQRT2),
                           (1, 2, fnt.FNT_ALPHA_2), (5, 6, fnt.FNT_ALPHA_2)]:
        with pytest.raises(fnt.FntError) as e:
            fnt.fnt_forward(torch.zeros((2, 1 << log2n), dtype=torch.int32, device=dev), t, log2n, kind)
        assert e.value.code == fnt.FNT_E_INVAL
    # a residue >= 257 is out of range for F_3
    y = torch.zeros((3, 32), dtype=torch.int32, device=dev)
    y[2, 31] = 257
    note("fnt_inverse out-of-range residue mod 257")
    fnt.fnt_inverse(y, 3, 5, fnt.FNT_ALPHA_SQRT2)
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_check()
    assert e.value.code == fnt.FNT_E_RANGE


# ----------------------------------------------------------------------- CDC --
CDC_CASES = [(1, 1, 0, 0), (31, 8, 3, 0), (32, 32, 7, 1), (33, 17, 6, 0), (64, 32, 7, 0),
             (95, 5, 2, 1), (1000, 32, 7, 1), (4099, 24, 5, 0), (5000, 32, 0, 1), (12345, 32, 8, 0)]


@pytest.mark.parametrize("n,L,shift,phase", CDC_CASES)
def test_cdc_random_vs_oracle(torch_dev, n, L, shift, phase):
    torch, dev = torch_dev
    x = synth.random_samples(n, seed=1000 + n)
    h = synth.random_taps(L, seed=L + n)
    zr, ar = O.cdc(x, h, shift, phase)
    note(f"fnt_cdc n={n} L={L} shift={shift} phase={phase}")
    z, a = fnt.fnt_cdc(to_dev(torch, dev, x), fnt.cdc_params(h, shift, phase))
    assert np.array_equal(z.cpu().numpy(), zr)
    assert np.array_equal(a.cpu().numpy(), ar)
    # without the exact output: the lane-per-block kernel, 16-byte aligned input
    # (vector loads) and an input 4 bytes off alignment (word loads)
    note(f"fnt_cdc lane kernel n={n} L={L} shift={shift} phase={phase}")
    _, a = fnt.fnt_cdc(to_dev(torch, dev, x), fnt.cdc_params(h, shift, phase), exact=False)
    assert np.array_equal(a.cpu().numpy(), ar)
    xb = torch.zeros((n + 1, 4), dtype=torch.int8, device=dev)
    xb[1:] = to_dev(torch, dev, x)
    _, a = fnt.fnt_cdc(xb[1:], fnt.cdc_params(h, shift, phase), exact=False)
    assert np.array_equal(a.cpu().numpy(), ar)
    fnt.fnt_check()


def test_cdc_eq5_worst_case(torch_dev):
    torch, dev = torch_dev
    n = 256
    for xv, hv in (((-16, -16), (-32, -32)), ((-16, -16), (-32, 31)), ((15, -16), (31, -32))):
        x = np.tile(np.array([xv[0], xv[1], xv[1], xv[0]], np.int8), (n, 1))
        h = np.tile(np.array(hv, np.int8), (32, 1))
        zr, ar = O.cdc(x, h, 11)
        note(f"fnt_cdc worst case x={xv} h={hv}")
        z, a = fnt.fnt_cdc(to_dev(torch, dev, x), fnt.cdc_params(h, 11))
        assert np.array_equal(z.cpu().numpy(), zr)
        assert np.array_equal(a.cpu().numpy(), ar)
        for ph in (0, 1):
            _, ar2 = O.cdc(x, h, 0, ph)
            _, a = fnt.fnt_cdc(to_dev(torch, dev, x), fnt.cdc_params(h, 0, ph), exact=False)
            assert np.array_equal(a.cpu().numpy(), ar2)
    assert np.abs(zr).max() <= 32768
    fnt.fnt_check()


def test_cdc_generated_channel(torch_dev):
    torch, dev = torch_dev
    ch = synth.single_channel(1 << 14)
    zr, ar = O.cdc(ch.samples, ch.taps, ch.requant_shift)
    note("fnt_cdc 75 km channel 2^14 symbols")
    z, a = fnt.fnt_cdc(to_dev(torch, dev, ch.samples), fnt.cdc_params(ch.taps, ch.requant_shift))
    assert np.array_equal(z.cpu().numpy(), zr)
    assert np.array_equal(a.cpu().numpy(), ar)
    fnt.fnt_check()


def test_cdc_range_flag(torch_dev):
    torch, dev = torch_dev
    x = synth.random_samples(100, seed=3)
    x[57, 2] = 16
    note("fnt_cdc out-of-range sample")
    fnt.fnt_cdc(to_dev(torch, dev, x), fnt.cdc_params(synth.random_taps(8, 1), 4))
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_check()
    assert e.value.code == fnt.FNT_E_RANGE
    bad = synth.random_taps(8, 1)
    bad[3, 0] = -33
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_cdc(to_dev(torch, dev, x), fnt.cdc_params(bad, 4))
    assert e.value.code == fnt.FNT_E_RANGE


# ----------------------------------------------------------------------- AEQ --
AEQ_PARAMS = [dict(out_shift=7, err_shift=16, mu_shift=3, const_unit=52, update_enable=1),
              dict(out_shift=7, err_shift=16, mu_shift=3, const_unit=52, update_enable=0),
              dict(out_shift=0, err_shift=10, mu_shift=0, const_unit=4096, update_enable=1),
              dict(out_shift=12, err_shift=30, mu_shift=9, const_unit=1, update_enable=1)]


@pytest.mark.parametrize("M", [0, 1, 15, 16, 17, 100, 1000])
@pytest.mark.parametrize("pi", range(len(AEQ_PARAMS)))
def test_aeq_random_vs_oracle(torch_dev, M, pi):
    torch, dev = torch_dev
    prm = AEQ_PARAMS[pi]
    rng = np.random.default_rng(M * 7 + pi)
    a = rng.integers(-16, 16, (M, 4)).astype(np.int8)
    w = synth.random_aeq_taps(seed=M + pi) if pi != 0 else synth.centre_spike_taps()
    if pi == 3:
        w[0, :, :] = -8192
        w[1, :, :] = 8191
    outr, wr = O.aeq(a, w, O.params(**prm))
    taps = to_dev(torch, dev, w)
    note(f"fnt_aeq M={M} params={prm}")
    out = fnt.fnt_aeq(to_dev(torch, dev, a), taps, fnt.aeq_params(**prm))
    assert np.array_equal(out.cpu().numpy(), outr)
    assert np.array_equal(taps.cpu().numpy(), wr)
    fnt.fnt_check()


def test_aeq_extreme_inputs(torch_dev):
    torch, dev = torch_dev
    M = 160
    a = np.full((M, 4), -16, np.int8)
    a[::3] = 15
    for tap in (-8192, 8191, -8128, 8127, -64):
        w = np.full((4, 4, 16), tap, np.int16)
        prm = dict(out_shift=9, err_shift=20, mu_shift=2, const_unit=300, update_enable=1)
        outr, wr = O.aeq(a, w, O.params(**prm))
        taps = to_dev(torch, dev, w)
        note(f"fnt_aeq extreme tap={tap}")
        out = fnt.fnt_aeq(to_dev(torch, dev, a), taps, fnt.aeq_params(**prm))
        assert np.array_equal(out.cpu().numpy(), outr)
        assert np.array_equal(taps.cpu().numpy(), wr)
    fnt.fnt_check()


def test_cdc_aeq_chain_c0(torch_dev):
    torch, dev = torch_dev
    ch = synth.single_channel(1 << 14)
    prm = synth.aeq_params_for(ch)
    outr, wr, _ = O.cdc_aeq(ch.samples, ch.taps, ch.requant_shift, synth.centre_spike_taps(), O.params(**prm))
    taps = to_dev(torch, dev, synth.centre_spike_taps())
    note("fnt_cdc_aeq 75 km 2^14 symbols")
    out = fnt.fnt_cdc_aeq(to_dev(torch, dev, ch.samples), fnt.cdc_params(ch.taps, ch.requant_shift), taps,
                          fnt.aeq_params(**prm))
    assert np.array_equal(out.cpu().numpy(), outr)
    assert np.array_equal(taps.cpu().numpy(), wr)
    fnt.fnt_check()


# --------------------------------------------------------------------- plans --
def _batch(nch, lo, hi, seed):
    specs = synth.batched_specs(nch, lo, hi, base_seed=seed, tag="plan-test")
    chans = synth.gen_many(specs, workers=4)
    return chans


def _plan_channels(torch, dev, chans, rng):
    out = []
    for i, ch in enumerate(chans):
        w0 = synth.centre_spike_taps() if i % 3 else synth.random_aeq_taps(seed=i, lo=-300, hi=300)
        prm = synth.aeq_params_for(ch)
        M = O.n_symbols(ch.n, 0)
        out.append(dict(ch=ch, w0=w0, prm=prm,
                        x=to_dev(torch, dev, ch.samples),
                        out=torch.full((M, 4), 12345, dtype=torch.int16, device=dev),
                        taps=to_dev(torch, dev, w0)))
    return out


@pytest.mark.parametrize("variant,wpp", [(0, 0), (0, 3), (0, 1), (0, 2), (0, 4), (0, 5), (1, 1), (2, 1), (3, 1)])
def test_plan_batched_vs_oracle(torch_dev, variant, wpp):
    torch, dev = torch_dev
    chans = _batch(40, 6, 11, seed=variant)
    chans.append(synth.gen_channel(3, 30.0, 20.0, seed=5))      # ragged, tiny
    chans.append(synth.gen_channel(0, 30.0, 20.0, seed=6))      # empty
    rng = np.random.default_rng(0)
    pc = _plan_channels(torch, dev, chans, rng)
    refs = [O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"], O.params(**c["prm"]))
            for c in pc]
    plan = fnt.Plan([(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                      fnt.aeq_params(**c["prm"])) for c in pc], autotune=False, use_graph=True)
    plan.set_aeq_variant(variant)
    plan.set_aeq_waves(wpp)
    for rep in range(3):
        for c in pc:        # eager work between replays: reset the tap state
            c["taps"].copy_(to_dev(torch, dev, c["w0"]))
            c["out"].fill_(-1)
        note(f"plan run variant={variant} wpp={wpp} replay={rep}")
        plan.run()
        torch.cuda.synchronize()
        for c, (outr, wr, _) in zip(pc, refs):
            assert np.array_equal(c["out"].cpu().numpy(), outr), (rep, c["ch"].n)
            assert np.array_equal(c["taps"].cpu().numpy(), wr), (rep, c["ch"].n)
    info = plan.info()
    assert info["channels"] == len(pc) and info["graph"] == 1 and info["aeq_variant"] == variant
    assert info["aeq_waves_per_pol"] == wpp
    # leads that leave only the tiny and the empty channel (last in the longest-first
    # order) to the others' CDC and AEQ, with and without a first level
    for lead, lf, top, tf in [(len(pc) - 1, 1, 0, -1), (len(pc) - 2, 3, 5, 2), (len(pc) - 1, 0, 40, 4)]:
        plan.set_lead(lead, lf, top, tf)
        assert plan.info()["lead_channels"] == lead
        for c in pc:
            c["taps"].copy_(to_dev(torch, dev, c["w0"]))
            c["out"].fill_(-1)
        note(f"plan run variant={variant} wpp={wpp} lead={lead}/{lf} top={top}/{tf}")
        plan.run()
        torch.cuda.synchronize()
        for c, (outr, wr, _) in zip(pc, refs):
            assert np.array_equal(c["out"].cpu().numpy(), outr), (lead, c["ch"].n)
            assert np.array_equal(c["taps"].cpu().numpy(), wr), (lead, c["ch"].n)
    plan.close()
    fnt.fnt_check()


EXTREME_AEQ = [dict(out_shift=24, err_shift=62, mu_shift=40, const_unit=4096, update_enable=1),
               dict(out_shift=0, err_shift=0, mu_shift=0, const_unit=1, update_enable=1),
               dict(out_shift=3, err_shift=20, mu_shift=17, const_unit=700, update_enable=1),
               dict(out_shift=9, err_shift=12, mu_shift=1, const_unit=33, update_enable=0)]



@pytest.mark.parametrize("wpp", [1, 2, 4, 5])
def test_plan_short_chains_pol_forms(torch_dev, wpp):
    """Chains of 1 to 5 blocks with ragged ends on the polarisation-split forms: the
    window symbols two blocks ahead are loaded from a clamped index and the zeros
    past the end applied when the window is used."""
    torch, dev = torch_dev
    lengths = [1, 2, 15, 16, 17, 31, 32, 33, 47, 48, 49, 63, 64, 65, 80]
    chans = [synth.gen_channel(m, 20.0 + m % 50, 20.0, seed=100 + m) for m in lengths]
    pc = _plan_channels(torch, dev, chans, np.random.default_rng(1))
    refs = [O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"], O.params(**c["prm"]))
            for c in pc]
    plan = fnt.Plan([(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                      fnt.aeq_params(**c["prm"])) for c in pc], autotune=False, use_graph=False)
    plan.set_aeq_waves(wpp)
    note(f"short chains, form {wpp}")
    plan.run()
    torch.cuda.synchronize()
    fnt.fnt_check()
    for m, c, (outr, wr, _) in zip(lengths, pc, refs):
        assert np.array_equal(c["out"].cpu().numpy(), outr), m
        assert np.array_equal(c["taps"].cpu().numpy(), wr), m
    plan.close()


@pytest.mark.parametrize("wpp", [0, 3, 1, 5])
def test_plan_extreme_aeq_params(torch_dev, wpp):
    """Shift and constant extremes (saturating taps and errors) on the batched kernels."""
    torch, dev = torch_dev
    chans = _batch(8, 6, 10, seed=77)
    pc = _plan_channels(torch, dev, chans, None)
    for i, c in enumerate(pc):
        c["prm"] = EXTREME_AEQ[i % len(EXTREME_AEQ)]
    plan = fnt.Plan([(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                      fnt.aeq_params(**c["prm"])) for c in pc], autotune=False, use_graph=False)
    plan.set_aeq_waves(wpp)
    note(f"plan extreme AEQ params wpp={wpp}")
    plan.run()
    torch.cuda.synchronize()
    for c in pc:
        outr, wr, _ = O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"],
                                O.params(**c["prm"]))
        assert np.array_equal(c["out"].cpu().numpy(), outr), c["prm"]
        assert np.array_equal(c["taps"].cpu().numpy(), wr), c["prm"]
    plan.close()
    fnt.fnt_check()


def test_plan_graph_replay_with_lead(torch_dev):
    """fnt_plan_run_graph: the captured graph of a schedule with a pipelined lead
    (the lead's branch forked and joined by events inside the capture) replayed
    several times, with eager work and synchronisation between replays, equals
    the direct launches and the oracle every time."""
    torch, dev = torch_dev
    chans = _batch(24, 6, 11, seed=41)
    pc = _plan_channels(torch, dev, chans, None)
    refs = [O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"], O.params(**c["prm"]))
            for c in pc]
    entries = [(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                fnt.aeq_params(**c["prm"])) for c in pc]
    plan = fnt.Plan(entries, autotune=False, use_graph=True)
    for lead, lf, top, tf in [(8, 1, 0, -1), (10, 2, 3, 4), (6, 6, 0, -1)]:
        plan.set_aeq_split(12, 1, 0)
        plan.set_lead(lead, lf, top, tf)
        for rep in range(3):
            for c in pc:                                # eager work between the replays
                c["taps"].copy_(to_dev(torch, dev, c["w0"]))
                c["out"].fill_(-7)
            torch.cuda.synchronize()
            note(f"graph replay with lead {lead}/{lf} top {top}/{tf}, replay {rep}")
            plan.run_graph()
            torch.cuda.synchronize()
            fnt.fnt_check()
            for c, (outr, wr, _) in zip(pc, refs):
                assert np.array_equal(c["out"].cpu().numpy(), outr), (lead, rep, c["ch"].n)
                assert np.array_equal(c["taps"].cpu().numpy(), wr), (lead, rep, c["ch"].n)
    plan.close()
    nog = fnt.Plan(entries[:3], autotune=False, use_graph=False)
    with pytest.raises(fnt.FntError) as e:
        nog.run_graph()
    assert e.value.code == fnt.FNT_E_STATE
    nog.close()


def test_plan_fermat_gradient_extremes(torch_dev):
    """AEQ variant 3 (the RDE gradient through FNT32 products) at the Eq. (5)
    bound of the gradient: windows of -16 and errors clipped at -128 give
    G = 16 * (-128) * (-16) = 32768 = (F - 1) / 2 in every full block (and -32512
    with +127), next to the extreme shift settings and random channels; every
    output and final tap equals the oracle's direct gradient."""
    torch, dev = torch_dev
    chans, inits, prms = [], [], []
    extreme = dict(out_shift=0, err_shift=0, mu_shift=30, const_unit=1, update_enable=1)
    for k, (sign, nsym) in enumerate([(-1, 16 * 40), (1, 16 * 40 + 7), (-1, 5)]):
        x = np.full((2 * nsym, 4), -16, dtype=np.int8)
        h = np.zeros((1, 2), dtype=np.int8)
        h[0, 0] = 31                                    # z = 31 x: requantised to -16 with shift 0
        chans.append((x, h, 0))
        w0 = np.zeros((4, 4, 16), dtype=np.int16)
        for q in range(4):
            w0[q, q, 8] = sign * 4096                   # y = -/+ 65536: outputs saturate, eps clips
        inits.append(w0)
        prms.append(extreme)
    for i, ch in enumerate(_batch(8, 6, 10, seed=91)):
        chans.append((ch.samples, ch.taps, ch.requant_shift))
        inits.append(synth.centre_spike_taps() if i % 2 else synth.random_aeq_taps(seed=i, lo=-300, hi=300))
        prms.append(EXTREME_AEQ[i % len(EXTREME_AEQ)] if i < 4 else synth.aeq_params_for(ch))
    entries, refs, outs, taps = [], [], [], []
    for (x, h, sh), w0, prm in zip(chans, inits, prms):
        M = O.n_symbols(x.shape[0], 0)
        outs.append(torch.full((M, 4), 12345, dtype=torch.int16, device=dev))
        taps.append(to_dev(torch, dev, w0))
        entries.append((to_dev(torch, dev, x), outs[-1], taps[-1], fnt.cdc_params(h, sh), fnt.aeq_params(**prm)))
        refs.append(O.cdc_aeq(x, h, sh, w0, O.params(**prm)))
    plan = fnt.Plan(entries, autotune=False, use_graph=False)
    plan.set_aeq_variant(3)
    note("plan AEQ variant 3 (Fermat-domain gradient) at the gradient's Eq. (5) bound")
    plan.run()
    torch.cuda.synchronize()
    fnt.fnt_check()
    for i, (o, w, (outr, wr, _)) in enumerate(zip(outs, taps, refs)):
        assert np.array_equal(o.cpu().numpy(), outr), i
        assert np.array_equal(w.cpu().numpy(), wr), i
    plan.close()


@pytest.mark.parametrize("aeq_variant", [0, 1])
def test_plan_direct_cdc_comparator(torch_dev, aeq_variant):
    """The direct time-domain CDC (and AEQ) comparators give the method's results bit for bit."""
    torch, dev = torch_dev
    rng = np.random.default_rng(31)
    chans = []
    for i, n in enumerate([1, 31, 32, 33, 95, 2048, 2049, 4133, 70000, 131072 + 96]):
        L = int(rng.integers(1, 33))
        x = synth.random_samples(n, seed=500 + i)
        h = synth.random_taps(L, seed=600 + i)
        if i == 3:                                     # Eq. (5) extreme for this channel
            x[:] = -16
            h[:, 0], h[:, 1] = -32, 31
        chans.append((x, h, int(rng.integers(0, 9)), i % 2))
    entries, refs = [], []
    w0 = synth.centre_spike_taps()
    for x, h, sh, ph in chans:
        prm = dict(synth.AEQ_DEFAULTS, const_unit=40)
        M = O.n_symbols(x.shape[0], ph)
        xd = to_dev(torch, dev, x)
        out = torch.full((M, 4), 777, dtype=torch.int16, device=dev)
        taps = to_dev(torch, dev, w0)
        entries.append((xd, out, taps, fnt.cdc_params(h, sh, ph), fnt.aeq_params(**prm)))
        refs.append(O.cdc_aeq(x, h, sh, w0, O.params(**prm), phase=ph))
    plan = fnt.Plan(entries, autotune=False, use_graph=True)
    plan.set_cdc_variant(1)
    plan.set_aeq_variant(aeq_variant)
    assert plan.info()["cdc_variant"] == 1
    for rep in range(2):
        for e in entries:
            e[2].copy_(to_dev(torch, dev, w0))
        note(f"plan with the direct CDC, AEQ variant {aeq_variant}, replay {rep}")
        plan.run()
        torch.cuda.synchronize()
        for e, (outr, wr, _) in zip(entries, refs):
            assert np.array_equal(e[1].cpu().numpy(), outr)
            assert np.array_equal(e[2].cpu().numpy(), wr)
    # with a two-level pipelined lead (the comparator kernels in every launch)
    plan.set_lead(6, -1, 2, -1)
    assert plan.info()["lead_channels"] == 6 and plan.info()["top_channels"] == 2
    for e in entries:
        e[2].copy_(to_dev(torch, dev, w0))
        e[1].fill_(-5)
    note(f"plan with the direct CDC, AEQ variant {aeq_variant}, pipelined lead")
    t = plan.run_timed()
    assert t["aeq_top_ms"] > 0 and t["aeq_lead_ms"] > 0
    for e, (outr, wr, _) in zip(entries, refs):
        assert np.array_equal(e[1].cpu().numpy(), outr)
        assert np.array_equal(e[2].cpu().numpy(), wr)
    with pytest.raises(fnt.FntError):
        plan.set_cdc_variant(2)
    plan.close()
    fnt.fnt_check()


def _fusable(long_form, rest_form):
    """Form pairs that run as one split launch (mirrors the library's table)."""
    return ((long_form in (1, 2, 4, 5) and rest_form in (0, 3)) or (long_form, rest_form) in ((3, 0), (2, 5)))


def test_plan_determinism_across_schedules(torch_dev):
    """Race check: identical outputs for every launch schedule and wave split."""
    torch, dev = torch_dev
    chans = _batch(24, 7, 11, seed=21)
    pc = _plan_channels(torch, dev, chans, None)
    plan = fnt.Plan([(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                      fnt.aeq_params(**c["prm"])) for c in pc], autotune=False, use_graph=True)
    ref = None
    for wpg, bpw, wpp, variant in [(4, 0, 1, 0), (4, 1, 1, 0), (1, 1, 2, 0), (2, 3, 4, 0), (4, 64, 1, 0),
                                   (1, 7, 2, 0), (1, 0, 2, 0), (2, 0, 4, 0), (4, 0, 0, 0), (4, 0, 3, 0),
                                   (2, 2, 1, 1), (4, 5, 1, 2), (1, 0, 5, 0)]:
        plan.set_cdc_schedule(wpg, bpw)
        plan.set_aeq_waves(wpp)
        plan.set_aeq_variant(variant)
        for rep in range(2):
            for c in pc:
                c["taps"].copy_(to_dev(torch, dev, c["w0"]))
            note(f"plan schedule wpg={wpg} bpw={bpw} wpp={wpp} variant={variant} rep={rep}")
            plan.run()
            torch.cuda.synchronize()
            got = [(c["out"].cpu().numpy().copy(), c["taps"].cpu().numpy().copy()) for c in pc]
            if ref is None:
                ref = got
                for c, (o, w) in zip(pc, got):
                    outr, wr, _ = O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"],
                                            O.params(**c["prm"]))
                    assert np.array_equal(o, outr) and np.array_equal(w, wr)
            else:
                for (o, w), (o2, w2) in zip(ref, got):
                    assert np.array_equal(o, o2) and np.array_equal(w, w2)
    # longest chains in their own concurrent launch
    plan.set_aeq_variant(0)
    for nl, wl, ws in [(5, 4, 1), (12, 2, 1), (1, 4, 2), (24, 4, 1), (3, 4, 0), (8, 2, 0), (23, 4, 0),
                       (6, 3, 0), (9, 1, 3), (2, 4, 3), (7, 5, 0), (10, 5, 3), (4, 2, 5), (1, 2, 5), (23, 2, 5)]:
        plan.set_aeq_split(nl, wl, ws)
        for c in pc:
            c["taps"].copy_(to_dev(torch, dev, c["w0"]))
        note(f"plan split long={nl} wl={wl} ws={ws}")
        plan.run()
        torch.cuda.synchronize()
        info = plan.info()
        assert info["aeq_long_channels"] == min(nl, len(pc)) and info["aeq_waves_long"] == wl
        for c, (o, w) in zip(pc, ref):
            assert np.array_equal(c["out"].cpu().numpy(), o) and np.array_equal(c["taps"].cpu().numpy(), w)
    # pipelined lead: the longest channels' CDC first, their AEQ on the side stream
    # while the others' CDC and AEQ run (graph replay, direct launch, timed launch)
    n = len(pc)
    for lead, lf, top, tf, nl, wl, ws, active in [
            (1, -1, 0, -1, 1, 1, 0, True), (3, 2, 0, -1, 5, 1, 3, True), (5, -1, 0, -1, 12, 2, 1, False),
            (n - 1, -1, 0, -1, n, 4, 0, True), (10, 0, 0, -1, 2, 4, 3, True),
            (4, 4, 0, -1, 9, 3, 0, True), (7, 3, 0, -1, 7, 1, 0, True),
            (n, -1, 0, -1, 3, 1, 0, False), (0, 2, 0, -1, 3, 1, 0, False),
            # two levels: the first level's CDC first and its AEQ on a third stream
            (6, -1, 2, 2, 9, 1, 0, True), (12, 1, 1, -1, 12, 1, 3, True), (n - 1, 3, 5, 4, n, 2, 0, True),
            (4, -1, 4, 2, 4, 1, 0, True), (5, -1, 2, 1, 12, 2, 1, False),
            # a first level that pairs with the lead's form runs inside the lead's launch
            (6, 5, 2, 2, 9, 1, 0, True), (8, 5, 3, -1, 8, 2, 0, True), (n - 1, 5, 7, 2, n, 1, 3, True),
            # a fused lead (form 6: the lead's CDC and AEQ in one fused launch; no first level)
            (6, 6, 0, -1, 9, 1, 0, True), (n - 1, 6, 0, -1, n, 4, 0, True), (3, 6, 0, -1, 12, 2, 1, False)]:
        plan.set_aeq_split(nl, wl, ws)
        plan.set_lead(lead, lf, top, tf)
        info = plan.info()
        top_eff = top if active and top < lead else 0
        lf_e, tf_e = (wl if lf == -1 else lf), (wl if tf == -1 else tf)
        own_top = top_eff > 0 and not _fusable(tf_e, lf_e)
        assert info["lead_channels"] == (lead if active else 0)
        assert info["lead_form"] == (wl if lf == -1 else lf)
        assert info["top_channels"] == top_eff and info["top_form"] == (wl if tf == -1 else tf)
        for mode in ("run", "timed", "stages"):
            for c in pc:
                c["taps"].copy_(to_dev(torch, dev, c["w0"]))
                c["out"].fill_(-3)
            note(f"plan lead={lead}/{lf} top={top}/{tf} long={nl} wl={wl} ws={ws} {mode}")
            if mode == "run":
                plan.run()
            elif mode == "timed":
                t = plan.run_timed()
                assert t["step_ms"] > 0 and t["cdc_ms"] > 0 and t["aeq_ms"] > 0
                assert (t["aeq_lead_ms"] > 0) == active and (t["aeq_top_ms"] > 0) == own_top
                assert t["aeq_blocks"] + t["aeq_lead_blocks"] + t["aeq_top_blocks"] == \
                    sum((c["out"].shape[0] + 15) // 16 for c in pc)
            else:
                plan.run_stage(fnt.FNT_STAGE_ALL)
            torch.cuda.synchronize()
            for c, (o, w) in zip(pc, ref):
                assert np.array_equal(c["out"].cpu().numpy(), o) and np.array_equal(c["taps"].cpu().numpy(), w)
    with pytest.raises(fnt.FntError):
        plan.set_lead(2, 7)
    with pytest.raises(fnt.FntError):
        plan.set_lead(4, 1, 2, 7)
    plan.set_aeq_waves(1)
    assert plan.info()["lead_channels"] == 0
    plan.close()
    fnt.fnt_check()


def test_plan_autotune_and_eager(torch_dev, tmp_path):
    torch, dev = torch_dev
    chans = _batch(12, 8, 12, seed=9)
    pc = _plan_channels(torch, dev, chans, None)
    cache = str(tmp_path / "tune.jsonl")
    note("plan autotune")
    plan = fnt.Plan([(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                      fnt.aeq_params(**c["prm"])) for c in pc], autotune=True, use_graph=False,
                    tune_cache=cache)
    plan.run()
    torch.cuda.synchronize()
    for c in pc:
        outr, wr, _ = O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"],
                                O.params(**c["prm"]))
        assert np.array_equal(c["out"].cpu().numpy(), outr)
        assert np.array_equal(c["taps"].cpu().numpy(), wr)
    assert os.path.exists(cache) and "wpg" in open(cache).read()
    info = plan.info()
    assert info["graph"] == 0 and 0 <= info["cdc_blocks_per_wave"] <= 64
    assert 0 <= info["lead_channels"] < len(pc)
    # a second plan over the same channels takes the schedule from the cache
    plan2 = fnt.Plan([(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                       fnt.aeq_params(**c["prm"])) for c in pc], autotune=True, use_graph=False,
                     tune_cache=cache)
    info2 = plan2.info()
    assert info2["tune_ms"] == 0.0
    for k in ("cdc_waves_per_group", "cdc_blocks_per_wave", "aeq_waves_per_pol", "aeq_waves_long",
              "aeq_long_channels", "lead_channels", "lead_form", "top_channels", "top_form"):
        assert info2[k] == info[k], k
    plan2.close()
    # the two stages launched one by one reproduce a whole run
    for c in pc:
        c["taps"].copy_(to_dev(torch, dev, c["w0"]))
        c["out"].fill_(-7)
    note("plan staged run")
    plan.run_stage(fnt.FNT_STAGE_CDC)
    plan.run_stage(fnt.FNT_STAGE_AEQ)
    torch.cuda.synchronize()
    for c in pc:
        outr, wr, _ = O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"],
                                O.params(**c["prm"]))
        assert np.array_equal(c["out"].cpu().numpy(), outr)
        assert np.array_equal(c["taps"].cpu().numpy(), wr)
    with pytest.raises(fnt.FntError):
        plan.run_stage(4)
    plan.close()
    fnt.fnt_check()


# ------------------------------------------------------------------ sessions --
def _session_channels(nch, seg_blocks, seed):
    """Per channel: a continuing stream cut into segments (multiples of 32 instants)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(nch):
        segs = [int(b) * 32 for b in rng.integers(1, seg_blocks, size=int(rng.integers(2, 5)))]
        ch = synth.gen_channel(sum(segs) // 2, float(rng.uniform(10, 80)), float(rng.uniform(18, 26)),
                               seed=synth.seed_for(seed, "session", c))
        out.append((ch, segs))
    return out


def _oracle_stream(ch, w0=None):
    prm = synth.aeq_params_for(ch)
    outr, wr, _ = O.cdc_aeq(ch.samples, ch.taps, ch.requant_shift,
                            synth.centre_spike_taps() if w0 is None else w0, O.params(**prm))
    return outr, wr


@pytest.mark.parametrize("form", [-1, 0, 3, 1, 2, 4, 5])
def test_session_streams_vs_oracle(torch_dev, form):
    """Tick after tick through every AEQ form: taps, CDC tail and AEQ tail carry over."""
    torch, dev = torch_dev
    chans = _session_channels(6, 40, seed=1)
    s = fnt.Session(max_channels=8, hbm_budget_bytes=64 << 20, chunk_blocks=8, aeq_form=form)
    outs = []
    for c, (ch, segs) in enumerate(chans):
        s.add_channel(c, fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch)))
        outs.append(torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev))
    xs = [to_dev(torch, dev, ch.samples) for ch, _ in chans]
    # interleave the segments of all channels
    order = []
    for c, (ch, segs) in enumerate(chans):
        off = 0
        for k, n in enumerate(segs):
            order.append((k, c, off, n))
            off += n
    order.sort()
    note(f"session submit interleaved segments, AEQ form {form}")
    tickets = [s.submit(c, xs[c][off:off + n], outs[c][off // 2:(off + n) // 2]) for _, c, off, n in order]
    s.drain()
    assert all(s.poll(t) for t in tickets)
    for c, (ch, segs) in enumerate(chans):
        outr, _ = _oracle_stream(ch)
        assert np.array_equal(outs[c].cpu().numpy(), outr), c
    st = s.stats()
    assert st["completed"] == len(tickets) and st["p99_us"] >= st["p50_us"] > 0
    s.close()
    fnt.fnt_check()


def test_session_state_export_import(torch_dev):
    torch, dev = torch_dev
    ch = synth.gen_channel(1536, 75.0, 22.0, seed=77)
    x = to_dev(torch, dev, ch.samples)
    out = torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev)
    cp, ap = fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch))
    k = 1024                     # split point (instants, multiple of 32)
    s1 = fnt.Session(max_channels=2, hbm_budget_bytes=16 << 20, chunk_blocks=4)
    s1.add_channel(1, cp, ap)
    note("session export after first segment")
    s1.wait(s1.submit(1, x[:k], out[:k // 2]))
    state = s1.get_state(1)
    assert len(state) == fnt.FNT_STATE_BYTES
    s1.close()
    s2 = fnt.Session(max_channels=4, hbm_budget_bytes=16 << 20, chunk_blocks=16)
    s2.add_channel(3, cp, ap)
    s2.set_state(3, state)
    note("session import and continue")
    s2.wait(s2.submit(3, x[k:], out[k // 2:]))
    outr, wr = _oracle_stream(ch)
    assert np.array_equal(out.cpu().numpy(), outr)
    st2 = s2.get_state(3)
    assert np.array_equal(np.frombuffer(st2[:512], np.int16).reshape(4, 4, 16), wr)
    s2.close()
    fnt.fnt_check()


@pytest.mark.parametrize("form", [1, 2, 4])
def test_session_history_after_each_segment(torch_dev, form):
    """After every request the exported state holds the oracle's histories.

    The polarisation-split forms run a channel's two halves as separate
    workgroups; a tick reads one copy of the AEQ history and writes the other,
    so the exported AEQ tail must be the last 16 symbols of the 1-sps stream
    and the CDC tail the last 32 instants, segment after segment."""
    torch, dev = torch_dev
    ch = synth.gen_channel(16 * 70, 60.0, 22.0, seed=91)
    x = to_dev(torch, dev, ch.samples)
    out = torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev)
    cp, ap = fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch))
    s = fnt.Session(max_channels=2, hbm_budget_bytes=16 << 20, chunk_blocks=4, aeq_form=form)
    s.add_channel(0, cp, ap)
    _, a_ref = O.cdc(ch.samples, ch.taps, ch.requant_shift)
    outr, _ = _oracle_stream(ch)
    off = 0
    for k, nb in enumerate([5, 1, 8, 3, 2, 4]):        # blocks of 32 instants; odd and even tick counts
        n = 32 * nb
        note(f"session history form {form} segment {k} n={n}")
        s.wait(s.submit(0, x[off:off + n], out[off // 2:(off + n) // 2]))
        off += n
        st = s.get_state(0)
        cdc_tail = np.frombuffer(st[512:640], np.int8).reshape(32, 4)
        aeq_tail = np.frombuffer(st[640:704], np.int8).reshape(16, 4)
        assert np.array_equal(cdc_tail, ch.samples[off - 32:off]), k
        assert np.array_equal(aeq_tail, a_ref[off // 2 - 16:off // 2]), k
    assert np.array_equal(out[:off // 2].cpu().numpy(), outr[:off // 2])
    s.close()
    fnt.fnt_check()


def test_session_reregister_right_after_submit(torch_dev):
    """Registering a channel again waits for the ticks still running on it."""
    torch, dev = torch_dev
    ch = synth.gen_channel(16 * 48, 40.0, 22.0, seed=92)
    x = to_dev(torch, dev, ch.samples)
    cp, ap = fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch))
    outr, _ = _oracle_stream(ch)
    s = fnt.Session(max_channels=1, hbm_budget_bytes=16 << 20, chunk_blocks=48)
    for rep in range(3):
        s.add_channel(0, cp, ap)
        out = torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev)
        note(f"session re-register rep {rep}")
        tk = s.submit(0, x, out)
        # the request leaves the queue when its last block is placed in a tick;
        # from then on add_channel succeeds, after that tick has retired
        while True:
            try:
                s.add_channel(0, cp, ap)
                break
            except fnt.FntError as e:
                assert e.code == fnt.FNT_E_STATE
        assert s.poll(tk)
        assert np.array_equal(out.cpu().numpy(), outr), rep
    s.close()
    fnt.fnt_check()


def test_session_cancel_and_destroy_in_flight(torch_dev):
    """Cancelled requests never run; closing a session with work queued drains it."""
    torch, dev = torch_dev
    ch = synth.gen_channel(16 * 64, 50.0, 22.0, seed=93)
    x = to_dev(torch, dev, ch.samples)
    cp, ap = fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch))
    outr, _ = _oracle_stream(ch)
    s = fnt.Session(max_channels=1, hbm_budget_bytes=16 << 20, chunk_blocks=2)
    s.add_channel(0, cp, ap)
    out = torch.full((ch.n // 2, 4), 777, dtype=torch.int16, device=dev)
    segs = [(i * 256, 256) for i in range(ch.n // 256)]           # 8 blocks each
    note("session cancel: submit segments")
    tks = [s.submit(0, x[o:o + n], out[o // 2:(o + n) // 2]) for o, n in segs]
    # the last segments are still queued behind the first: cancel them
    cancelled = []
    for tk in reversed(tks[2:]):
        try:
            s.cancel(tk)
            cancelled.append(tk)
        except fnt.FntError as e:
            assert e.code == fnt.FNT_E_STATE            # already started
            break
    assert cancelled, "nothing was left to cancel"
    with pytest.raises(fnt.FntError) as e:
        s.cancel(cancelled[0])                          # not queued any more
    assert e.value.code == fnt.FNT_E_STATE
    with pytest.raises(fnt.FntError) as e:
        s.cancel(10 ** 9)
    assert e.value.code == fnt.FNT_E_STATE
    s.drain()
    ran = [tk for tk in tks if tk not in cancelled]
    assert all(s.poll(tk) for tk in tks)
    done_inst = 256 * len(ran)                       # the requests that ran form a prefix
    o = out.cpu().numpy()
    assert np.array_equal(o[:done_inst // 2], outr[:done_inst // 2])
    assert (o[done_inst // 2:] == 777).all()         # cancelled outputs never written
    st = s.stats()
    assert st["cancelled"] == len(cancelled) and st["completed"] == len(ran)
    # destroy with requests still queued: close drains them first
    s2 = fnt.Session(max_channels=1, hbm_budget_bytes=16 << 20, chunk_blocks=1)
    s2.add_channel(0, cp, ap)
    out2 = torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev)
    note("session destroy with requests in flight")
    for o0, n in segs:
        s2.submit(0, x[o0:o0 + n], out2[o0 // 2:(o0 + n) // 2])
    s2.close()
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), outr)
    s.close()
    fnt.fnt_check()


def test_allocation_failure_leaves_sessions_usable(torch_dev):
    """A session or plan whose device memory cannot be allocated fails with
    FNT_E_NOMEM and frees what it took; a session created before keeps working."""
    torch, dev = torch_dev
    ch = synth.gen_channel(16 * 40, 55.0, 22.0, seed=95)
    x = to_dev(torch, dev, ch.samples)
    cp, ap = fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch))
    outr, _ = _oracle_stream(ch)
    s = fnt.Session(max_channels=2, hbm_budget_bytes=16 << 20, chunk_blocks=4)
    s.add_channel(0, cp, ap)
    out = torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev)
    half = ch.n // 64 * 32
    s.wait(s.submit(0, x[:half], out[:half // 2]))
    free0, _ = torch.cuda.mem_get_info()
    note("session with an HBM budget beyond the device")
    for _ in range(2):
        with pytest.raises(fnt.FntError) as e:
            fnt.Session(max_channels=4, hbm_budget_bytes=1 << 50, chunk_blocks=8)
        assert e.value.code == fnt.FNT_E_NOMEM
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < (64 << 20)       # nothing of the failed sessions is left behind
    # the first session continues its channel's stream, bit-exact
    s.wait(s.submit(0, x[half:], out[half // 2:]))
    assert np.array_equal(out.cpu().numpy(), outr)
    s.close()
    fnt.fnt_check()


def test_session_alone_equals_in_mix(torch_dev):
    torch, dev = torch_dev
    chans = _session_channels(12, 60, seed=5)
    target = 4

    def run(which):
        s = fnt.Session(max_channels=16, hbm_budget_bytes=64 << 20, chunk_blocks=3, max_active=5)
        outs = {}
        for c in which:
            ch, segs = chans[c]
            s.add_channel(c, fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch)))
            outs[c] = torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev)
        xs = {c: to_dev(torch, dev, chans[c][0].samples) for c in which}
        for c in which:
            off = 0
            for n in chans[c][1]:
                s.submit(c, xs[c][off:off + n], outs[c][off // 2:(off + n) // 2])
                off += n
        s.drain()
        s.close()
        return outs[target].cpu().numpy()

    note("session alone")
    alone = run([target])
    note("session in mix")
    mixed = run(list(range(12)))
    assert np.array_equal(alone, mixed)
    assert np.array_equal(alone, _oracle_stream(chans[target][0])[0])
    fnt.fnt_check()


def test_session_host_buffers_admission_and_errors(torch_dev):
    torch, dev = torch_dev
    chans = _session_channels(3, 30, seed=8)
    fixed = 3 * 2 * 8 * 64 + 4 * fnt.FNT_STATE_BYTES
    biggest = max(sum(segs) for _, segs in chans)
    with pytest.raises(fnt.FntError):
        fnt.Session(max_channels=4, hbm_budget_bytes=64 << 20, chunk_blocks=8, aeq_form=7)
    # staging pool that holds roughly one request at a time
    s = fnt.Session(max_channels=4, hbm_budget_bytes=fixed + 8 * biggest + 4096, chunk_blocks=8, max_active=2)
    host_out = {}
    keep = []
    for c, (ch, segs) in enumerate(chans):
        s.add_channel(c, fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch)))
        host_out[c] = np.zeros((ch.n // 2, 4), np.int16)
        off = 0
        for n in segs:
            xin = np.ascontiguousarray(ch.samples[off:off + n])
            o = host_out[c][off // 2:(off + n) // 2]
            keep.append(xin)
            note(f"session host submit ch={c} n={n}")
            s.submit(c, xin, o, host=True)
            off += n
    s.drain()
    for c, (ch, _) in enumerate(chans):
        assert np.array_equal(host_out[c], _oracle_stream(ch)[0]), c
    # a request larger than the whole pool is refused
    big = np.zeros((64 * biggest, 4), np.int8)
    with pytest.raises(fnt.FntError) as e:
        s.submit(0, big, np.zeros((32 * biggest, 4), np.int16), host=True)
    assert e.value.code == fnt.FNT_E_BUSY
    with pytest.raises(fnt.FntError) as e:
        s.submit(0, np.zeros((33, 4), np.int8), np.zeros((16, 4), np.int16), host=True)
    assert e.value.code == fnt.FNT_E_INVAL
    with pytest.raises(fnt.FntError) as e:
        s.submit(3, np.zeros((32, 4), np.int8), np.zeros((16, 4), np.int16), host=True)
    assert e.value.code == fnt.FNT_E_STATE
    s.close()
    fnt.fnt_check()


def test_session_replay_poisson(torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(4)
    nch = 16
    chans = []
    for c in range(nch):
        ch = synth.gen_channel(16 * int(rng.integers(20, 200)), float(rng.uniform(10, 80)), 22.0, seed=c + 500)
        chans.append(ch)
    s = fnt.Session(max_channels=nch, hbm_budget_bytes=64 << 20, chunk_blocks=16)
    outs, xs, reqs = [], [], []
    t = 0
    for c, ch in enumerate(chans):
        s.add_channel(c, fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**synth.aeq_params_for(ch)))
        xs.append(to_dev(torch, dev, ch.samples))
        outs.append(torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev))
    # two requests per channel, Poisson arrivals at 20k/s
    half = [ch.n // 64 * 32 for ch in chans]
    for rep in range(2):
        for c in range(nch):
            t += int(rng.exponential(50_000))
            lo = 0 if rep == 0 else half[c]
            hi = half[c] if rep == 0 else chans[c].n
            reqs.append((c, xs[c][lo:hi], outs[c][lo // 2:hi // 2], t))
    note("session replay")
    s.replay(reqs)
    s.drain()
    for c, ch in enumerate(chans):
        assert np.array_equal(outs[c].cpu().numpy(), _oracle_stream(ch)[0]), c
    st = s.stats()
    assert st["completed"] == len(reqs)
    s.close()
    fnt.fnt_check()


# ------------------------------------------------------------------ full size --
def test_full_size_single_stream(torch_dev):
    """2^24 symbols per polarisation, 75 km: the benchmark's workload and launch path."""
    torch, dev = torch_dev
    note("generate 2^24-symbol channel")
    ch = synth.single_channel(1 << 24, tag="bench")
    prm = synth.aeq_params_for(ch)
    x = to_dev(torch, dev, ch.samples)
    taps = to_dev(torch, dev, synth.centre_spike_taps())
    note("fnt_cdc_aeq 2^24 symbols")
    out = fnt.fnt_cdc_aeq(x, fnt.cdc_params(ch.taps, ch.requant_shift), taps, fnt.aeq_params(**prm))
    torch.cuda.synchronize()
    fnt.fnt_check()
    note("oracle 2^24 symbols")
    outr, wr, ar = O.cdc_aeq(ch.samples, ch.taps, ch.requant_shift, synth.centre_spike_taps(), O.params(**prm))
    assert np.array_equal(out.cpu().numpy(), outr)
    assert np.array_equal(taps.cpu().numpy(), wr)
    # exact CDC at sampled windows (the oracle with the preceding 32 instants as history)
    z, a = fnt.fnt_cdc(x, fnt.cdc_params(ch.taps, ch.requant_shift))
    zc = z.cpu().numpy()
    assert np.array_equal(a.cpu().numpy(), ar)
    rng = np.random.default_rng(0)
    for start in rng.integers(32, ch.n - 4096, size=8):
        seg = ch.samples[start:start + 4096]
        zr, _ = O.cdc(seg, ch.taps, ch.requant_shift, hist=ch.samples[start - 32:start])
        assert np.array_equal(zc[start:start + 4096], zr)


# ------------------------------------------------------- RDE step schedule --
def _gear(prm, mu, late, gear):
    return dict(prm, mu_shift=mu, mu_shift_late=late, gear_blocks=gear)


def test_step_schedule_every_form(torch_dev):
    """The step schedule (mu_shift before stream block gear_blocks, mu_shift_late
    after) in every AEQ kernel: the batched forms and variants, the fused
    schedules, fnt_aeq and fnt_cdc_aeq, against the oracle."""
    torch, dev = torch_dev
    chans = _batch(12, 6, 10, seed=123)
    pc = _plan_channels(torch, dev, chans, None)
    gears = [1, 7, 7, 3, 10 ** 6, 0, 7, 2, 7, 5, 40, 7]
    for c, g in zip(pc, gears):
        c["prm"] = _gear(c["prm"], 2, 6, g)
    refs = [O.cdc_aeq(c["ch"].samples, c["ch"].taps, c["ch"].requant_shift, c["w0"], O.params(**c["prm"]))
            for c in pc]
    entries = [(c["x"], c["out"], c["taps"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift),
                fnt.aeq_params(**c["prm"])) for c in pc]
    plan = fnt.Plan(entries, autotune=False, use_graph=True)

    def check(what):
        for c in pc:
            c["taps"].copy_(to_dev(torch, dev, c["w0"]))
            c["out"].fill_(-3)
        note(f"step schedule: {what}")
        plan.run()
        torch.cuda.synchronize()
        fnt.fnt_check()
        for i, (c, (outr, wr, _)) in enumerate(zip(pc, refs)):
            assert np.array_equal(c["out"].cpu().numpy(), outr), (what, i)
            assert np.array_equal(c["taps"].cpu().numpy(), wr), (what, i)

    for form in (0, 3, 1, 2, 4, 5):
        plan.set_aeq_waves(form)
        check(f"form {form}")
    for variant in (1, 2, 3):
        plan.set_aeq_variant(variant)
        check(f"variant {variant}")
    plan.set_aeq_variant(0)
    for lpt, split in ((4, False), (8, False), (16, True)):
        plan.set_fused(lpt, 2, split)
        check(f"fused lpt {lpt} split {split}")
    plan.close()
    # single-channel calls
    c = pc[1]
    outr, wr, ar = refs[1]
    taps = to_dev(torch, dev, c["w0"])
    note("step schedule: fnt_cdc_aeq and fnt_aeq")
    out = fnt.fnt_cdc_aeq(c["x"], fnt.cdc_params(c["ch"].taps, c["ch"].requant_shift), taps,
                          fnt.aeq_params(**c["prm"]))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), outr) and np.array_equal(taps.cpu().numpy(), wr)
    taps.copy_(to_dev(torch, dev, c["w0"]))
    out2 = fnt.fnt_aeq(to_dev(torch, dev, ar), taps, fnt.aeq_params(**c["prm"]))
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), outr) and np.array_equal(taps.cpu().numpy(), wr)
    with pytest.raises(fnt.FntError) as e:
        fnt.fnt_aeq(to_dev(torch, dev, ar), taps, fnt.aeq_params(**_gear(c["prm"], 2, 41, 3)))
    assert e.value.code == fnt.FNT_E_INVAL
    fnt.fnt_check()


@pytest.mark.parametrize("form", [-1, 1, 0])
def test_session_step_schedule_across_segments(torch_dev, form):
    """Sessions count the step schedule's blocks over the whole stream: segments of
    one to a few blocks cross gear_blocks mid-stream, and a state exported and
    imported into another session continues the count."""
    torch, dev = torch_dev
    chans = _session_channels(4, 6, seed=9)
    s = fnt.Session(max_channels=4, hbm_budget_bytes=64 << 20, chunk_blocks=2, aeq_form=form)
    outs, prms = [], []
    for c, (ch, segs) in enumerate(chans):
        prm = _gear(synth.aeq_params_for(ch), 2, 6, 3 + 2 * c)
        prms.append(prm)
        s.add_channel(c, fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**prm))
        outs.append(torch.zeros((ch.n // 2, 4), dtype=torch.int16, device=dev))
    xs = [to_dev(torch, dev, ch.samples) for ch, _ in chans]
    note(f"session step schedule, AEQ form {form}")
    for c, (ch, segs) in enumerate(chans):
        off = 0
        for k, n in enumerate(segs):
            if c == 0 and k == 1:                       # move channel 0 to another session mid-stream
                state = s.get_state(0)
                s2 = fnt.Session(max_channels=2, hbm_budget_bytes=16 << 20, chunk_blocks=3, aeq_form=form)
                s2.add_channel(1, fnt.cdc_params(ch.taps, ch.requant_shift), fnt.aeq_params(**prms[0]))
                s2.set_state(1, state)
                s2.wait(s2.submit(1, xs[c][off:off + n], outs[c][off // 2:(off + n) // 2]))
                s.set_state(0, s2.get_state(1))
                s2.close()
            else:
                s.wait(s.submit(c, xs[c][off:off + n], outs[c][off // 2:(off + n) // 2]))
            off += n
    s.drain()
    for c, (ch, segs) in enumerate(chans):
        outr, _, _ = O.cdc_aeq(ch.samples, ch.taps, ch.requant_shift, synth.centre_spike_taps(), O.params(**prms[c]))
        assert np.array_equal(outs[c].cpu().numpy(), outr), c
    s.close()
    fnt.fnt_check()
