"""GPU parity at the full workload sizes, in the launch configurations the
benchmark uses, every channel compared with the oracle (OpenMP over channels on
the host cores, streamed in chunks to bound host memory).

* 4096 channels, log-uniform 2^12..2^20 symbols per polarisation, fibre
  U(10, 80) km, OSNR U(18, 26) dB: one autotuned plan, hipGraph replay and the
  staged launches; 4096/4096 channels bit-exact.
* 16384 channels, log-uniform 2^14..2^22 symbols (about 2^34.5 instants, every
  channel generated from its own seed): one plan with quick autotuning;
  16384/16384 channels bit-exact.
* Serving: 1024 persistent channels, Poisson arrivals at 20 k requests/s for
  0.5 s, segments log-uniform 2^13..2^18 symbols; every channel's outputs equal
  the oracle's over its whole concatenated stream (1024/1024).
"""
import os
import time

import numpy as np
import pytest

import oracle as O
from paper_2405_04253_amd import fnt, synth

pytestmark = pytest.mark.gpu

THREADS = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)


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


def oracle_every_channel(what, samples, taps, shifts, prms, outs, finals, chunk_instants=1 << 28):
    """Compare every channel's GPU output and final taps with the oracle, in chunks
    of about chunk_instants instants (OpenMP over the chunk's channels)."""
    n = len(samples)
    done, ok, t0 = 0, 0, time.perf_counter()
    i = 0
    while i < n:
        j, tot = i, 0
        while j < n and (tot == 0 or tot + samples[j].shape[0] <= chunk_instants):
            tot += samples[j].shape[0]
            j += 1
        jobs = [dict(samples=samples[k].cpu().numpy(), taps=taps[k], shift=shifts[k], phase=0,
                     w=synth.centre_spike_taps(), params=O.params(**prms[k])) for k in range(i, j)]
        ref_out, ref_w, _ = O.batch(jobs, threads=THREADS)
        for k in range(i, j):
            good = (np.array_equal(outs[k].cpu().numpy(), ref_out[k - i]) and
                    np.array_equal(finals[k].cpu().numpy(), ref_w[k - i]))
            assert good, f"{what}: channel {k} ({samples[k].shape[0]} instants) differs from the oracle"
            ok += 1
        done = j
        note(f"{what}: {done}/{n} channels checked ({time.perf_counter() - t0:.0f} s)")
        i = j
    note(f"{what}: {ok}/{n} channels bit-exact")
    return ok


def test_full_size_batched_4096(torch_dev):
    torch, dev = torch_dev
    t0 = time.perf_counter()
    specs = synth.batched_specs(4096, 12, 20, tag="bench-batched")
    _, chans = synth.gen_batch_torch(specs, dev)
    torch.cuda.synchronize()
    note(f"4096-channel batch: generated in {time.perf_counter() - t0:.1f} s")
    w0 = torch.from_numpy(synth.centre_spike_taps()).to(dev)
    taps_all = w0.unsqueeze(0).repeat(len(chans), 1, 1, 1).contiguous()
    prms, entries = [], []
    for i, (q, taps, sh, unit) in enumerate(chans):
        prm = dict(synth.AEQ_DEFAULTS, const_unit=unit)
        prms.append(prm)
        out = torch.full((q.shape[0] // 2, 4), -1, dtype=torch.int16, device=dev)
        entries.append((q, out, taps_all[i], fnt.cdc_params(taps, sh), fnt.aeq_params(**prm)))
    note("4096-channel batch: plan with autotuning")
    plan = fnt.Plan(entries, autotune=True, use_graph=True)
    note(f"4096-channel batch: {plan.info()}")
    # the two stages launched directly
    plan.run_stage(fnt.FNT_STAGE_CDC)
    plan.run_stage(fnt.FNT_STAGE_AEQ)
    torch.cuda.synchronize()
    fnt.fnt_check()
    staged = [e[1].clone() for e in entries]
    staged_taps = taps_all.clone()
    # the tuned schedule (graph replay, or direct launches with a lead) from the same taps
    taps_all.copy_(w0.unsqueeze(0).expand_as(taps_all))
    note("4096-channel batch: plan run")
    plan.run()
    torch.cuda.synchronize()
    fnt.fnt_check()
    assert torch.equal(taps_all, staged_taps)
    assert all(torch.equal(e[1], s) for e, s in zip(entries, staged))
    # and the fused persistent schedule
    plan.set_fused(4, 512)
    taps_all.copy_(w0.unsqueeze(0).expand_as(taps_all))
    note("4096-channel batch: fused schedule")
    plan.run()
    torch.cuda.synchronize()
    fnt.fnt_check()
    assert torch.equal(taps_all, staged_taps)
    assert all(torch.equal(e[1], s) for e, s in zip(entries, staged))
    plan.close()
    ok = oracle_every_channel("4096-channel batch", [c[0] for c in chans], [c[1] for c in chans],
                              [c[2] for c in chans], prms, [e[1] for e in entries], taps_all)
    assert ok == 4096


LARGE_PARTS = 16
_large = {}


@pytest.fixture(scope="module")
def large_batch(torch_dev):
    """The 16384-channel batch generated, planned (quick autotuning) and run once;
    the parts below compare it with the oracle a sixteenth at a time."""
    torch, dev = torch_dev
    if "chans" in _large:
        return _large
    t0 = time.perf_counter()
    specs = synth.batched_specs(16384, 14, 22, tag="large")

    def prog(done, total):
        if done % 2048 < 8 or done == total:
            note(f"16384-channel batch: generated {done}/{total} ({time.perf_counter() - t0:.0f} s)")

    _, chans = synth.gen_batch_torch(specs, dev, progress=prog)
    torch.cuda.synchronize()
    total = sum(c[0].shape[0] for c in chans)
    note(f"16384-channel batch: {total} instants ({total / 2 ** 34:.2f} x 2^34) in "
         f"{time.perf_counter() - t0:.0f} s")
    w0 = torch.from_numpy(synth.centre_spike_taps()).to(dev)
    taps_all = w0.unsqueeze(0).repeat(len(specs), 1, 1, 1).contiguous()
    entries, prms = [], []
    for i, (q, taps, sh, unit) in enumerate(chans):
        prm = dict(synth.AEQ_DEFAULTS, const_unit=unit)
        out = torch.empty((q.shape[0] // 2, 4), dtype=torch.int16, device=dev)
        prms.append(prm)
        entries.append((q, out, taps_all[i], fnt.cdc_params(taps, sh), fnt.aeq_params(**prm)))
    note("16384-channel batch: plan with quick autotuning")
    plan = fnt.Plan(entries, autotune=True, use_graph=True, tune_quick=True)
    info = plan.info()
    assert info["instants"] == total and info["channels"] == len(specs)
    note(f"16384-channel batch: {info}")
    taps_all.copy_(w0.unsqueeze(0).expand_as(taps_all))
    note("16384-channel batch: run")
    t1 = time.perf_counter()
    plan.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    fnt.fnt_check()
    note(f"16384-channel batch: {dt:.2f} s, {total / dt / 1e9:.2f} Gsamples/s")
    plan.close()
    _large.update(chans=chans, prms=prms, outs=[e[1] for e in entries], taps=taps_all, ok=0)
    return _large


@pytest.mark.parametrize("part", range(LARGE_PARTS))
def test_full_size_large_batch_16384(large_batch, part):
    """Channels part, part + 16, part + 32, ... of the 16384 (every length range in
    every part), each against the oracle."""
    chans, idx = large_batch["chans"], list(range(part, len(large_batch["chans"]), LARGE_PARTS))
    ok = oracle_every_channel(f"16384-channel batch, part {part + 1}/{LARGE_PARTS}",
                              [chans[i][0] for i in idx], [chans[i][1] for i in idx], [chans[i][2] for i in idx],
                              [large_batch["prms"][i] for i in idx], [large_batch["outs"][i] for i in idx],
                              large_batch["taps"][idx])
    assert ok == len(idx)
    large_batch["ok"] += ok
    if part == LARGE_PARTS - 1:
        note(f"16384-channel batch: {large_batch['ok']}/{len(chans)} channels bit-exact")
        assert large_batch["ok"] == len(chans)
        large_batch.clear()


def test_full_size_served_1024(torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(12345)
    nch, rate, window = 1024, 20000.0, 0.5
    times, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window:
            break
        times.append(t)
    seg = [16 * max(1, int(2 ** rng.uniform(13, 18)) // 16) for _ in times]
    owner = rng.integers(0, nch, size=len(times))
    per = np.zeros(nch, np.int64)
    for i, c in enumerate(owner):
        per[c] += seg[i]
    t0 = time.perf_counter()
    streams, params = {}, {}
    sess = fnt.Session(max_channels=nch, hbm_budget_bytes=1 << 30, chunk_blocks=512, max_active=nch)
    for c in range(nch):
        r = np.random.default_rng(synth.seed_for(0, "served", c))
        km, osnr = float(r.uniform(10, 80)), float(r.uniform(18, 26))
        q, taps, sh, unit = synth.gen_channel_torch(max(int(per[c]), 16), km, osnr,
                                                    synth.seed_for(1, "served", c), dev)
        streams[c] = q
        prm = dict(synth.AEQ_DEFAULTS, const_unit=unit)
        params[c] = (taps, sh, prm)
        sess.add_channel(c, fnt.cdc_params(taps, sh), fnt.aeq_params(**prm))
        if c % 256 == 0:
            torch.cuda.synchronize()
            note(f"served: generated {c} streams ({time.perf_counter() - t0:.1f} s)")
    outs = {c: torch.full((streams[c].shape[0] // 2, 4), -1, dtype=torch.int16, device=dev) for c in range(nch)}
    reqs, offs = [], [0] * nch
    for i in range(len(times)):
        c = int(owner[i])
        n = 2 * seg[i]
        o = offs[c]
        reqs.append((c, streams[c][o:o + n], outs[c][o // 2:(o + n) // 2], int(times[i] * 1e9)))
        offs[c] += n
    torch.cuda.synchronize()
    note(f"served: replaying {len(reqs)} requests")
    sess.replay(reqs)
    sess.drain()
    st = sess.stats()
    sess.close()
    fnt.fnt_check()
    assert st["completed"] == len(reqs)
    note(f"served: {st['gsamples_per_s']:.2f} Gsamples/s, p50 {st['p50_us']:.0f} us, p99 {st['p99_us']:.0f} us")
    # every channel over its whole concatenated stream
    chs = [c for c in range(nch) if offs[c] > 0]
    jobs_samples = [streams[c][:offs[c]] for c in chs]
    ref_final = [None] * len(chs)       # final taps stay in the session: outputs only here
    ok, i0 = 0, 0
    while i0 < len(chs):
        i1, tot = i0, 0
        while i1 < len(chs) and (tot == 0 or tot + jobs_samples[i1].shape[0] <= (1 << 28)):
            tot += jobs_samples[i1].shape[0]
            i1 += 1
        jobs = [dict(samples=jobs_samples[k].cpu().numpy(), taps=params[chs[k]][0], shift=params[chs[k]][1],
                     phase=0, w=synth.centre_spike_taps(), params=O.params(**params[chs[k]][2]))
                for k in range(i0, i1)]
        ref_out, _, _ = O.batch(jobs, threads=THREADS)
        for k in range(i0, i1):
            c = chs[k]
            assert np.array_equal(outs[c][: offs[c] // 2].cpu().numpy(), ref_out[k - i0]), f"served channel {c}"
            ok += 1
        note(f"served: {i1}/{len(chs)} channels checked")
        i0 = i1
    note(f"served: {ok}/{len(chs)} channels with requests bit-exact ({nch - len(chs)} without requests)")
    assert ok == len(chs)
