#!/usr/bin/env python3
"""Throughput of the FNT-CDC + FNT-AEQ receiver path on one MI355X.

Headline workload ("batched"): 4096 independent channels in one plan, lengths
log-uniform 2^12..2^20 PDM-16QAM symbols per polarisation at 2 samples/symbol,
fibre U(10, 80) km (8-32 six-bit CD-inverse taps), OSNR U(18, 26) dB, 5-bit
samples, N = 64 FNT mod 65537 with alpha = sqrt 2 for the CDC, then resample,
requantise and the N = 32 FNT-AEQ with the RDE update.  A step is one pass of
the whole path over every channel, inputs resident in HBM; the taps restart
from the centre spike at each step.

Reported beside it: the plain single-stream path (one channel of 2^24 symbols,
75 km: the comparator the batched figure is set against), the plain
per-channel launch loop on a sample of the same channels, and a served
workload (Poisson arrivals into a session; p50/p99 latency).

Prints one JSON line.  Gsamples/s counts instants (one dual-polarisation
2-samples/symbol sample = 4 int8).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
# Vector ALU peak from the chip's unit counts and clock: the published fp32 vector
# rate (157.3 TFLOP/s) with an FMA counted as one operation, 256 CUs x 4 SIMDs x 32
# lane-operations per cycle x 2.4 GHz = 78643.2 G lane-ops/s.  That rate is reached
# by packed (two-wide) fp32 instructions on 16-lane SIMDs; 32-bit integer
# instructions have no packed form, so the chip's own rates are set beside it
# (measured_peaks): v_add_u32 ~57.9 T, the SDWA fold / shift / 24-bit multiply
# forms ~37.1 T (16 lanes per cycle).
PEAK_ALU_GOPS = 256 * 4 * 32 * 2.4

# Algorithmic integer operations of the method, per unit: a modular add, subtract,
# shift, product or an integer multiply-accumulate counts one.
FNT64_OPS = 384 + 129            # 192 butterflies (add + sub) + 129 nontrivial twiddles
FNT32_OPS = 160 + 49             # 80 butterflies + 49 twiddles
# CDC, per block of 32 new instants and one polarisation: packing u, v (128),
# forward FNT64 x 2, products (128), P +- Q (128), the inverse folded to the kept
# 1-sps outputs (two 32-point inverses of the folded spectra: 2 x (209 + 32)) and
# scale/lift (64)
CDC_OPS_PER_POL_BLOCK = 128 + 2 * FNT64_OPS + 128 + 128 + 2 * (FNT32_OPS + 32) + 64      # 1956
CDC_OPS_PER_BLOCK = 2 * CDC_OPS_PER_POL_BLOCK                                             # 3912
# AEQ, per block of 16 symbols (= 32 instants): input FNT32 x 4, tap-digit
# re-transform 32 x FNT32, products (1024), pair sums (512) + 16 inverse FNT32,
# RDE error (~400), gradient MACs (4096), tap update (~512)
AEQ_OPS_PER_BLOCK = (4 * FNT32_OPS + 32 * FNT32_OPS + 1024 + (512 + 16 * FNT32_OPS)
                     + 400 + 4096 + 512)                                                   # 17412
METRIC = "bit-exact Gsamples/s, batched/served vs plain FNT-CDC+AEQ; p50/p99 latency"
CDC_BYTES_PER_INSTANT = 4 + 2              # int8[4] in, int8[4] per symbol out
AEQ_BYTES_PER_SYMBOL = 4 + 8               # int8[4] in, int16[4] out
FUSED_BYTES_PER_INSTANT = 4 + 4            # int8[4] in, int16[4] per symbol (2 instants) out


def kernel_source_hash() -> str:
    """Hash of the device code's source without comments and blank lines, so that
    a profile summary stays tied to the code it measured but not to its prose."""
    h = hashlib.sha256()
    for f in ("fnt_kernels.hip", "fnt_device.hpp"):
        with open(os.path.join(ROOT, "paper_2405_04253_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code.strip():
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, blocks: int | None = None, per_block: bool = False):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source, and where it comes from; (None, reason)
    otherwise.  Given `blocks`, a launch of another number of AEQ blocks gets the
    profiled bytes per block times its blocks if `per_block`, else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(p))
    except Exception:
        return None, "no counter summary"
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None, "no counters taken on the current kernel source"
    nb = e.get("aeq_blocks")
    if blocks is None or nb in (None, blocks):
        return e.get("bytes_per_launch"), "rocprofv3 FETCH_SIZE + WRITE_SIZE of this launch, copy-calibrated"
    if per_block and nb:
        return (round(e["bytes_per_launch"] * blocks / nb),
                f"rocprofv3 FETCH_SIZE + WRITE_SIZE per block of a profiled {nb}-block launch of this kernel, "
                f"times {blocks} blocks")
    return None, "profiled launch had another block count"


def cpu_baseline_single(ch, prm, budget_s: float):
    """The oracle, single-threaded (the AEQ is a serial chain), on a bounded prefix."""
    import oracle as O
    from paper_2405_04253_amd import synth
    nsym = ch.n // 2
    # size the sample from a short calibration run
    probe = min(nsym, 1 << 16)
    t0 = time.perf_counter()
    O.cdc_aeq(ch.samples[: 2 * probe], ch.taps, ch.requant_shift, synth.centre_spike_taps(), O.params(**prm))
    rate = probe / max(time.perf_counter() - t0, 1e-6)
    take = int(min(nsym, max(probe, rate * budget_s)))
    take -= take % 16
    t0 = time.perf_counter()
    O.cdc_aeq(ch.samples[: 2 * take], ch.taps, ch.requant_shift, synth.centre_spike_taps(), O.params(**prm))
    dt = time.perf_counter() - t0
    return {"value": round(2 * take / dt / 1e9, 6), "unit": "Gsamples/s", "cores": 1, "kind": "oracle",
            "sample": f"first {take} symbols/pol ({2 * take} instants) of the workload, CDC+AEQ, "
                      f"single thread, {dt:.1f} s"}


def bench_single(args, torch, dev):
    from paper_2405_04253_amd import fnt, synth
    t0 = time.perf_counter()
    ch = synth.single_channel(1 << args.log2_symbols, tag="bench")
    gen_s = time.perf_counter() - t0
    prm = synth.aeq_params_for(ch)
    n = ch.n
    M = n // 2
    x = torch.from_numpy(ch.samples).to(dev)
    w0 = torch.from_numpy(synth.centre_spike_taps()).to(dev)
    taps = w0.clone()
    a = torch.empty((M, 4), dtype=torch.int8, device=dev)
    out = torch.empty((M, 4), dtype=torch.int16, device=dev)
    cp = fnt.cdc_params(ch.taps, ch.requant_shift)
    ap = fnt.aeq_params(**prm)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        taps.copy_(w0)                      # fresh adaptive state every step
        if ev is not None:
            ev[0].record(stream)
        fnt.fnt_cdc(x, cp, exact=False, a_out=a, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        fnt.fnt_aeq(a, taps, ap, out=out, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    progress(f"single: generated {n} instants in {gen_s:.1f} s; warmup")
    for _ in range(1):
        step()
    torch.cuda.synchronize()
    fnt.fnt_check()
    steps = max(1, args.single_steps)
    progress(f"single: timing {steps} steps")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fnt.fnt_check()
    cdc_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    aeq_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms = wall / steps * 1e3
    # the same chain as ONE launch (fnt_cdc_aeq: the fused kernel, one workgroup per
    # polarisation half, the 1-sps stream kept in LDS), same outputs bit for bit
    ref_out, ref_taps = out.clone(), taps.clone()
    out1 = torch.empty_like(out)

    def one():
        taps.copy_(w0)
        fnt.fnt_cdc_aeq(x, cp, taps, ap, out=out1, stream=stream)

    one()
    torch.cuda.synchronize()
    fnt.fnt_check()
    if not (torch.equal(out1, ref_out) and torch.equal(taps, ref_taps)):
        raise SystemExit("single stream: fnt_cdc_aeq differs from fnt_cdc + fnt_aeq")
    one_ms = _time_events(torch, one, max(1, steps - 1), stream)
    blocks_cdc = (n + 31) // 32
    blocks_aeq = (M + 15) // 16
    aeq_ops = AEQ_OPS_PER_BLOCK * blocks_aeq
    cdc_ops = CDC_OPS_PER_BLOCK * blocks_cdc
    kernels = {
        "cdc": {"ms": round(cdc_ms, 4),
                "gbs": round(n * CDC_BYTES_PER_INSTANT / cdc_ms / 1e6, 2),
                "gops": round(cdc_ops / cdc_ms / 1e6, 2)},
        "aeq": {"ms": round(aeq_ms, 4),
                "gbs": round(M * AEQ_BYTES_PER_SYMBOL / aeq_ms / 1e6, 2),
                "gops": round(aeq_ops / aeq_ms / 1e6, 2),
                "us_per_block": round(aeq_ms * 1e3 / blocks_aeq, 4)},
    }
    achieved = aeq_ops / (aeq_ms / 1e3) / 1e9
    roof = {"kernel": "aeq_pol_kernel<16, 1>", "bound": "alu", "achieved": round(achieved, 3),
            "peak": PEAK_ALU_GOPS, "unit": "Gops/s", "frac": round(achieved / PEAK_ALU_GOPS, 6),
            "traffic": load_traffic("aeq_pol_kernel<16, 1>", "single", blocks_aeq)[0],
            "algorithmic_ops_per_launch": aeq_ops}
    res = {
        "value": round(n / (ms / 1e3) / 1e9, 6), "unit": "Gsamples/s",
        "steps": steps, "ms_per_step": round(ms, 3),
        "workload": "plain single-stream FNT-CDC+AEQ (fnt_cdc then fnt_aeq), 1 channel x 2^%d "
                    "symbols/pol, 75 km, 32 taps" % args.log2_symbols,
        "instants": n, "roofline": roof, "kernels": kernels, "gen_s": round(gen_s, 1),
        "one_launch": {"value": round(n / (one_ms / 1e3) / 1e9, 6), "unit": "Gsamples/s", "ms": round(one_ms, 3),
                       "kernel": "cdc_aeq_fused_kernel<16, 4, 1>",
                       "what": "fnt_cdc_aeq: CDC and AEQ in one launch, the 1-sps stream in LDS; bit-identical "
                               "to the two launches"},
        "launches": [launch_entry("cdc_lane_kernel<4>", "cdc_lane_kernel<4>", 0, blocks_cdc, n),
                     launch_entry("aeq_pol_kernel<16, 1>", "aeq_pol_kernel<16, 1>", blocks_aeq),
                     launch_entry("cdc_aeq_fused_kernel<16, 4, 1>", "cdc_aeq_fused_kernel<16, 4, 1>", blocks_aeq,
                                  blocks_cdc, n)],
    }
    if args.single_cpu_baseline:
        progress("single: oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline_single(ch, prm, args.cpu_budget)
    return res


# FNT128: 448 butterflies (add + sub) + 321 nontrivial twiddles (stage of span h:
# (h - 1) N / 2h of them)
FNT128_OPS = 896 + 321
# CDC with N = 128 and 3-bit tap digits, per block of 64 new instants and one
# polarisation: packing u, v (256), forward FNT128 x 2, products (2 digits x P, Q:
# 512), P +- Q (512), four inverses, scale / lift / digit combine (4 per output: 256)
CDC_LONG_OPS_PER_POL_BLOCK = 256 + 2 * FNT128_OPS + 512 + 512 + 4 * FNT128_OPS + 256
CDC_LONG_OPS_PER_BLOCK = 2 * CDC_LONG_OPS_PER_POL_BLOCK                                   # 17676


def bench_cdc_long(args, torch, dev):
    """fnt_cdc_long (N = 128, 65 taps of 3-bit digits) on one long-fibre channel,
    against fnt_cdc (N = 64, 32 taps) on the same samples."""
    import oracle as O
    from paper_2405_04253_amd import fnt, synth
    km = 150.0
    nsym = 1 << args.log2_symbols
    t0 = time.perf_counter()
    q, taps32, sh32, _ = synth.gen_channel_torch(nsym, km, 22.0, synth.seed_for(0, "cdc-long", 0), dev)
    taps65, sh65, _ = synth.design_cdc_taps(km, 65)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    n = q.shape[0]
    stream = torch.cuda.current_stream()
    res = {}
    for name, fn in (("long", lambda: fnt.fnt_cdc_long(q, taps65, sh65, 0, exact=False, stream=stream)),
                     ("n64", lambda: fnt.fnt_cdc(q, fnt.cdc_params(taps32, sh32), exact=False, stream=stream))):
        fn()
        torch.cuda.synchronize()
        fnt.fnt_check()
        res[name] = _time_events(torch, fn, 5, stream)
    # parity on a prefix (causal: the first outputs depend only on the first inputs)
    _, a = fnt.fnt_cdc_long(q, taps65, sh65, 0, exact=False, stream=stream)
    torch.cuda.synchronize()
    k = 1 << 17
    _, ar = O.cdc(q[:k].cpu().numpy(), taps65, sh65, 0)
    if not np.array_equal(a[: ar.shape[0]].cpu().numpy(), ar):
        raise SystemExit("fnt_cdc_long parity failure")
    blocks = (n + 63) // 64
    ops = CDC_LONG_OPS_PER_BLOCK * blocks
    achieved = ops / (res["long"] / 1e3) / 1e9
    return {"value": round(n / (res["long"] / 1e3) / 1e9, 3), "unit": "Gsamples/s", "ms": round(res["long"], 3),
            "workload": f"1 channel x 2^{args.log2_symbols} symbols/pol, {km:.0f} km, 65 taps (N = 128 FNT, "
                        f"3-bit tap digits), to the 5-bit 1-sps stream",
            "roofline": {"kernel": "cdc_long_kernel", "bound": "alu", "achieved": round(achieved, 1),
                         "peak": PEAK_ALU_GOPS, "unit": "Gops/s", "frac": round(achieved / PEAK_ALU_GOPS, 5),
                         "ops_per_unit": {"cdc_long_block_64_instants": CDC_LONG_OPS_PER_BLOCK}},
            "n64_32_taps": {"value": round(n / (res["n64"] / 1e3) / 1e9, 3), "ms": round(res["n64"], 3),
                            "kernel": "cdc_lane_kernel (fnt_cdc, N = 64, the 32-tap design)"},
            "parity": f"bit-exact vs oracle on the first {k} instants", "gen_s": round(gen_s, 1)}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _time_events(torch, fn, reps, stream):
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


AEQ_FORM_KERNEL = {0: "aeq_lane_kernel<1>", 3: "aeq_duo_kernel<1>", 1: "aeq_pol_kernel<4, 1>",
                   2: "aeq_pol_kernel<8, 1>", 4: "aeq_pol_kernel<16, 1>", 5: "aeq_pol_kernel<4, 2>"}
SPLIT_WPG = {1: 1, 3: 1, 2: 2, 4: 4, 5: 2}


def split_fusable(long_form: int, rest_form: int) -> bool:
    """Form pairs that run as one split launch (the library's table)."""
    return (long_form in (1, 2, 4, 5) and rest_form in (0, 3)) or (long_form, rest_form) in ((3, 0), (2, 5))


def split_name(long_form: int, rest_form: int) -> str:
    return "aeq_split_kernel<%d, %d, %d>" % (long_form, rest_form, SPLIT_WPG[long_form])


SCHEDULE_KEYS = ("cdc_variant", "cdc_waves_per_group", "cdc_blocks_per_wave", "aeq_variant", "aeq_waves_per_pol",
                 "aeq_waves_long", "aeq_long_channels", "lead_channels", "lead_form", "top_channels", "top_form",
                 "fused_lpt", "fused_prio_channels", "fused_split")


def apply_schedule(plan, s: dict):
    """Sets a plan's schedule from keys of Plan.info() (a stored tuner choice, or
    one written by hand for a profile); absent keys take the plan's defaults."""
    plan.set_cdc_schedule(int(s.get("cdc_waves_per_group", 2)), int(s.get("cdc_blocks_per_wave", 0)))
    plan.set_cdc_variant(int(s.get("cdc_variant", 0)))
    plan.set_aeq_variant(int(s.get("aeq_variant", 0)))
    if s.get("fused_lpt"):
        plan.set_fused(int(s["fused_lpt"]), int(s.get("fused_prio_channels", 0)), bool(s.get("fused_split", 0)))
        return
    plan.set_aeq_split(int(s.get("aeq_long_channels", 0)), int(s.get("aeq_waves_long", 1)),
                       int(s.get("aeq_waves_per_pol", 0)))
    plan.set_lead(int(s.get("lead_channels", 0)), int(s.get("lead_form", -1)), int(s.get("top_channels", 0)),
                  int(s.get("top_form", -1)))


def launch_entry(kernel, key, aeq_blocks=0, cdc_blocks=0, instants=0, grid=None):
    """One launch of a step: the kernel name as a kernel trace shows it, the key its
    counters are stored under, its units and their algorithmic work and bytes
    (AEQ 12 B per symbol, CDC 6 B per instant, the fused chain 8 B per instant)."""
    e = {"kernel": kernel, "key": key, "aeq_blocks": aeq_blocks, "cdc_blocks": cdc_blocks,
         "algorithmic_ops": AEQ_OPS_PER_BLOCK * aeq_blocks + CDC_OPS_PER_BLOCK * cdc_blocks}
    if grid is not None:
        e["grid"] = grid                    # threads of the launch, to tell launches of one kernel apart
    if aeq_blocks and cdc_blocks:
        e["algorithmic_bytes"] = instants * FUSED_BYTES_PER_INSTANT
    elif cdc_blocks:
        e["algorithmic_bytes"] = instants * CDC_BYTES_PER_INSTANT
    else:
        e["algorithmic_bytes"] = aeq_blocks * 16 * AEQ_BYTES_PER_SYMBOL
    return e


def launches_of(info, timing, kname, lead_name, top_name, aeq_blocks, lead_blocks, top_blocks, lengths):
    """The plan's launches in one step (launch_entry).  lengths: every channel's
    instants; the plan orders channels longest chain first (stable), and a lead
    runs the CDC of its segment as a launch of its own."""
    order = sorted(range(len(lengths)), key=lambda i: -((lengths[i] + 1) // 2))
    n = [lengths[i] for i in order]
    blocks = [(v + 31) // 32 for v in n]
    chunks = [(b + 63) // 64 for b in blocks]
    inst = sum(n)
    if timing["fused"]:
        wg = 64 * (2 * (info["fused_lpt"] // 4) + info["fused_lpt"] // 4) if not info["fused_split"] else None
        return [launch_entry(kname, kname, aeq_blocks, sum(blocks), inst,
                             grid=info["fused_grid"] * wg if wg else None)]
    wpg = info["cdc_waves_per_group"]
    cdc = ("cdc_lane_kernel<%d>" % wpg) if info["cdc_blocks_per_wave"] == 0 else "cdc_kernel<false>"
    if info["cdc_variant"] == 1:
        cdc = "cdc_direct_kernel<%d>" % wpg
    lane_cdc = info["cdc_blocks_per_wave"] == 0

    def seg(a, b, key):
        g = -(-sum(chunks[a:b]) // wpg) * 64 * wpg if lane_cdc else None
        return launch_entry(cdc, key, 0, sum(blocks[a:b]), sum(n[a:b]), grid=g)

    lead = info["lead_channels"]
    top = info["top_channels"] if top_name else 0
    if lead:
        out = ([seg(0, top, cdc + " (first level)")] if top else []) + \
              [seg(top, lead, cdc + " (lead)"), seg(lead, len(n), cdc)]
    else:
        out = [seg(0, len(n), cdc)]
    if "+" not in kname:
        out.append(launch_entry(kname, kname, aeq_blocks))
    if lead_name:
        out.append(launch_entry(lead_name, lead_name + " (lead)", lead_blocks))
    if top_name:
        out.append(launch_entry(top_name, top_name + " (first level)", top_blocks))
    return out


def aeq_kernel_name(info) -> str:
    """Kernel of the AEQ launch on the launch stream (the channels after a
    pipelined lead, or every channel)."""
    form = AEQ_FORM_KERNEL
    if info["aeq_variant"] == 0:
        wl, ws = info["aeq_waves_long"], info["aeq_waves_per_pol"]
        nlong = max(info["aeq_long_channels"] - info["lead_channels"], 0)
        rest = info["channels"] - info["lead_channels"]
        if nlong >= rest:
            return form[wl]
        if nlong and split_fusable(wl, ws):
            return split_name(wl, ws)                                   # one launch
        k = form[ws]
        if nlong:
            k = form[wl] + "+" + k
        return k
    if info["aeq_variant"] == 1:
        return "aeq_direct_kernel"
    return "aeq_fnt_kernel"                                             # variant 2


def cpu_baseline_batched(chans, prms, budget_s: float):
    """The oracle with OpenMP over channels on the host cores, on a random sample
    of the workload's channels sized to about `budget_s` of CPU time."""
    import oracle as O
    from paper_2405_04253_amd import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    rng = np.random.default_rng(11)
    order = [int(i) for i in rng.permutation(len(chans))]
    # single-thread rate from a short probe on the smallest sampled channel
    probe = min(order[:8], key=lambda i: chans[i][1].shape[0])
    q = chans[probe][1].cpu().numpy()
    t0 = time.perf_counter()
    O.cdc_aeq(q, chans[probe][2], chans[probe][3], synth.centre_spike_taps(), O.params(**prms[probe]))
    rate1 = q.shape[0] / max(time.perf_counter() - t0, 1e-6)
    want = rate1 * threads * budget_s
    pick, tot = [], 0
    for i in order:
        n = chans[i][1].shape[0]
        if tot + n > want and pick:
            continue
        pick.append(i)
        tot += n
        if tot >= 0.9 * want:
            break
    jobs = [dict(samples=chans[i][1].cpu().numpy(), taps=chans[i][2], shift=chans[i][3], phase=0,
                 w=synth.centre_spike_taps(), params=O.params(**prms[i])) for i in pick]
    t0 = time.perf_counter()
    _, _, used = O.batch(jobs, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(tot / dt / 1e9, 6), "unit": "Gsamples/s", "cores": used, "kind": "oracle",
            "sample": f"{len(pick)} random channels of the workload ({tot} instants), CDC+AEQ, "
                      f"OpenMP over channels, {dt:.1f} s"}


def bench_batched(args, torch, dev):
    """Many channels of log-uniform length in one plan (autotuned; hipGraph for plan.run)."""
    import oracle as O
    from paper_2405_04253_amd import fnt, synth
    t0 = time.perf_counter()
    specs = synth.batched_specs(args.nch, args.log2_min, args.log2_max, tag="bench-batched")
    chans = []
    for k, sp in enumerate(specs):
        q, taps, sh, unit = synth.gen_channel_torch(sp.nsym, sp.fibre_km, sp.osnr_db, sp.seed, dev)
        chans.append((sp, q, taps, sh, unit))
        if k % 512 == 0:
            torch.cuda.synchronize()
            progress(f"batched: generated {k + 1}/{len(specs)} channels ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    progress(f"batched: generation done in {gen_s:.1f} s")
    w0 = torch.from_numpy(synth.centre_spike_taps()).to(dev)
    taps_all = w0.unsqueeze(0).repeat(len(chans), 1, 1, 1).contiguous()
    entries, prms = [], []
    inst = 0
    for i, (sp, q, taps, sh, unit) in enumerate(chans):
        prm = dict(synth.AEQ_DEFAULTS, const_unit=unit)
        prms.append(prm)
        out = torch.empty((q.shape[0] // 2, 4), dtype=torch.int16, device=dev)
        entries.append((q, out, taps_all[i], fnt.cdc_params(taps, sh), fnt.aeq_params(**prm)))
        inst += q.shape[0]
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    sched = json.loads(args.schedule) if args.schedule else None
    progress(f"batched: plan create over {len(entries)} channels, " +
             (f"schedule {sched}" if sched else "autotuned"))
    plan = fnt.Plan(entries, autotune=sched is None, use_graph=True, stream=stream, tune_cache=args.tune_cache)
    if sched:
        apply_schedule(plan, sched)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    info = plan.info()
    progress(f"batched: plan ready in {tune_s:.1f} s: {info}")
    w_all = w0.unsqueeze(0).expand_as(taps_all)

    def step():
        taps_all.copy_(w_all)               # fresh adaptive state every step
        # the plan's launch sequence, launched directly with HIP events around
        # every launch on the stream it runs on (the lead's AEQ on the plan's
        # side stream); waits for the step to end
        return plan.run_timed(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fnt.fnt_check()
    progress(f"batched: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fnt.fnt_check()
    cdc_ms = float(np.mean([t["cdc_ms"] for t in times]))
    aeq_ms = float(np.mean([t["aeq_ms"] for t in times]))
    lead_ms = float(np.mean([t["aeq_lead_ms"] for t in times]))
    top_ms = float(np.mean([t["aeq_top_ms"] for t in times]))
    event_step_ms = float(np.mean([t["step_ms"] for t in times]))
    event_step_med = float(np.median([t["step_ms"] for t in times]))
    ms = wall / max(args.steps, 1) * 1e3
    progress(f"batched: {ms:.1f} ms per step (events {event_step_ms:.1f}: cdc {cdc_ms:.1f} ms, "
             f"aeq {aeq_ms:.1f} ms, lead aeq {lead_ms:.1f} ms, first-level aeq {top_ms:.1f} ms)")
    # fnt_plan_run of the same plan (the graph replay when no lead is in effect), for comparison
    taps_all.copy_(w_all)
    run_ms = _time_events(torch, plan.run, 2, stream)
    # the same schedule as a hipGraph replay (a lead's fork and join are events
    # inside the capture); the first replay uploads the graph and is not timed
    plan.run_graph(stream)
    torch.cuda.synchronize()
    graph_ms = _time_events(torch, lambda: plan.run_graph(stream), 3, stream)
    # parity on sampled channels: reset the taps, run once more, compare with the oracle
    taps_all.copy_(w_all)
    plan.run(stream)
    torch.cuda.synchronize()
    fnt.fnt_check()
    order = sorted(range(len(chans)), key=lambda i: chans[i][1].shape[0])
    pick = sorted(set([order[0], order[len(order) // 2], order[-1]]))
    progress(f"batched: parity on channels {pick}")
    for i in pick:
        sp, q, taps, sh, unit = chans[i]
        outr, wr, _ = O.cdc_aeq(q.cpu().numpy(), taps, sh, synth.centre_spike_taps(), O.params(**prms[i]))
        if not (np.array_equal(entries[i][1].cpu().numpy(), outr) and np.array_equal(taps_all[i].cpu().numpy(), wr)):
            raise SystemExit(f"batched parity failure on channel {i}")
    direct_out = {i: entries[i][1].clone() for i in pick}
    direct_taps = {i: taps_all[i].clone() for i in pick}
    taps_all.copy_(w_all)
    plan.run_graph(stream)
    torch.cuda.synchronize()
    fnt.fnt_check()
    for i in pick:
        if not (torch.equal(entries[i][1], direct_out[i]) and torch.equal(taps_all[i], direct_taps[i])):
            raise SystemExit(f"graph replay differs from the direct launches on channel {i}")
    plain_gsps = None
    fused = None
    if not args.no_comparisons:
        # plain comparator: the single-stream call (fnt_cdc_aeq) channel after channel, on
        # a random sample of channels; its rate over the sample stands for the loop
        rng = np.random.default_rng(7)
        sample = [int(i) for i in rng.choice(len(chans), size=min(32, len(chans)), replace=False)]
        tmp_taps = w0.clone()
        s_inst = sum(chans[i][1].shape[0] for i in sample)
        progress(f"batched: plain per-channel loop over {len(sample)} sampled channels")

        # the faster of the two plain single-channel paths on this GPU: fnt_cdc to the
        # 1-sps stream, then fnt_aeq (the one-launch fnt_cdc_aeq is timed in the
        # single-stream leg)
        abuf = torch.empty((max(chans[i][1].shape[0] for i in sample) // 2 + 1, 4), dtype=torch.int8, device=dev)

        def plain_loop():
            for i in sample:
                tmp_taps.copy_(w0)
                m = entries[i][1].shape[0]
                fnt.fnt_cdc(chans[i][1], entries[i][3], exact=False, a_out=abuf[:m], stream=stream)
                fnt.fnt_aeq(abuf[:m], tmp_taps, entries[i][4], out=entries[i][1], stream=stream)

        plain_ms = _time_events(torch, plain_loop, 1, stream)
        plain_gsps = s_inst / (plain_ms / 1e3) / 1e9
        # comparator: the same plan with the direct time-domain CDC and AEQ kernels
        # (no Fermat-domain arithmetic), bit-identical outputs.  Kernels are compared
        # in the staged schedule (every CDC, then the AEQ; no lead), which the lead
        # was not tuned for but which treats both paths alike
        progress("batched: direct time-domain comparator")
        ref_out = {i: entries[i][1].clone() for i in pick}
        ref_taps = {i: taps_all[i].clone() for i in pick}
        plan.set_lead(0)

        def staged_runs():
            ts = []
            for k in range(2):
                taps_all.copy_(w_all)
                ts.append(plan.run_timed(stream))
            torch.cuda.synchronize()
            fnt.fnt_check()
            for i in pick:
                if not (torch.equal(entries[i][1], ref_out[i]) and torch.equal(taps_all[i], ref_taps[i])):
                    raise SystemExit(f"staged run differs on channel {i}")
            return tuple(float(np.mean([t[k] for t in ts])) for k in ("cdc_ms", "aeq_ms", "step_ms"))

        f_cdc, f_aeq, f_step = staged_runs()
        plan.set_cdc_variant(1)
        plan.set_aeq_variant(1)
        d_cdc, d_aeq, d_step = staged_runs()
        plan.set_cdc_variant(0)
        # the RDE gradient through dot products and in the Fermat domain, on the
        # one-wave-per-channel AEQ kernel (variants 2 and 3)
        progress("batched: Fermat-domain gradient comparator")
        plan.set_aeq_variant(2)
        _, g_dot, _ = staged_runs()
        plan.set_aeq_variant(3)
        _, g_fnt, _ = staged_runs()
        plan.set_aeq_variant(0)
        # the fused persistent schedule (one launch, hipGraph), whether or not the tuner chose it
        progress("batched: fused persistent schedule")
        fused = {}
        for prio in (0, 512):
            plan.set_fused(4, prio)
            ts = []
            for k in range(3):
                taps_all.copy_(w_all)
                ts.append(plan.run_timed(stream))
            torch.cuda.synchronize()
            fnt.fnt_check()
            for i in pick:
                if not (torch.equal(entries[i][1], ref_out[i]) and torch.equal(taps_all[i], ref_taps[i])):
                    raise SystemExit(f"fused run differs on channel {i}")
            fms = float(np.median([t["aeq_ms"] for t in ts]))
            if not fused or fms < fused["ms"]:
                fused = {"ms": round(fms, 3), "value": round(inst / (fms / 1e3) / 1e9, 4), "unit": "Gsamples/s",
                         "prio_channels": prio, "grid": plan.info()["fused_grid"],
                         "kernel": "cdc_aeq_fused_kernel<4, 1, 2>"}
        taps_all.copy_(w_all)
        plan.run(stream)                    # the first replay of the fused graph uploads it
        torch.cuda.synchronize()
        fused["graph_ms"] = round(_time_events(torch, plan.run, 3, stream), 3)
        plan.set_fused(0)
    # back to the tuned (or given) schedule
    apply_schedule(plan, info)
    value = inst / (ms / 1e3) / 1e9
    aeq_blocks = times[0]["aeq_blocks"]           # the AEQ launch on the launch stream
    lead_blocks = times[0]["aeq_lead_blocks"]
    top_blocks = times[0]["aeq_top_blocks"]
    cdc_blocks = sum((e[0].shape[0] + 31) // 32 for e in entries)
    aeq_ops = AEQ_OPS_PER_BLOCK * aeq_blocks
    all_aeq_ops = AEQ_OPS_PER_BLOCK * (aeq_blocks + lead_blocks + top_blocks)
    cdc_ops = CDC_OPS_PER_BLOCK * cdc_blocks
    achieved = aeq_ops / (aeq_ms / 1e3) / 1e9
    kname = aeq_kernel_name(info)
    fused_top = bool(info["top_channels"]) and split_fusable(info["top_form"], info["lead_form"])
    lead_name = None
    if info["lead_channels"]:
        lead_name = (split_name(info["top_form"], info["lead_form"]) if fused_top
                     else AEQ_FORM_KERNEL[info["lead_form"]])
    top_name = AEQ_FORM_KERNEL[info["top_form"]] if info["top_channels"] and not fused_top else None
    # the dominant kernel: the AEQ launch with the most algorithmic work (with a
    # lead, a launch on one of the plan's side streams can be the largest)
    if times[0]["fused"]:
        kname = "cdc_aeq_fused_kernel<%d, %d, %d>" % (info["fused_lpt"], info["fused_lpt"] // 4,
                                                       1 if info["fused_split"] else 2)
    launches = [(aeq_blocks, kname, aeq_ms, kname, "launch stream")]
    if lead_name:
        launches.append((lead_blocks, lead_name, lead_ms, lead_name + " (lead)", "lead channels, plan side stream"))
    if top_name:
        launches.append((top_blocks, top_name, top_ms, top_name + " (first level)",
                         "first lead level, plan third stream"))
    dom_blocks, dom_name, dom_ms, dom_key, dom_where = max(launches, key=lambda x: x[0])
    if times[0]["fused"]:
        # the fused launch does every channel's CDC and AEQ: 8 B per instant of HBM
        dom_ops = AEQ_OPS_PER_BLOCK * dom_blocks + CDC_OPS_PER_BLOCK * cdc_blocks
        dom_bytes = inst * FUSED_BYTES_PER_INSTANT
    else:
        dom_ops = AEQ_OPS_PER_BLOCK * dom_blocks
        dom_bytes = dom_blocks * 16 * AEQ_BYTES_PER_SYMBOL
    dom_achieved = dom_ops / (dom_ms / 1e3) / 1e9
    dom_traffic, traffic_basis = load_traffic(dom_key, "batched", dom_blocks, per_block=True)
    roof = {"kernel": dom_name, "bound": "alu", "achieved": round(dom_achieved, 1), "peak": PEAK_ALU_GOPS,
            "unit": "Gops/s", "frac": round(dom_achieved / PEAK_ALU_GOPS, 5),
            "traffic": dom_traffic, "traffic_basis": traffic_basis,
            "algorithmic_ops_per_launch": dom_ops,
            "ops_per_unit": {"aeq_block_16_symbols": AEQ_OPS_PER_BLOCK, "cdc_block_32_instants": CDC_OPS_PER_BLOCK},
            "launch": dom_where,
            "hbm_algorithmic_gbs": round(dom_bytes / dom_ms / 1e6, 1),
            "hbm_frac": round(dom_bytes / dom_ms / 1e6 / PEAK_HBM_GBS, 5)}
    kernels = {
        "aeq": {"kernel": kname, "ms": round(aeq_ms, 3), "gops": round(achieved, 1), "blocks": aeq_blocks,
                "us_per_block_per_channel_longest":
                    round(max(aeq_ms, lead_ms) * 1e3 / max(info["aeq_blocks_max"], 1), 4)},
    }
    if not times[0]["fused"]:                      # a CDC launch of its own (not the fused schedule)
        kernels["cdc"] = {
            "kernel": ("cdc_lane_kernel<%d>" % info["cdc_waves_per_group"]) if info["cdc_blocks_per_wave"] == 0
                      else "cdc_kernel<false>", "ms": round(cdc_ms, 3),
            "gops": round(cdc_ops / cdc_ms / 1e6, 1), "frac_alu": round(cdc_ops / cdc_ms / 1e6 / PEAK_ALU_GOPS, 5),
            "gbs": round(inst * CDC_BYTES_PER_INSTANT / cdc_ms / 1e6, 1)}
    if info["lead_channels"]:
        kernels["aeq_lead"] = {
            "kernel": lead_name, "channels": info["lead_channels"] - (info["top_channels"] if top_name else 0),
            "ms": round(lead_ms, 3), "blocks": lead_blocks,
            "gops": round(AEQ_OPS_PER_BLOCK * lead_blocks / lead_ms / 1e6, 1),
            "what": "the longest channels' AEQ, started after their own CDC on a second stream, "
                    "concurrent with the other channels' CDC and AEQ"}
    if top_name:
        kernels["aeq_top"] = {
            "kernel": top_name, "channels": info["top_channels"],
            "ms": round(top_ms, 3), "blocks": top_blocks,
            "gops": round(AEQ_OPS_PER_BLOCK * top_blocks / top_ms / 1e6, 1),
            "what": "the first lead level: the very longest channels, CDC first of all, AEQ on a third stream"}
    res = {
        "metric": METRIC,
        "value": round(value, 4), "unit": "Gsamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"batched FNT-CDC+AEQ, {len(chans)} channels, log-uniform "
                               f"2^{args.log2_min}..2^{args.log2_max} symbols/pol, fibre U(10,80) km, "
                               f"8-32 taps, OSNR U(18,26) dB, N=64 FNT mod 65537 alpha=sqrt2, AEQ N=32",
                   "channels": len(chans), "instants": inst, "longest_aeq_chain_blocks": info["aeq_blocks_max"]},
        "roofline": roof,
        "kernels": kernels,
        "plan_run_ms": round(run_ms, 3),
        "graph_replay_ms": round(graph_ms, 3),
        "event_ms_per_step": round(event_step_ms, 3),
        "event_ms_per_step_median": round(event_step_med, 3),
        "roofline_whole_path": {"bound": "alu", "achieved": round((all_aeq_ops + cdc_ops) / (ms / 1e3) / 1e9, 1),
                                "peak": PEAK_ALU_GOPS, "unit": "Gops/s",
                                "frac": round((all_aeq_ops + cdc_ops) / (ms / 1e3) / 1e9 / PEAK_ALU_GOPS, 5)},
        "plan": {k: info[k] for k in ("cdc_waves_per_group", "cdc_blocks_per_wave", "aeq_variant",
                                      "aeq_waves_per_pol", "aeq_waves_long", "aeq_long_channels",
                                      "lead_channels", "lead_form", "top_channels", "top_form", "graph",
                                      "tune_run_ms", "fused_lpt", "fused_split", "fused_prio_channels")},
        "parity": f"bit-exact vs oracle on channels {pick}", "gen_s": round(gen_s, 1),
        "autotune_s": round(tune_s, 1),
        "launches": launches_of(info, times[0], kname, lead_name, top_name, aeq_blocks, lead_blocks, top_blocks,
                                [e[0].shape[0] for e in entries]),
    }
    if plain_gsps is not None:
        res["vs_plain"] = round(value / plain_gsps, 2)
        res["plain_loop"] = {"value": round(plain_gsps, 5), "unit": "Gsamples/s",
                             "sample": f"{len(sample)} random channels, fnt_cdc then fnt_aeq, one channel after "
                                       f"another"}
        res["fused_schedule"] = fused
        res["direct_comparator"] = {
            "value": round(inst / (d_step / 1e3) / 1e9, 4), "unit": "Gsamples/s",
            "cdc_ms": round(d_cdc, 3), "aeq_ms": round(d_aeq, 3), "step_ms": round(d_step, 3),
            "fermat_staged": {"value": round(inst / (f_step / 1e3) / 1e9, 4), "cdc_ms": round(f_cdc, 3),
                              "aeq_ms": round(f_aeq, 3), "step_ms": round(f_step, 3)},
            "what": "same plan in the staged schedule (all CDC, then the AEQ; no lead), time-domain CDC "
                    "(int8 dot products over the 32-instant window) and time-domain AEQ, no Fermat-domain "
                    "arithmetic, against the Fermat-domain kernels in the same schedule; bit-identical on "
                    "the parity channels"}
        res["fermat_gradient"] = {
            "aeq_ms_dot_gradient": round(g_dot, 3), "aeq_ms_fermat_gradient": round(g_fnt, 3),
            "kernel": "aeq_fnt_kernel<false> / aeq_fnt_kernel<true>",
            "what": "AEQ variants 2 and 3 (one wave per channel, staged schedule): the RDE gradient of the "
                    "block update by 4-byte dot products, or through FNT32 products in the Fermat domain "
                    "(4 error transforms, 512 products, 16 inverse transforms per block); bit-identical"}
    if not args.no_cpu_baseline:
        progress("batched: oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline_batched(chans, prms, args.cpu_budget)
    plan.close()
    return res


def bench_transforms(args, torch, dev):
    """fnt_forward / fnt_inverse throughput for every supported (t, N, alpha):
    2^26 residues per call (uint32 in, uint32 out, 512 MiB moved), HBM-bound by construction."""
    from paper_2405_04253_amd import fnt
    stream = torch.cuda.current_stream()
    out = []
    for t, log2n, kind, name in [(2, 3, fnt.FNT_ALPHA_2, "2"), (2, 4, fnt.FNT_ALPHA_SQRT2, "sqrt2"),
                                 (3, 4, fnt.FNT_ALPHA_2, "2"), (3, 5, fnt.FNT_ALPHA_SQRT2, "sqrt2"),
                                 (4, 5, fnt.FNT_ALPHA_2, "2"), (4, 6, fnt.FNT_ALPHA_SQRT2, "sqrt2")]:
        F = (1 << (1 << t)) + 1
        n = 1 << 26
        x = torch.randint(0, F, (n >> log2n, 1 << log2n), dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        for _ in range(2):
            fnt.fnt_forward(x, t, log2n, kind, out=y, stream=stream)
        fwd = _time_events(torch, lambda: fnt.fnt_forward(x, t, log2n, kind, out=y, stream=stream), 5, stream)
        inv = _time_events(torch, lambda: fnt.fnt_inverse(y, t, log2n, kind, out=x, stream=stream), 5, stream)
        fnt.fnt_check()
        gbs = 8 * n / (fwd / 1e3) / 1e9
        out.append({"t": t, "F": F, "N": 1 << log2n, "alpha": name, "forward_ms": round(fwd, 4),
                    "inverse_ms": round(inv, 4), "forward_gbs": round(gbs, 1),
                    "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)})
    return out


def measured_peaks(torch, dev):
    """Measured ceilings beside the published ones: the 32-bit integer VALU rate
    (a loop of independent v_add_u32 over 4096 workgroups) and the HBM copy
    bandwidth (16-byte grid-stride copy of 1 GiB), from libfntprobe.so."""
    import ctypes
    path = os.path.join(ROOT, "paper_2405_04253_amd", "libfntprobe.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    blocks, trips = 4096, 1024
    sink = torch.empty(blocks * 256, dtype=torch.int32, device=dev)
    ops, ops_base = ctypes.c_double(0), ctypes.c_double(0)
    rc = lib.fntprobe_alu(0, ctypes.c_void_p(sink.data_ptr()), blocks, trips, ctypes.byref(ops), sp)
    rc1 = lib.fntprobe_alu(1, ctypes.c_void_p(sink.data_ptr()), blocks, trips, ctypes.byref(ops_base), sp)
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    bw = ctypes.c_double(0)
    rc2 = lib.fntprobe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                            ctypes.c_size_t(nbytes), ctypes.byref(bw), sp)
    torch.cuda.synchronize()
    del src, dst, sink
    return {"alu_gops": round(ops.value / 1e9, 1) if rc == 0 else None,
            "alu_base_rate_gops": round(ops_base.value / 1e9, 1) if rc1 == 0 else None,
            "alu_peak": PEAK_ALU_GOPS,
            "copy_gbs": round(bw.value / 1e9, 1) if rc2 == 0 else None, "hbm_peak_published": PEAK_HBM_GBS,
            "what": "16 independent chains of v_add_u32 (fastest 32-bit form) and of SDWA v_sub_u32 (the "
                    "Fermat fold; base rate, like shifts and 24-bit multiplies) on every SIMD; 16-byte "
                    "grid-stride copy of 1 GiB (read + write bytes)"}


def bench_served(args, torch, dev, host: bool = False):
    """Poisson arrivals of stream segments into a session; p50/p99 latency.
    host=True: the payloads and outputs live in pinned host memory and every
    request is staged through the session's HBM pool (host-to-device and back
    inside the measured latency), over a shorter window."""
    import oracle as O
    from paper_2405_04253_amd import fnt, synth
    rng = np.random.default_rng(12345)
    nch = args.served_channels
    window = args.h2d_window if host else args.window
    # arrivals over the window, each to a uniformly random channel
    times, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / args.rate)
        if t > window:
            break
        times.append(t)
    seg_sym = [16 * max(1, int(2 ** rng.uniform(13, 18)) // 16) for _ in times]
    owner = rng.integers(0, nch, size=len(times))
    per_ch = [[] for _ in range(nch)]
    for i, c in enumerate(owner):
        per_ch[c].append(i)
    t0 = time.perf_counter()
    streams, params = {}, {}
    sess = fnt.Session(max_channels=nch, hbm_budget_bytes=1 << 30, chunk_blocks=args.chunk,
                       max_active=nch, aeq_form=args.served_form)
    progress(f"served: {len(times)} requests over {nch} channels; generating streams")
    for c in range(nch):
        if c % 128 == 0:
            torch.cuda.synchronize()
            progress(f"served: generated {c}/{nch} channel streams ({time.perf_counter() - t0:.1f} s)")
        nsym = sum(seg_sym[i] for i in per_ch[c])
        r = np.random.default_rng(synth.seed_for(0, "served", c))
        km, osnr = float(r.uniform(10, 80)), float(r.uniform(18, 26))
        q, taps, sh, unit = synth.gen_channel_torch(max(nsym, 16), km, osnr, synth.seed_for(1, "served", c), dev)
        streams[c] = q
        prm = dict(synth.AEQ_DEFAULTS, const_unit=unit)
        params[c] = (taps, sh, prm)
        sess.add_channel(c, fnt.cdc_params(taps, sh), fnt.aeq_params(**prm))
    if host:
        streams = {c: q.cpu().pin_memory() for c, q in streams.items()}
        outs = {c: torch.zeros((streams[c].shape[0] // 2, 4), dtype=torch.int16).pin_memory() for c in range(nch)}
    else:
        outs = {c: torch.zeros((streams[c].shape[0] // 2, 4), dtype=torch.int16, device=dev) for c in range(nch)}
    reqs, offs = [], [0] * nch
    for i in range(len(times)):
        c = int(owner[i])
        n = 2 * seg_sym[i]
        o = offs[c]
        reqs.append((c, streams[c][o:o + n], outs[c][o // 2:(o + n) // 2], int(times[i] * 1e9)))
        offs[c] += n
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    progress(f"served{' (host buffers)' if host else ''}: replaying {len(reqs)} arrivals over {window} s")
    sess.replay(reqs, host=host)
    t_end = time.perf_counter()
    while sess.stats()["completed"] < len(reqs):
        time.sleep(1.0)
        progress(f"served: {sess.stats()['completed']}/{len(reqs)} done "
                 f"({time.perf_counter() - t_end:.1f} s after the last arrival)")
    sess.drain()
    st = sess.stats()
    sess.close()
    fnt.fnt_check()
    # parity: the two busiest channels against the oracle on their concatenated streams
    busiest = sorted(range(nch), key=lambda c: -offs[c])[:2]
    for c in busiest:
        taps, sh, prm = params[c]
        n = offs[c]
        outr, _, _ = O.cdc_aeq(streams[c][:n].cpu().numpy(), taps, sh, synth.centre_spike_taps(), O.params(**prm))
        if not np.array_equal(outs[c][: n // 2].cpu().numpy(), outr):
            raise SystemExit(f"served parity failure on channel {c}")
    inst = sum(2 * x for x in seg_sym)
    what = ("payloads and outputs in pinned host memory, staged through the session's HBM pool "
            "(PCIe both ways inside the latency)" if host else "payloads resident in HBM")
    return {"value": round(st["gsamples_per_s"], 4), "unit": "Gsamples/s", "buffers": what,
            "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
            "mean_us": round(st["mean_us"], 1), "max_us": round(st["max_us"], 1),
            "requests": int(st["completed"]), "ticks": int(st["ticks"]),
            "offered_gsamples_per_s": round(inst / window / 1e9, 3),
            "workload": f"{nch} channels, Poisson {args.rate:.0f} req/s for {window} s, segments "
                        f"log-uniform 2^13..2^18 symbols, chunk {args.chunk} blocks/tick, "
                        f"AEQ form {args.served_form}",
            "parity": f"bit-exact vs oracle on channels {busiest} (whole streams)", "gen_s": round(gen_s, 1)}


def bench_large(args, torch, dev):
    """The large batch at full HBM occupancy: 16384 channels, log-uniform
    2^14..2^22 symbols/pol (about 2^34.5 instants, 99.5 GB in and out), every
    channel from its own seed; one plan with quick autotuning; against the plain
    per-channel loop on a sample; parity on sampled channels (every channel is
    checked in the full-size GPU test)."""
    import oracle as O
    from paper_2405_04253_amd import fnt, synth
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    specs = synth.batched_specs(16384, 14, 22, tag="large")
    _, chans = synth.gen_batch_torch(specs, dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    inst = sum(c[0].shape[0] for c in chans)
    progress(f"large: generated {inst} instants in {gen_s:.1f} s")
    w0 = torch.from_numpy(synth.centre_spike_taps()).to(dev)
    taps_all = w0.unsqueeze(0).repeat(len(chans), 1, 1, 1).contiguous()
    entries, prms = [], []
    for i, (q, taps, sh, unit) in enumerate(chans):
        prm = dict(synth.AEQ_DEFAULTS, const_unit=unit)
        prms.append(prm)
        out = torch.empty((q.shape[0] // 2, 4), dtype=torch.int16, device=dev)
        entries.append((q, out, taps_all[i], fnt.cdc_params(taps, sh), fnt.aeq_params(**prm)))
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    plan = fnt.Plan(entries, autotune=True, use_graph=True, stream=stream, tune_quick=True)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    info = plan.info()
    progress(f"large: plan ready in {tune_s:.1f} s: {info}")
    w_all = w0.unsqueeze(0).expand_as(taps_all)

    def step():
        taps_all.copy_(w_all)
        plan.run(stream)

    step()
    torch.cuda.synchronize()
    fnt.fnt_check()
    steps = max(1, args.large_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    fnt.fnt_check()
    order = sorted(range(len(chans)), key=lambda i: chans[i][0].shape[0])
    pick = sorted(set([order[0], order[len(order) // 2], order[-1]]))
    for i in pick:
        q, taps, sh, unit = chans[i]
        outr, wr, _ = O.cdc_aeq(q.cpu().numpy(), taps, sh, synth.centre_spike_taps(), O.params(**prms[i]))
        if not (np.array_equal(entries[i][1].cpu().numpy(), outr) and np.array_equal(taps_all[i].cpu().numpy(), wr)):
            raise SystemExit(f"large batch parity failure on channel {i}")
    rng = np.random.default_rng(9)
    sample = [int(i) for i in rng.choice(len(chans), size=16, replace=False)]
    s_inst = sum(chans[i][0].shape[0] for i in sample)
    abuf = torch.empty((max(chans[i][0].shape[0] for i in sample) // 2 + 1, 4), dtype=torch.int8, device=dev)
    tmp_taps = w0.clone()

    def plain_loop():
        for i in sample:
            tmp_taps.copy_(w0)
            m = entries[i][1].shape[0]
            fnt.fnt_cdc(chans[i][0], entries[i][3], exact=False, a_out=abuf[:m], stream=stream)
            fnt.fnt_aeq(abuf[:m], tmp_taps, entries[i][4], out=entries[i][1], stream=stream)

    plain_ms = _time_events(torch, plain_loop, 1, stream)
    plain = s_inst / (plain_ms / 1e3) / 1e9
    value = inst / (ms / 1e3) / 1e9
    plan.close()
    return {"value": round(value, 4), "unit": "Gsamples/s", "ms_per_step": round(ms, 3), "steps": steps,
            "workload": "16384 channels, log-uniform 2^14..2^22 symbols/pol, fibre U(10,80) km, OSNR U(18,26) dB, "
                        "every channel from its own seed",
            "instants": inst, "vs_plain": round(value / plain, 2),
            "plain_loop": {"value": round(plain, 5), "unit": "Gsamples/s",
                           "sample": "16 random channels, fnt_cdc then fnt_aeq, one channel after another"},
            "plan": {k: info[k] for k in ("cdc_waves_per_group", "aeq_waves_per_pol", "aeq_waves_long",
                                          "aeq_long_channels", "lead_channels", "lead_form", "graph",
                                          "fused_lpt", "fused_split", "fused_prio_channels")},
            "parity": f"bit-exact vs oracle on channels {pick}", "gen_s": round(gen_s, 1),
            "autotune_s": round(tune_s, 1)}


def bench_served_capacity(args, torch, dev):
    """The session's throughput ceiling: the served workload (1024 channels,
    segments log-uniform 2^13..2^18 symbols) replayed at rising Poisson rates, a
    fresh session per rate on the same channel streams, until the delivered rate
    falls below 90% of the offered one or p99 exceeds 10x the first point's."""
    from paper_2405_04253_amd import fnt, synth
    nch = args.served_channels
    window = args.sweep_window
    rates = [float(r) for r in args.sweep_rates.split(",")]
    plans = []
    for k, rate in enumerate(rates):
        rng = np.random.default_rng(777 + k)
        times, t = [], 0.0
        while True:
            t += rng.exponential(1.0 / rate)
            if t > window:
                break
            times.append(t)
        seg = [16 * max(1, int(2 ** rng.uniform(13, 18)) // 16) for _ in times]
        owner = rng.integers(0, nch, size=len(times))
        plans.append((rate, times, seg, owner))
    need = np.zeros(nch, np.int64)
    for _, times, seg, owner in plans:
        per = np.zeros(nch, np.int64)
        np.add.at(per, owner, np.array(seg, np.int64))
        need = np.maximum(need, per)
    t0 = time.perf_counter()
    streams, params = {}, {}
    for c in range(nch):
        r = np.random.default_rng(synth.seed_for(0, "served", c))
        km, osnr = float(r.uniform(10, 80)), float(r.uniform(18, 26))
        q, taps, sh, unit = synth.gen_channel_torch(max(int(need[c]), 16), km, osnr,
                                                    synth.seed_for(2, "served", c), dev)
        streams[c] = q
        params[c] = (taps, sh, dict(synth.AEQ_DEFAULTS, const_unit=unit))
        if c % 256 == 0:
            torch.cuda.synchronize()
            progress(f"served sweep: generated {c}/{nch} streams ({time.perf_counter() - t0:.1f} s)")
    outs = {c: torch.zeros((streams[c].shape[0] // 2, 4), dtype=torch.int16, device=dev) for c in range(nch)}
    torch.cuda.synchronize()
    points = []
    for rate, times, seg, owner in plans:
        sess = fnt.Session(max_channels=nch, hbm_budget_bytes=1 << 30, chunk_blocks=args.chunk,
                           max_active=nch, aeq_form=args.served_form)
        for c in range(nch):
            taps, sh, prm = params[c]
            sess.add_channel(c, fnt.cdc_params(taps, sh), fnt.aeq_params(**prm))
        reqs, offs = [], [0] * nch
        for i in range(len(times)):
            c = int(owner[i])
            n = 2 * seg[i]
            o = offs[c]
            reqs.append((c, streams[c][o:o + n], outs[c][o // 2:(o + n) // 2], int(times[i] * 1e9)))
            offs[c] += n
        progress(f"served sweep: {rate:.0f} req/s, {len(reqs)} requests over {window} s")
        sess.replay(reqs)
        t_end = time.perf_counter()
        while sess.stats()["completed"] < len(reqs):
            time.sleep(0.5)
            progress(f"served sweep: {sess.stats()['completed']}/{len(reqs)} done "
                     f"({time.perf_counter() - t_end:.1f} s after the last arrival)")
        sess.drain()
        st = sess.stats()
        sess.close()
        fnt.fnt_check()
        offered = 2 * sum(seg) / window / 1e9
        pt = {"rate_req_s": rate, "offered_gsamples_per_s": round(offered, 3),
              "delivered_gsamples_per_s": round(st["gsamples_per_s"], 3), "p50_us": round(st["p50_us"], 1),
              "p99_us": round(st["p99_us"], 1), "requests": int(st["completed"]), "ticks": int(st["ticks"])}
        points.append(pt)
        progress(f"served sweep: {pt}")
        if st["gsamples_per_s"] < 0.9 * offered or st["p99_us"] > 10 * points[0]["p99_us"]:
            break
    sustained = [p for p in points if p["delivered_gsamples_per_s"] >= 0.9 * p["offered_gsamples_per_s"]
                 and p["p99_us"] <= 10 * points[0]["p99_us"]]
    return {"points": points, "unit": "Gsamples/s",
            "capacity_gsamples_per_s": max((p["delivered_gsamples_per_s"] for p in sustained), default=None),
            "saturated_delivered_gsamples_per_s": points[-1]["delivered_gsamples_per_s"],
            "workload": f"{nch} channels, segments log-uniform 2^13..2^18 symbols, chunk {args.chunk} blocks/tick, "
                        f"{window} s of Poisson arrivals per rate, rates {args.sweep_rates} req/s until the "
                        f"delivered rate drops below 90% of the offered one or p99 exceeds 10x the first point's",
            "gen_s": round(time.perf_counter() - t0, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2-symbols", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--single-cpu-baseline", action="store_true",
                    help="also time the single-threaded oracle on a prefix of the single stream")
    ap.add_argument("--single-steps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-served", action="store_true")
    ap.add_argument("--skip-single", action="store_true")
    ap.add_argument("--skip-transforms", action="store_true")
    ap.add_argument("--skip-cdc-long", action="store_true")
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--large-steps", type=int, default=3)
    ap.add_argument("--nch", type=int, default=4096)
    ap.add_argument("--log2-min", type=int, default=12)
    ap.add_argument("--log2-max", type=int, default=20)
    ap.add_argument("--served-channels", type=int, default=1024)
    ap.add_argument("--rate", type=float, default=20000.0)
    ap.add_argument("--window", type=float, default=1.0)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--h2d-window", type=float, default=0.25,
                    help="arrival window of the served leg with host buffers (0: skip it)")
    ap.add_argument("--sweep-rates", default="20000,40000,80000,120000,160000,240000",
                    help="Poisson rates (req/s) of the served capacity sweep")
    ap.add_argument("--sweep-window", type=float, default=0.25)
    ap.add_argument("--skip-sweep", action="store_true")
    ap.add_argument("--served-form", type=int, default=-1,
                    help="AEQ form of the session ticks (0, 3, 1, 2, 4; -1: automatic)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines file for the plan autotuner: reuse a schedule stored there for the same "
                         "workload, else tune and append it (keeps profiled runs on one schedule)")
    ap.add_argument("--schedule", default=None,
                    help="JSON object of plan schedule keys (as in the bench line's 'plan'): use this schedule "
                         "instead of autotuning, e.g. for a profile of a fixed schedule")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="batched leg: skip the plain per-channel loop, the direct comparator and the fused "
                         "schedule comparison (profiles of one schedule)")
    ap.add_argument("--launches-out", default=None,
                    help="write the timed legs' launches (kernel, counter key, blocks) to this JSON file")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run 5 plain 256 MiB elementwise copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "channels would shard across GPUs with no exchange, which is not built here.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_probe:
        x = torch.randint(-16, 16, (256 << 20,), dtype=torch.int8, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(5):
            torch.neg(x, out=y)             # a plain elementwise kernel: reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel(), "copies": 5}), flush=True)
        return
    res = {}
    if not args.skip_batched:
        progress("batched")
        res = bench_batched(args, torch, dev)
        progress(f"batched done: {res['value']}")
        peaks = measured_peaks(torch, dev)
        if peaks:
            res["measured_peaks"] = peaks
            if peaks["alu_gops"]:
                res["roofline"]["measured_fast_gops"] = peaks["alu_gops"]
                res["roofline"]["frac_of_measured_fast"] = round(res["roofline"]["achieved"] / peaks["alu_gops"], 5)
            if peaks["alu_base_rate_gops"]:
                res["roofline"]["measured_base_gops"] = peaks["alu_base_rate_gops"]
                res["roofline"]["frac_of_measured_base"] = round(
                    res["roofline"]["achieved"] / peaks["alu_base_rate_gops"], 5)
            progress(f"measured peaks: {peaks}")
    if not args.skip_large:
        progress("large batch")
        res["large_batch"] = bench_large(args, torch, dev)
        progress(f"large batch done: {res['large_batch']['value']}")
    if not args.skip_single:
        progress("plain single stream")
        res["plain_single_stream"] = bench_single(args, torch, dev)
        progress(f"single done: {res['plain_single_stream']['value']}")
        if "value" in res:
            res["vs_single_stream"] = round(res["value"] / res["plain_single_stream"]["value"], 1)
    if not args.skip_cdc_long:
        progress("cdc long")
        res["cdc_long"] = bench_cdc_long(args, torch, dev)
        progress(f"cdc long done: {res['cdc_long']['value']}")
    if not args.skip_transforms:
        progress("transforms")
        res["transforms"] = bench_transforms(args, torch, dev)
    if not args.skip_served:
        progress("served")
        res["served"] = bench_served(args, torch, dev)
        progress(f"served done: {res['served']['value']}")
        if args.h2d_window > 0:
            progress("served with host buffers")
            res["served_h2d"] = bench_served(args, torch, dev, host=True)
            progress(f"served with host buffers done: {res['served_h2d']['value']}")
        if not args.skip_sweep:
            progress("served capacity sweep")
            res["served_capacity"] = bench_served_capacity(args, torch, dev)
            progress(f"served capacity sweep done: {res['served_capacity']['capacity_gsamples_per_s']}")
    if args.launches_out:
        with open(args.launches_out, "w") as f:
            json.dump({"batched": res.get("launches", []),
                       "single": res.get("plain_single_stream", {}).get("launches", [])}, f, indent=1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
