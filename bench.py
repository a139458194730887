#!/usr/bin/env python3
"""Throughput of the FNT-CDC + FNT-AEQ receiver path on one MI355X.

Default workload ("single"): one channel, 2^24 PDM-16QAM symbols per
polarisation at 2 samples/symbol (2^25 instants), 75 km SSMF, 5-bit samples,
32 six-bit CD-inverse taps, N = 64 FNT mod 65537 with alpha = sqrt 2, then the
N = 32 FNT-AEQ with the RDE update.  A step is one pass of the whole path over
the stream (CDC + resample/requantise + AEQ), inputs resident in HBM.

Other workloads: "batched" (many channels of log-uniform length in one plan,
hipGraph replay) and "served" (Poisson arrivals into a session; p50/p99).

Prints one JSON line.  Gsamples/s counts instants (one dual-polarisation
2-samples/symbol sample = 4 int8).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
PEAK_ALU_GOPS = 256 * 4 * 16 * 2.4   # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39321.6 G int32 ops/s

# Algorithmic integer operations of the method, per unit:
# a radix-2 butterfly = 3 ops (add, sub, twiddle), a Z_F product or MAC = 2 ops, etc.
FNT32_OPS = 80 * 3
FNT64_OPS = 192 * 3
# CDC, per block of 32 new instants (both polarisations)
CDC_OPS_PER_BLOCK = (2 * 2 * 64            # residue packing u, v
                     + 4 * FNT64_OPS       # forward transforms
                     + 2 * (128 + 128)     # products and P +- Q
                     + 4 * FNT64_OPS       # inverse transforms
                     + 2 * 2 * 32 * 2      # Eq. (7)/(8) scale and lift of the kept outputs
                     + 16 * 4 * 2)         # requantise the 16 kept symbols
# AEQ, per block of 16 symbols (= 32 instants)
AEQ_OPS_PER_BLOCK = (4 * FNT32_OPS         # input spectra
                     + 256 * 2 * 2         # digit split
                     + 32 * FNT32_OPS      # tap-digit spectra
                     + 1024 + 512          # products and pair sums
                     + 16 * FNT32_OPS      # inverse transforms
                     + 16 * 4 * 8          # lift + recombine
                     + 64 * 2              # output rounding
                     + 16 * 2 * 12         # RDE error terms
                     + 4096 * 2            # gradient MACs
                     + 256 * 3)            # tap update
CDC_BYTES_PER_INSTANT = 4 + 2              # int8[4] in, int8[4] per symbol out
AEQ_BYTES_PER_SYMBOL = 4 + 8               # int8[4] in, int16[4] out


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("fnt_kernels.hip", "fnt_device.hpp"):
        with open(os.path.join(ROOT, "paper_2405_04253_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(p))
    except Exception:
        return None
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fnt.fnt_check()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fnt.fnt_check()
    cdc_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    aeq_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms = wall / args.steps * 1e3
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
    roof = {"kernel": "aeq_fnt_kernel", "bound": "alu", "achieved": round(achieved, 3),
            "peak": PEAK_ALU_GOPS, "unit": "Gops/s", "frac": round(achieved / PEAK_ALU_GOPS, 6),
            "traffic": load_traffic("aeq_fnt_kernel", "single"),
            "algorithmic_ops_per_launch": aeq_ops}
    res = {
        "metric": "bit-exact Gsamples/s, batched/served vs plain FNT-CDC+AEQ; p50/p99 latency",
        "value": round(n / (ms / 1e3) / 1e9, 6), "unit": "Gsamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "single-stream plain FNT-CDC+AEQ, 1 channel x 2^%d symbols/pol, "
                               "75 km, 32 taps, N=64 FNT mod 65537 alpha=sqrt2, AEQ N=32" % args.log2_symbols,
                   "instants": n, "symbols": M, "aeq_variant": "fnt"},
        "roofline": roof,
        "kernels": kernels,
        "gen_s": round(gen_s, 1),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_single(ch, prm, args.cpu_budget)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="single", choices=["single"])
    ap.add_argument("--log2-symbols", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
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
    res = bench_single(args, torch, dev)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
