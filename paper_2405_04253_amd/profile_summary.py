"""Summaries of rocprofv3 runs of the benchmark, for profiles/.

Reads the CSV files rocprofv3 writes (``--kernel-trace --stats -f csv`` and
``--pmc ... -f csv``) under the given output directories and writes

* a markdown table per workload (kernel durations from the trace, HBM bytes
  from FETCH_SIZE / WRITE_SIZE scaled by a plain copy kernel's readings, SQ
  instruction counters), with the commands that produced the inputs;
* the entries of profiles/traffic.json that bench.py reads for its roofline
  ``traffic`` (bytes per launch of a kernel, tied to the device code's hash).

Only the dispatches with a kernel's largest grid are used: those are the plan's
full launches (autotuning and parity runs may launch the same kernel on fewer
channels).

Usage (from the repository root, after the rocprofv3 runs of
``bench.py ... --launches-out L.json``, which lists each timed launch with its
algorithmic work and bytes)::

    python -m paper_2405_04253_amd.profile_summary --workload batched \\
        --launches L.json --trace OUT/p_trace --fetch OUT/p_fetch --write OUT/p_write \\
        --calib-fetch OUT/p_cfetch --calib-write OUT/p_cwrite --sq OUT/p_sq \\
        --cmd "rocprofv3 ..." --md profiles/batched4096_fused.md --traffic profiles/traffic.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def short_name(full: str) -> str:
    """'void (anonymous namespace)::aeq_pol_kernel<4, 1>(fnti::AeqItem const*, ...)' -> 'aeq_pol_kernel<4, 1>'."""
    s = re.sub(r"^void\s+", "", full.strip())
    s = s.replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in s:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _rows(dirs, suffix):
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True):
            with open(path, newline="") as f:
                yield from csv.DictReader(f)


def _grid(row) -> int:
    for k in ("Grid_Size", "Grid_Size_X"):
        if k in row and row[k] not in (None, ""):
            g = int(float(row[k]))
            if k == "Grid_Size_X":
                g *= int(float(row.get("Grid_Size_Y", 1) or 1)) * int(float(row.get("Grid_Size_Z", 1) or 1))
            return g
    return 0


def trace_durations(dirs):
    """{kernel: {grid: [duration ms, ...]}} from kernel_trace.csv."""
    out = {}
    for r in _rows(dirs, "kernel_trace.csv"):
        name = short_name(r.get("Kernel_Name", ""))
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        out.setdefault(name, {}).setdefault(_grid(r), []).append(dt)
    return out


def counters(dirs):
    """{kernel: {grid: {counter: [value per dispatch, ...]}}} from counter_collection.csv
    (values of one counter in one dispatch summed over the rows that split it)."""
    per = {}
    for r in _rows(dirs, "counter_collection.csv"):
        name = short_name(r.get("Kernel_Name", ""))
        key = (name, _grid(r), r.get("Dispatch_Id", ""), r["Counter_Name"])
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, grid, _, cname), v in per.items():
        out.setdefault(name, {}).setdefault(grid, {}).setdefault(cname, []).append(v)
    return out


def _largest(d):
    g = max(d)
    return g, d[g]


def _mean(v):
    return sum(v) / len(v) if v else 0.0


def calibration(fetch_dirs, write_dirs, nbytes):
    """Scale factors so that FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the
    plain copy kernel (reads and writes nbytes) read as nbytes."""
    def one(dirs, cname):
        best = None
        for name, grids in counters(dirs).items():
            g, cs = _largest(grids)
            if cname in cs and (best is None or _mean(cs[cname]) > best[1]):
                best = (name, _mean(cs[cname]))
        return best
    f, w = one(fetch_dirs, "FETCH_SIZE"), one(write_dirs, "WRITE_SIZE")
    return {"kernel": f[0], "copy_bytes": nbytes, "fetch_kib": f[1], "write_kib": w[1],
            "fetch_scale": nbytes / (f[1] * 1024.0), "write_scale": nbytes / (w[1] * 1024.0)}


def stats_table(path, include=r"aeq_|cdc_"):
    """Rows of rocprofv3's --stats kernel_stats.csv for the kernels matching
    `include`, with short names, as markdown."""
    lines = ["| kernel | calls | average ms | min ms | max ms | total ms |", "|---|---|---|---|---|---|"]
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = short_name(r["Name"])
            if not re.search(include, name):
                continue
            lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                         f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | "
                         f"{float(r['TotalDurationNs']) / 1e6:.1f} |")
    return lines


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--append-stats", default=None,
                    help="only append the --stats table of this kernel_stats.csv to --md, then exit")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--title", default=None)
    ap.add_argument("--trace", action="append", default=[])
    ap.add_argument("--fetch", action="append", default=[])
    ap.add_argument("--write", action="append", default=[])
    ap.add_argument("--calib-fetch", action="append", default=[])
    ap.add_argument("--calib-write", action="append", default=[])
    ap.add_argument("--calib-bytes", type=int, default=256 << 20,
                    help="bytes the copy kernel reads (and writes) per dispatch")
    ap.add_argument("--sq", action="append", default=[])
    ap.add_argument("--kernel", action="append", default=[],
                    help="'<kernel short name>=<key>[:<aeq blocks per launch>]'; key names the entry")
    ap.add_argument("--launches", default=None,
                    help="JSON written by bench.py --launches-out; its entries for --leg (default: the workload) "
                         "name the kernels, with their algorithmic work and bytes")
    ap.add_argument("--leg", default=None)
    ap.add_argument("--cmd", action="append", default=[], help="a command that produced the inputs")
    ap.add_argument("--note", action="append", default=[], help="a line of text for the summary")
    ap.add_argument("--md", required=True)
    ap.add_argument("--traffic", default=None)
    a = ap.parse_args(argv)
    if a.append_stats:
        with open(a.md, "a") as f:
            f.write("\n".join(["", "## `--kernel-trace --stats` summary of the trace run (kernels of the path)", ""]
                              + stats_table(a.append_stats)) + "\n")
        print(f"appended {a.append_stats} to {a.md}")
        return
    if not a.workload:
        ap.error("--workload is required")

    sys.path.insert(0, ROOT)
    import bench  # the device-code hash the bench compares against

    trace = trace_durations(a.trace)
    fetch, write = counters(a.fetch), counters(a.write)
    sq = {}
    for d in a.sq:
        for name, grids in counters([d]).items():
            for g, cs in grids.items():
                sq.setdefault(name, {}).setdefault(g, {}).update(cs)
    cal = calibration(a.calib_fetch, a.calib_write, a.calib_bytes) if a.calib_fetch and a.calib_write else None
    wanted, alg, grids = [], {}, {}
    for spec in a.kernel:
        name, rest = spec.split("=", 1)
        key, _, blocks = rest.partition(":")
        wanted.append((name.strip(), key.strip(), int(blocks) if blocks else None))
    if a.launches:
        for e in json.load(open(a.launches)).get(a.leg or a.workload, []):
            wanted.append((e["kernel"], e["key"], e.get("aeq_blocks") or None))
            alg[e["key"]] = e
            if e.get("grid"):
                grids[e["key"]] = int(e["grid"])

    lines = [f"# {a.title or a.workload}: rocprofv3 summary", ""]
    lines += a.note + ([""] if a.note else [])
    lines += ["Commands (repository root, MI355X, `cd /tmp && export TMPDIR=/tmp` first in the script):", ""]
    for c in a.cmd:
        lines += ["```", c, "```"]
    lines += ["", "## Kernel durations (`--kernel-trace`), the plan's full launches", "",
              "| kernel | grid (threads) | dispatches | average ms |", "|---|---|---|---|"]
    entries = {}
    for name, key, blocks in wanted:
        if name not in trace:
            lines.append(f"| `{key}` | - | 0 | (not in the trace) |")
            continue
        # the launch's own grid when given (a kernel launched on two segments),
        # else the kernel's largest grid (the plan's full launches)
        g, ds = (grids[key], trace[name][grids[key]]) if grids.get(key) in trace[name] else _largest(trace[name])
        lines.append(f"| `{key}` | {g} | {len(ds)} | {_mean(ds):.3f} |")
        entries[key] = {"grid": g, "dispatches": len(ds), "avg_ms": _mean(ds)}
        if blocks is not None:
            entries[key]["aeq_blocks"] = blocks
    if alg:
        lines += ["", "## Against the roofline: algorithmic work per launch / average duration", "",
                  f"Vector ALU peak {bench.PEAK_ALU_GOPS:.1f} Gops/s (the fp32 vector rate with an FMA as one operation: 256 CUs x 4 SIMDs x 32 lane-ops per cycle x 2.4 GHz); "
                  f"algorithmic ops per unit: {bench.AEQ_OPS_PER_BLOCK} per 16-symbol AEQ block, "
                  f"{bench.CDC_OPS_PER_BLOCK} per 32-instant CDC block (both polarisations).", "",
                  "| kernel | AEQ blocks | CDC blocks | algorithmic ops | Gops/s | frac of peak | algorithmic bytes |",
                  "|---|---|---|---|---|---|---|"]
        for name, key, _ in wanted:
            if key in entries and key in alg:
                e = alg[key]
                g = e["algorithmic_ops"] / entries[key]["avg_ms"] / 1e6
                entries[key].update({"algorithmic_ops": e["algorithmic_ops"],
                                     "algorithmic_bytes": e["algorithmic_bytes"],
                                     "cdc_blocks": e.get("cdc_blocks", 0)})
                lines.append(f"| `{key}` | {e.get('aeq_blocks', 0)} | {e.get('cdc_blocks', 0)} | "
                             f"{e['algorithmic_ops']:.4g} | {g:.1f} | {g / bench.PEAK_ALU_GOPS:.4f} | "
                             f"{e['algorithmic_bytes']:.4g} |")
    if cal:
        lines += ["", "## HBM traffic per launch (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`, separate runs)", "",
                  f"Calibration: `{cal['kernel']}` reads and writes {cal['copy_bytes']} bytes per dispatch; it "
                  f"reads FETCH_SIZE {cal['fetch_kib']:.0f} KiB and WRITE_SIZE {cal['write_kib']:.0f} KiB, so "
                  f"FETCH x {cal['fetch_scale']:.5f} and WRITE x {cal['write_scale']:.5f} (per KiB read: bytes "
                  f"= KiB x 1024 x scale).", "",
                  "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled bytes / launch | algorithmic bytes | "
                  "GB/s at the average duration |",
                  "|---|---|---|---|---|---|"]
        for name, key, _ in wanted:
            if key not in entries or name not in fetch or name not in write:
                continue
            g = entries[key]["grid"]
            fk = _mean(fetch[name].get(g, {}).get("FETCH_SIZE", []))
            wk = _mean(write[name].get(g, {}).get("WRITE_SIZE", []))
            fb, wb = fk * 1024 * cal["fetch_scale"], wk * 1024 * cal["write_scale"]
            entries[key].update({"fetch_kib_raw": fk, "write_kib_raw": wk, "fetch_bytes": fb, "write_bytes": wb,
                                 "bytes_per_launch": fb + wb, "source_hash": bench.kernel_source_hash()})
            ab = alg[key]["algorithmic_bytes"] if key in alg else None
            lines.append(f"| `{key}` | {fk:.0f} | {wk:.0f} | {fb + wb:.4g} | "
                         f"{'-' if ab is None else format(ab, '.4g')} | "
                         f"{(fb + wb) / entries[key]['avg_ms'] / 1e6:.1f} |")
    if sq:
        names = sorted({c for name, _, _ in wanted if name in sq for g in sq[name] for c in sq[name][g]})
        if names:
            keys = [(name, key) for name, key, _ in wanted if name in sq and key in entries]
            lines += ["", "## Instruction counters (`--pmc SQ_...`), per launch", "",
                      "| counter | " + " | ".join(f"`{k}`" for _, k in keys) + " |",
                      "|---" * (len(keys) + 1) + "|"]
            for c in names:
                vals = []
                for name, key in keys:
                    v = sq[name].get(entries[key]["grid"], {}).get(c, [])
                    vals.append(f"{_mean(v):.4g}" if v else "-")
                    if v:
                        entries[key][c] = _mean(v)
                lines.append(f"| {c} | " + " | ".join(vals) + " |")
            lines += ["", "VALU issue at 4 cycles per wave64 instruction on one of 1024 SIMDs at 2.4 GHz (the rate "
                      "of the SDWA folds, shifts and 24-bit multiplies; adds and logic issue faster):", "",
                      "| kernel | VALU instr / launch | VALU-issue ms | measured ms | VALU busy |", "|---|---|---|---|---|"]
            for name, key in keys:
                e = entries[key]
                if "SQ_INSTS_VALU" in e:
                    t = e["SQ_INSTS_VALU"] * 4 / 1024 / 2.4e9 * 1e3
                    lines.append(f"| `{key}` | {e['SQ_INSTS_VALU']:.4g} | {t:.1f} | {e['avg_ms']:.1f} | "
                                 f"{t / e['avg_ms']:.2f} |")
    with open(a.md, "w") as f:
        f.write("\n".join(lines) + "\n")
    if a.traffic:
        try:
            d = json.load(open(a.traffic))
        except Exception:
            d = {}
        if cal:
            d["calibration"] = cal
        wl = d.setdefault(a.workload, {})
        for k, v in entries.items():
            wl[k] = v
        with open(a.traffic, "w") as f:
            json.dump(d, f, indent=1)
    print(f"wrote {a.md}" + (f" and {a.traffic}" if a.traffic else ""))


if __name__ == "__main__":
    main()
