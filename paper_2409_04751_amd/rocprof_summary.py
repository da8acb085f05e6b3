"""Summaries of rocprofv3 CSV output (kernel stats and PMC counters).

    python -m paper_2409_04751_amd.rocprof_summary stats KERNEL_STATS.csv
    python -m paper_2409_04751_amd.rocprof_summary stats KERNEL_TRACE.csv --after preprocess_fused_kernel
    python -m paper_2409_04751_amd.rocprof_summary traffic \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \
        --copy-bytes 1073741824 --out profiles/traffic_<workload>.json
    python -m paper_2409_04751_amd.rocprof_summary counters C.csv --counters SQ_WAVES ...
    python -m paper_2409_04751_amd.rocprof_summary table --trace KERNEL_TRACE.csv --pmc A.csv B.csv \
        [--after preprocess_fused_kernel]
    python -m paper_2409_04751_amd.rocprof_summary marks KERNEL_TRACE.csv --match preprocess_kernel
    python -m paper_2409_04751_amd.rocprof_summary window KERNEL_TRACE.csv --begin I --end J --count preprocess_kernel

`marks` lists the launch indices (in start-time order) of the kernels whose
name contains a string; `window` sums the launches [I, J) of a kernel trace
per kernel, with the span from the first start to the last end and the
share of it the GPU was busy, per occurrence of the `--count` kernel (per
batch, per view).

`table` prints, per library kernel, the average duration in a rocprofv3
kernel trace and the
mean per dispatch of the SQ / TCC / GRBM counters found in the counter CSVs,
with derived figures (cycles = duration x 2.4 GHz, the peak engine clock,
so busy and occupancy figures are lower bounds when the clock runs lower;
GRBM_GUI_ACTIVE / 8, the cycles of the counter window per XCD, runs
longer than the kernel for short dispatches and is not used):
  VALU busy   SQ_INSTS_VALU / (256 CUs x cycles): a CU issues at most one
              wave64 VALU instruction per cycle (four SIMD16 units, four
              cycles per wave64 instruction);
  waves/SIMD  SQ_WAVE_CYCLES x 4 / (1024 SIMDs x cycles): resident waves per
              SIMD averaged over the dispatch (SQ_WAVE_CYCLES counts
              wave-cycles in units of four cycles);
  wait        SQ_WAIT_ANY / SQ_WAVE_CYCLES: share of wave time spent waiting;
  fp32 TFLOP/s  64 x (SQ_INSTS_VALU_FLOPS_FP32 + SQ_INSTS_VALU_FLOPS_FP32_TRANS)
              / duration: the counters count the flops of each wave64
              instruction once, not per lane;
  atomics/s   TCC_ATOMIC / the rocprofv3 average duration.

`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch, from two
separate `rocprofv3 --pmc` runs) into HBM bytes per launch of each library
kernel.
Each counter is scaled by what it reads for a plain device copy of a known
size: the factor is (copy bytes / 1024) / counter value for the copy kernel,
so a counter that samples only part of the memory channels, or counts in
other units, is corrected by the same ratio.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys

COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_stats(path: str) -> list[dict]:
    """Rows of a rocprofv3 `*_kernel_stats.csv`, heaviest first."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            rows.append(dict(name=r["Name"], calls=int(r["Calls"]), total_ns=float(r["TotalDurationNs"]),
                             avg_ns=float(r["AverageNs"]), pct=float(r["Percentage"])))
    rows.sort(key=lambda r: -r["total_ns"])
    return rows


def trace_stats(path: str, after: str | None = None) -> list[dict]:
    """kernel_stats rows computed from a `*_kernel_trace.csv`, counting only
    the launches from the first launch of `after` on."""
    start = first_dispatch(path, after)
    agg: dict[str, list] = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if int(r["Dispatch_Id"]) < start:
                continue
            a = agg.setdefault(r["Kernel_Name"], [0, 0])
            a[0] += 1
            a[1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    total = sum(a[1] for a in agg.values()) or 1
    rows = [dict(name=k, calls=a[0], total_ns=float(a[1]), avg_ns=a[1] / a[0], pct=100.0 * a[1] / total)
            for k, a in agg.items()]
    rows.sort(key=lambda r: -r["total_ns"])
    return rows


def first_dispatch(path: str, kernel_substr: str | None) -> int:
    """Dispatch id of the first launch of a kernel whose name contains
    `kernel_substr` (0 if None): launches before it, such as a scene's
    one-off set-up, are left out of the per-dispatch means."""
    if not kernel_substr:
        return 0
    first = None
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if kernel_substr in r["Kernel_Name"]:
                d = int(r["Dispatch_Id"])
                first = d if first is None else min(first, d)
    if first is None:
        raise SystemExit(f"no kernel matching {kernel_substr!r} in {path}")
    return first


def counter_means(path: str, kernel_substr: str, counter: str, after: str | None = None) -> tuple[float, int]:
    """Mean value of `counter` per dispatch over kernels whose name contains
    `kernel_substr` (from the first launch of `after` on); returns (mean,
    dispatches)."""
    start = first_dispatch(path, after)
    per_dispatch: dict[str, float] = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter or kernel_substr not in r["Kernel_Name"]:
                continue
            if int(r["Dispatch_Id"]) < start:
                continue
            d = r["Dispatch_Id"]
            per_dispatch[d] = per_dispatch.get(d, 0.0) + float(r["Counter_Value"])
    if not per_dispatch:
        raise SystemExit(f"no {counter} rows for a kernel matching {kernel_substr!r} in {path}")
    return sum(per_dispatch.values()) / len(per_dispatch), len(per_dispatch)


# profiler kernel names of the library's kernels, as they appear (demangled)
# in rocprofv3 output, keyed by the names the library's event profiler uses
KERNELS = {
    "preprocess": "::preprocess_fused_kernel<",
    "preprocess_batch": "::preprocess_kernel<",
    "color": "::color_kernel<",
    "compact": "::compact_kernel(",
    "depth_sort_scatter": "::radix_scatter_kernel<3,",
    "rows": "::rows_kernel(",
    "duplicate_hist": "::dup_hist_kernel(",
    "duplicate": "::dup_scatter_kernel<",
    "tile_sort_hist": "::radix_hist_kernel<12,",
    "tile_sort_scatter": "::radix_scatter_kernel<1,",
    "ranges": "::ranges_kernel(",
    "blend_forward": "::blend_forward_kernel<false>",
    "blend_backward": "::blend_backward_kernel<false>",
    "preprocess_backward": "::backward_fused_kernel<",
    "loss": "::l1_",
}


def traffic(args) -> dict:
    """HBM bytes per launch of each library kernel, calibrated by the copy."""
    copy_kib = args.copy_bytes / 1024.0
    cf, _ = counter_means(args.copy_fetch, COPY_KERNEL, "FETCH_SIZE")
    cw, _ = counter_means(args.copy_write, COPY_KERNEL, "WRITE_SIZE")
    fetch_factor = copy_kib / cf
    write_factor = copy_kib / cw
    kernels = {}
    for name, sub in KERNELS.items():
        try:
            fk, nf = counter_means(args.fetch, sub, "FETCH_SIZE", args.after)
            wk, nw = counter_means(args.write, sub, "WRITE_SIZE", args.after)
        except SystemExit:
            continue
        read_b = fk * 1024.0 * fetch_factor
        write_b = wk * 1024.0 * write_factor
        kernels[name] = dict(dispatches=nf, fetch_kib_raw=round(fk, 1), write_kib_raw=round(wk, 1),
                             read_bytes_per_launch=round(read_b), write_bytes_per_launch=round(write_b),
                             bytes_per_launch=round(read_b + write_b))
    rec = dict(workload=args.workload, command=args.command, source_sha=args.source_sha,
               copy_calibration=dict(bytes=args.copy_bytes, fetch_kib=round(cf, 1), write_kib=round(cw, 1),
                                     fetch_factor=round(fetch_factor, 4), write_factor=round(write_factor, 4)),
               kernels=kernels)
    return rec


def trace_launches(path: str) -> list[tuple[str, int, int]]:
    """(short kernel name, start ns, end ns) of a rocprofv3 `*_kernel_trace.csv`,
    in start order."""
    out = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"].replace("fgs::(anonymous namespace)::", "").replace("void ", "")
            out.append((name.split("(")[0], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    out.sort(key=lambda x: x[1])
    return out


def window(launches, begin: int, end: int, count: str) -> dict:
    sub = launches[begin:end]
    agg: dict[str, list] = {}
    for name, t0, t1 in sub:
        a = agg.setdefault(name, [0, 0])
        a[0] += 1
        a[1] += t1 - t0
    busy = sum(a[1] for a in agg.values())
    span = sub[-1][2] - sub[0][1]
    units = sum(1 for name, _, _ in sub if count in name)
    return dict(launches=len(sub), span_ms=span / 1e6, busy_ms=busy / 1e6, busy_frac=busy / span, units=units,
                kernels=sorted(((n, a[0], a[1] / 1e6) for n, a in agg.items()), key=lambda x: -x[2]))


def counter_table(path: str, counters: list[str]) -> dict:
    """Mean per dispatch of each counter for each library kernel."""
    out = {}
    for name, sub in KERNELS.items():
        row = {}
        for c in counters:
            try:
                row[c], row["dispatches"] = counter_means(path, sub, c)
            except SystemExit:
                pass
        if row:
            out[name] = row
    return out


CLOCK_HZ = 2.4e9  # MI355X peak engine clock


def trace_avg_ms(path: str, sub: str, after: str | None = None) -> float | None:
    """Average duration (ms) of the launches in a rocprofv3 kernel trace whose
    name contains `sub`, from the first launch of `after` on."""
    start = first_dispatch(path, after)
    calls = 0
    total = 0
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if sub in r["Kernel_Name"] and int(r["Dispatch_Id"]) >= start:
                calls += 1
                total += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    return total / calls / 1e6 if calls else None


def counter_rows(trace_csv: str, pmc_csvs: list[str], after: str | None = None) -> dict:
    """Per library kernel: duration, raw counter means and derived figures."""
    names = set()
    for path in pmc_csvs:
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                names.add(r["Counter_Name"])
    out = {}
    for kname, sub in KERNELS.items():
        ms = trace_avg_ms(trace_csv, sub, after)
        if ms is None:
            continue
        raw = {}
        for path in pmc_csvs:
            for c in sorted(names):
                if c in raw:
                    continue
                try:
                    raw[c], _ = counter_means(path, sub, c, after)
                except SystemExit:
                    pass
        if not raw:
            continue
        row = dict(ms=ms, raw=raw)
        cyc = ms * 1e-3 * CLOCK_HZ
        if "SQ_INSTS_VALU" in raw:
            row["valu_busy"] = raw["SQ_INSTS_VALU"] / (256.0 * cyc)
        if "SQ_WAVE_CYCLES" in raw:
            row["waves_per_simd"] = raw["SQ_WAVE_CYCLES"] * 4.0 / (1024.0 * cyc)
        if raw.get("SQ_WAVE_CYCLES", 0.0) > 0 and "SQ_WAIT_ANY" in raw:
            row["wait"] = raw["SQ_WAIT_ANY"] / raw["SQ_WAVE_CYCLES"]
        if "TCC_ATOMIC" in raw:
            row["atomics_per_s"] = raw["TCC_ATOMIC"] / (ms * 1e-3)
        if "SQ_INSTS_VALU_FLOPS_FP32" in raw:
            fl = 64.0 * (raw["SQ_INSTS_VALU_FLOPS_FP32"] + raw.get("SQ_INSTS_VALU_FLOPS_FP32_TRANS", 0.0))
            row["fp32_gflop"] = fl / 1e9
            row["fp32_tflops"] = fl / (ms * 1e-3) / 1e12
        out[kname] = row
    return out


def print_table(rows: dict) -> None:
    cols = [("ms", "ms", "{:.4f}"), ("valu_busy", "VALU busy", "{:.2f}"),
            ("waves_per_simd", "waves/SIMD", "{:.2f}"), ("wait", "wait", "{:.2f}"),
            ("fp32_gflop", "fp32 GFLOP", "{:.3f}"), ("fp32_tflops", "fp32 TFLOP/s", "{:.1f}"),
            ("atomics_per_s", "atomics/s", "{:.3e}")]
    print(f"{'kernel':<20}" + "".join(f"{h:>13}" for _, h, _ in cols))
    for k, r in rows.items():
        print(f"{k:<20}" + "".join(f"{fmt.format(r[c]) if c in r else '-':>13}" for c, _, fmt in cols))
    counters = sorted({c for r in rows.values() for c in r["raw"]})
    print()
    print("raw counter means per dispatch")
    for i in range(0, len(counters), 6):
        part = counters[i:i + 6]
        print(f"{'kernel':<20}" + "".join(f"{c[-22:]:>24}" for c in part))
        for k, r in rows.items():
            print(f"{k:<20}" + "".join(f"{r['raw'][c]:>24.4e}" if c in r["raw"] else f"{'-':>24}" for c in part))
        print()


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv", help="*_kernel_stats.csv, or a *_kernel_trace.csv (then --after applies)")
    s.add_argument("--top", type=int, default=30)
    s.add_argument("--after", default=None, help="leave out launches before the first of this kernel")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--workload", default="")
    t.add_argument("--source-sha", default=None)
    t.add_argument("--command", default=None)
    t.add_argument("--out", default=None)
    t.add_argument("--after", default=None, help="leave out dispatches before the first of this kernel")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--counters", nargs="+", required=True)
    tb = sub.add_parser("table")
    tb.add_argument("--trace", required=True, help="rocprofv3 *_kernel_trace.csv for the durations")
    tb.add_argument("--pmc", nargs="+", required=True)
    tb.add_argument("--after", default=None, help="leave out dispatches before the first of this kernel")
    m = sub.add_parser("marks")
    m.add_argument("csv")
    m.add_argument("--match", required=True)
    w = sub.add_parser("window")
    w.add_argument("csv")
    w.add_argument("--begin", type=int, required=True)
    w.add_argument("--end", type=int, required=True)
    w.add_argument("--count", required=True)
    w.add_argument("--top", type=int, default=20)
    args = ap.parse_args(argv)
    if args.cmd == "marks":
        print(" ".join(str(i) for i, (name, _, _) in enumerate(trace_launches(args.csv)) if args.match in name))
        return 0
    if args.cmd == "window":
        r = window(trace_launches(args.csv), args.begin, args.end, args.count)
        u = max(r["units"], 1)
        print(f"launches [{args.begin}, {args.end}): {r['launches']}; span {r['span_ms']:.3f} ms; GPU busy "
              f"{r['busy_ms']:.3f} ms ({r['busy_frac']:.2f}); {r['units']} x {args.count}: "
              f"{r['busy_ms'] / u:.3f} ms busy each")
        print(f"{'kernel':<46} {'calls':>6} {'total_ms':>10} {'per unit ms':>12}")
        for name, calls, ms in r["kernels"][:args.top]:
            print(f"{name[:46]:<46} {calls:>6} {ms:>10.3f} {ms / u:>12.3f}")
        return 0
    if args.cmd == "stats":
        rows = trace_stats(args.csv, args.after) if args.csv.endswith("kernel_trace.csv") else kernel_stats(args.csv)
        total = sum(r["total_ns"] for r in rows)
        print(f"{'kernel':<70} {'calls':>6} {'total_ms':>10} {'avg_us':>10} {'pct':>6}")
        for r in rows[:args.top]:
            print(f"{r['name'][:70]:<70} {r['calls']:>6} {r['total_ns'] / 1e6:>10.3f} {r['avg_ns'] / 1e3:>10.2f} "
                  f"{r['pct']:>6.2f}")
        print(f"{'total':<70} {'':>6} {total / 1e6:>10.3f}")
        return 0
    if args.cmd == "table":
        print_table(counter_rows(args.trace, args.pmc, args.after))
        return 0
    if args.cmd == "counters":
        print(json.dumps(counter_table(args.csv, args.counters), indent=1))
        return 0
    rec = traffic(args)
    text = json.dumps(rec, indent=1)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
