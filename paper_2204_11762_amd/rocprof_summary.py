"""Short text summaries of rocprofv3 CSV output for the ray caster.

Two subcommands:

``kernels``  turns ``<prefix>_kernel_stats.csv`` of a
             ``rocprofv3 --kernel-trace --stats --output-format csv`` run into
             a fixed-width table (calls, total, average, min, max per kernel).

``traffic``  turns the ``<prefix>_counter_collection.csv`` files of two
             ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
             ``bench.py --copy-calib MIB`` into HBM bytes per launch of the
             render kernel.  Each counter is scaled by the factor that makes
             it read the known traffic of the calibration copy (MIB MiB read
             and MIB MiB written by one device-to-device copy), and the
             result is keyed by the SHA-256 of the kernel source that the
             profiled bench printed, so that a stale summary is recognised.

``counters`` turns the ``<prefix>_counter_collection.csv`` files of one or
             more ``rocprofv3 --pmc ...`` passes into the median value per
             dispatch of each counter for the kernels matching a pattern,
             and that value per unit of work (composited samples or
             points per dispatch, given); counts of wave instructions
             (``SQ_INSTS_*``) are also given per lane (times 64).

Each writes the full profiling commands into the summary.
"""

from __future__ import annotations

import argparse
import csv
import json
import re
import statistics
import sys

# render_brick_kernel<P, STORE, SHADE, ...>: degree, storage and shading of
# the hot kernel
RENDER_RE = re.compile(r"render_brick_kernel<(\d+), (\d+), (true|false),")


def kernel_table(stats_csv: str) -> list[dict]:
    rows = []
    with open(stats_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]),
                         "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                         "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"]),
                         "pct": float(r["Percentage"])})
    rows.sort(key=lambda x: -x["total_ns"])
    return rows


def short_name(name: str) -> str:
    name = name.replace("mfa::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*\)$", "", name)


def cmd_counters(args) -> None:
    pat = re.compile(args.kernel)
    vals: dict[str, list[float]] = {}
    kernels: set[str] = set()
    for path in args.csv:
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                if not pat.search(r["Kernel_Name"]):
                    continue
                kernels.add(short_name(r["Kernel_Name"]))
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {args.kernel!r}")
    out = [f"# rocprofv3 counters: {args.title}", "#"]
    out += [f"# command: {c}" for c in args.command]
    out += ["#", f"# kernel(s): {', '.join(sorted(kernels))}",
            f"# per {args.unit}: {args.per:.6g} {args.unit}s per dispatch", "#",
            f"{'counter':28s} {'dispatches':>10} {'median':>14} {'min':>14} {'max':>14} "
            f"{'per ' + args.unit:>14} {'x64 per ' + args.unit:>16}"]
    for name in sorted(vals):
        v = vals[name]
        med = statistics.median(v)
        lane = f"{64.0 * med / args.per:16.3f}" if name.startswith("SQ_INSTS_") else f"{'':16s}"
        out.append(f"{name:28s} {len(v):10d} {med:14.6g} {min(v):14.6g} {max(v):14.6g} "
                   f"{med / args.per:14.6g} {lane}")
    if args.log:
        out += ["", "# the profiled program's own report (same run):"]
        for path in args.log:
            with open(path) as fh:
                out += ["#   " + ln.rstrip() for ln in fh if ln.startswith("[profile]")]
    text = "\n".join(out) + "\n"
    with open(args.out, "w") as fh:
        fh.write(text)
    sys.stdout.write(text)


# lines of the profiled program's report that a kernel table quotes: the
# per-leg figures of the bench and of profile_frames
BENCH_LINES = ("[bench] store=", "[bench] batch:", "[bench] tuned batch:",
               "[bench] autotune model", "[bench] serve:", "[bench] curvature:",
               "[bench] eval sweep", "[profile]")


def cmd_kernels(args) -> None:
    rows = kernel_table(args.stats)
    out = [f"# rocprofv3 kernel statistics: {args.title}", "#", f"# command: {args.command}",
           "#", f"{'calls':>6} {'total_ms':>10} {'avg_us':>10} {'min_us':>10} {'max_us':>10} "
           f"{'pct':>6}  kernel"]
    for r in rows:
        out.append(f"{r['calls']:6d} {r['total_ns'] / 1e6:10.3f} {r['avg_ns'] / 1e3:10.2f} "
                   f"{r['min_ns'] / 1e3:10.2f} {r['max_ns'] / 1e3:10.2f} {r['pct']:6.2f}  "
                   f"{short_name(r['name'])}")
    if args.bench_log:
        out += ["", "# the profiled program's own report (same run):"]
        with open(args.bench_log) as fh:
            out += ["#   " + ln.rstrip() for ln in fh
                    if ln.startswith(BENCH_LINES) or "kernel source sha256" in ln]
    text = "\n".join(out) + "\n"
    with open(args.out, "w") as fh:
        fh.write(text)
    sys.stdout.write(text)


def counter_rows(path: str, counter: str) -> list[dict]:
    with open(path, newline="") as fh:
        return [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]


def source_hash(log_path: str) -> str:
    with open(log_path) as fh:
        for line in fh:
            m = re.search(r"kernel source sha256 ([0-9a-f]{64})", line)
            if m:
                return m.group(1)
    raise SystemExit(f"{log_path}: no 'kernel source sha256' line")


def calibration(rows: list[dict], copy_bytes: int) -> tuple[float, float]:
    """(counter KiB of the calibration copy, bytes per counter KiB)."""
    copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    if not copies:
        raise SystemExit("no copy dispatch found for calibration")
    kib = max(copies)              # the calibration copy is the largest copy of the run
    return kib, copy_bytes / kib


def per_leg(rows: list[dict]) -> dict:
    legs: dict[str, list[float]] = {}
    names: dict[str, str] = {}
    for r in rows:
        m = RENDER_RE.search(r["Kernel_Name"])
        if not m:
            continue
        # shaded frames are the storage's leg; value-only frames a leg of their own
        store = {"0": "fp32", "1": "bf16", "2": "fp16"}[m.group(2)]
        if m.group(3) == "false":
            store += "_value_only"
        legs.setdefault(store, []).append(float(r["Counter_Value"]))
        names[store] = short_name(r["Kernel_Name"])
    return {k: {"kernel": names[k], "dispatches": len(v), "kib_median": statistics.median(v),
                "kib_min": min(v), "kib_max": max(v)} for k, v in legs.items()}


def cmd_traffic(args) -> None:
    copy_bytes = args.copy_mib << 20
    fetch = counter_rows(args.fetch, "FETCH_SIZE")
    write = counter_rows(args.write, "WRITE_SIZE")
    f_kib, f_scale = calibration(fetch, copy_bytes)
    w_kib, w_scale = calibration(write, copy_bytes)
    hf, hw = source_hash(args.fetch_log), source_hash(args.write_log)
    if hf != hw:
        raise SystemExit("the two counter runs profiled different kernel sources")
    fl, wl_ = per_leg(fetch), per_leg(write)
    legs = {}
    for store in sorted(set(fl) & set(wl_)):
        rd = fl[store]["kib_median"] * f_scale
        wr = wl_[store]["kib_median"] * w_scale
        legs[store] = {"kernel": fl[store]["kernel"], "dispatches": fl[store]["dispatches"],
                       "fetch_kib_median": fl[store]["kib_median"],
                       "write_kib_median": wl_[store]["kib_median"],
                       "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr,
                       "hbm_bytes_per_launch": rd + wr}
    rec = {"kernel_source_sha256": hf,
           "commands": {"fetch": args.fetch_command, "write": args.write_command},
           "calibration": {"copy_bytes_read": copy_bytes, "copy_bytes_written": copy_bytes,
                           "copy_fetch_kib": f_kib, "copy_write_kib": w_kib,
                           "fetch_bytes_per_kib": f_scale, "write_bytes_per_kib": w_scale},
           "legs": legs}
    with open(args.out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    json.dump(rec, sys.stdout, indent=1)
    sys.stdout.write("\n")


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("stats")
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--bench-log", help="stderr of the profiled bench.py, whose per-leg "
                                       "lines are appended")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--fetch-log", required=True)
    t.add_argument("--write-log", required=True)
    t.add_argument("--fetch-command", required=True)
    t.add_argument("--write-command", required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+", help="counter_collection.csv of each pass")
    c.add_argument("--kernel", default=r"render_brick_kernel<",
                   help="pattern of the kernel names summarised")
    c.add_argument("--per", type=float, required=True,
                   help="units of work per dispatch (e.g. composited samples)")
    c.add_argument("--unit", default="sample")
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", required=True,
                   help="profiling command of a pass (repeat per pass)")
    c.add_argument("--log", action="append", help="output of a profiled program")
    c.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    {"kernels": cmd_kernels, "traffic": cmd_traffic, "counters": cmd_counters}[args.cmd](args)


if __name__ == "__main__":
    main()
