"""Summarise rocprofv3 CSV output into the short text/JSON records kept under profiles/.

  python -m paper_1806_10550_amd.profsum stats DIR [--title T]
      kernel-trace statistics (DIR holds *kernel_stats.csv) as a text table
  python -m paper_1806_10550_amd.profsum traffic --fetch D1 --write D2 --copy-fetch D3 \
      --copy-write D4 --copy-bytes B --hash H [--bench-args ARGS]
      per-kernel FETCH_SIZE / WRITE_SIZE per dispatch (KiB), with the scale factor that
      maps the counters onto the known byte count of a plain copy kernel, as JSON
  python -m paper_1806_10550_amd.profsum sq DIR [DIR ...] --hash H [--bench-args ARGS]
      per-kernel means per dispatch of the SQ counters of the given runs, as JSON
"""
import argparse
import csv
import glob
import json
import os
import re
import statistics
import sys

KERNEL_CLASSES = [
    (r"k_pass<0, false", "relations_y"),
    (r"k_pass<0, true", "solve_y"),
    (r"k_pass<1, false", "relations_x"),
    (r"k_pass<1, true", "solve_x"),
    (r"k_chain", "chain"),
    (r"k_xrow", "xrow"),
    (r"k_mass", "mass"),
    (r"k_flux_divergence", "rhs_theta"),
]


def classify(name):
    for pat, cls in KERNEL_CLASSES:
        if pat in name:
            return cls
    return name.split("(")[0][:60]


def _find(d, pattern):
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits[0]


def stats(d, title=None):
    path = _find(d, "*kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    out = []
    if title:
        out.append(title)
    out.append(f"{'kernel':60s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}")
    for r in rows:
        name = r.get("Name") or r.get("KernelName") or ""
        calls = int(r.get("Calls", 0))
        tot = float(r.get("TotalDurationNs", 0))
        avg = float(r.get("AverageNs", 0))
        mn = float(r.get("MinNs", 0))
        mx = float(r.get("MaxNs", 0))
        pct = float(r.get("Percentage", 0))
        out.append(f"{name[:60]:60s} {calls:7d} {tot / 1e6:10.3f} {avg / 1e3:10.1f} {mn / 1e3:10.1f} "
                   f"{mx / 1e3:10.1f} {pct:6.2f}")
    return "\n".join(out)


def counter_means(d, counter):
    path = _find(d, "*counter_collection.csv")
    per = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        per.setdefault(name, []).append(float(r["Counter_Value"]))
    return {k: statistics.mean(v) for k, v in per.items()}, {k: len(v) for k, v in per.items()}


def copy_duration_us(d, counter):
    """Mean duration of the calibration copy (the dispatches with the largest counter value)."""
    path = _find(d, "*counter_collection.csv")
    rows = [r for r in csv.DictReader(open(path)) if r.get("Counter_Name") == counter]
    top = max(float(r["Counter_Value"]) for r in rows)
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows
            if float(r["Counter_Value"]) >= 0.99 * top and "copy" in r.get("Kernel_Name", "").lower()]
    return statistics.mean(durs) if durs else None


# kernel classes that make up one iteration of the ADI-Newton step (the ones the records keep)
STEP_CLASSES = ("relations_y", "solve_y", "relations_x", "solve_x", "chain", "xrow")


def commands(bench_args):
    """The counter runs a traffic record summarises (R: the repository root, OUT: any output
    directory; run from /tmp with TMPDIR=/tmp); one counter per pass. bench_args: the
    arguments of the profiled bench.py run."""
    run = f"python $R/bench.py {bench_args}"
    return [
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_fetch -o run -- {run}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_write -o run -- {run}",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/copy_fetch -o run -- "
        "python $R/bench.py --calibrate-copy",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/copy_write -o run -- "
        "python $R/bench.py --calibrate-copy",
        "python -m paper_1806_10550_amd.profsum traffic --fetch $OUT/pmc_fetch --write $OUT/pmc_write "
        "--copy-fetch $OUT/copy_fetch --copy-write $OUT/copy_write --copy-bytes 1073741824 "
        f"--bench-args '{bench_args}' --hash $(python bench.py --print-hash)",
    ]


def traffic(a):
    fetch, nf = counter_means(a.fetch, "FETCH_SIZE")
    write, nw = counter_means(a.write, "WRITE_SIZE")
    cf, _ = counter_means(a.copy_fetch, "FETCH_SIZE")
    cw, _ = counter_means(a.copy_write, "WRITE_SIZE")
    # the copy kernel is the one with the largest counter value in the calibration run
    cf_kib = max(cf.values())
    cw_kib = max(cw.values())
    known_kib = a.copy_bytes / 1024.0
    out = {
        "commands": commands(a.bench_args),
        "kernel_hash": a.hash,
        "copy_bytes": a.copy_bytes,
        "copy_fetch_kib": cf_kib,
        "copy_write_kib": cw_kib,
        "fetch_scale": known_kib / cf_kib,
        "write_scale": known_kib / cw_kib,
        "copy_scale": 0.5 * (known_kib / cf_kib + known_kib / cw_kib),
        # the plain copy's own rate (read + write of copy_bytes; measured under the counters)
        "copy_us": copy_duration_us(a.copy_fetch, "FETCH_SIZE"),
        "kernels": {},
    }
    for name in fetch:
        cls = classify(name)
        if cls not in STEP_CLASSES:
            continue
        rec = out["kernels"].setdefault(cls, {"fetch_kib": 0.0, "write_kib": 0.0, "dispatches": 0})
        rec["fetch_kib"] = fetch[name] * (known_kib / cf_kib)
        rec["write_kib"] = write.get(name, 0.0) * (known_kib / cw_kib)
        rec["dispatches"] = nf[name]
    out["copy_gbs"] = 2.0 * a.copy_bytes / (out["copy_us"] * 1e3) if out["copy_us"] else None
    # bench.py multiplies (fetch + write) by copy_scale; the per-counter scales are
    # already applied above, so the combined scale is 1
    out["copy_scale"] = 1.0
    return out


def sq_commands(bench_args):
    run = f"python $R/bench.py {bench_args}"
    return [
        "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FMA_F64 "
        "SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64 SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES "
        f"--output-format csv -d $OUT/pmc_sqa -o run -- {run}",
        "rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_INST_ANY SQ_INSTS_LDS SQ_ACTIVE_INST_LDS "
        f"SQ_INSTS_SALU --output-format csv -d $OUT/pmc_sqb -o run -- {run}",
        f"python -m paper_1806_10550_amd.profsum sq $OUT/pmc_sqa $OUT/pmc_sqb --bench-args '{bench_args}' "
        "--hash $(python bench.py --print-hash)",
    ]


def sq(dirs, khash, bench_args):
    """Per kernel class: the mean per dispatch of every SQ counter in the given runs (counters
    summed over the device's shader engines by rocprofv3)."""
    out = {"commands": sq_commands(bench_args), "kernel_hash": khash, "kernels": {}}
    for d in dirs:
        path = _find(d, "*counter_collection.csv")
        acc = {}
        for r in csv.DictReader(open(path)):
            cls = classify(r.get("Kernel_Name", ""))
            if cls not in STEP_CLASSES:
                continue
            acc.setdefault(cls, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for cls, cs in acc.items():
            rec = out["kernels"].setdefault(cls, {})
            for c, v in cs.items():
                rec[c] = statistics.mean(v)
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--title")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--hash", required=True)
    t.add_argument("--bench-args", default="--steps 2 --warmup 1 --no-cpu-baseline")
    q = sub.add_parser("sq")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--hash", required=True)
    q.add_argument("--bench-args", default="--steps 2 --warmup 1 --no-cpu-baseline")
    a = ap.parse_args()
    if a.cmd == "stats":
        print(stats(a.dir, a.title))
    elif a.cmd == "sq":
        print(json.dumps(sq(a.dirs, a.hash, a.bench_args), indent=1))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    sys.exit(main())
