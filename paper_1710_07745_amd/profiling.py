"""Summaries of rocprofv3 output for the measurements kept under profiles/.

  python -m paper_1710_07745_amd.profiling stats DIR [--title T] [--command C]
      kernel table from DIR/*_kernel_stats.csv (rocprofv3 --kernel-trace
      --stats --output-format csv).
  python -m paper_1710_07745_amd.profiling valu PMC_DIR [--kernel SUBSTR] [--command C ...]
      VALU instructions (SQ_INSTS_VALU, per wave) and waves (SQ_WAVES) per
      launch of the kernel, from one counter run (median over dispatches).
  python -m paper_1710_07745_amd.profiling traffic-table FETCH_DIR WRITE_DIR
      --copy-bytes N --kernel NAME=ALG_BYTES [--kernel ...]
      the same for several kernels of one run pair, as a table with each
      kernel's algorithmic bytes and the ratio.
  python -m paper_1710_07745_amd.profiling counters PMC_DIR --kernel SUBSTR [--kernel ...]
      every counter of one run, median per dispatch, for each kernel named.
  python -m paper_1710_07745_amd.profiling traffic FETCH_DIR WRITE_DIR
      --kernel SUBSTR --copy-bytes N [--command C ...]
      HBM bytes per launch of the kernel whose name contains SUBSTR, from two
      counter runs (FETCH_SIZE, then WRITE_SIZE, each in KiB per dispatch; the median over dispatches).
      Each counter is scaled by what it reads for the device copy kernel of
      N bytes in the same run (a copy fetches N and writes N bytes).

The float walk's traffic and VALU summaries carry a hash of the kernel's
sources; the benchmark reports their figures only while the hash still matches.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WALK_SOURCES = ("paper_1710_07745_amd/csrc/canny_f32_forward.hip",
                "paper_1710_07745_amd/csrc/canny_f32_common.h",
                "paper_1710_07745_amd/csrc/canny_internal.h")
WALK_KERNEL = "k_f32_forward_bal<3, 40, 23, true, false>"
COPY_KERNEL = "copy"  # the device-to-device copy kernel's name contains this


def walk_source_hash() -> str:
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _read_field(path: str, field: str):
    """A numeric field of a summary, or None when the file is missing or the
    walk's sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    kv = {}
    for ln in open(path):
        if ":" in ln and not ln.lstrip().startswith("#"):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != walk_source_hash():
        return None
    try:
        return float(kv[field])
    except (KeyError, ValueError):
        return None


def read_traffic(path: str):
    """traffic_bytes_per_launch of a traffic summary (None if missing or stale)."""
    return _read_field(path, "traffic_bytes_per_launch")


def read_valu(path: str):
    """valu_insts_per_launch (wave instructions) of a VALU summary (None if
    missing or stale)."""
    return _read_field(path, "valu_insts_per_launch")


def _one(pattern: str) -> str:
    files = sorted(glob.glob(pattern))
    if not files:
        sys.exit(f"no file matches {pattern}")
    return files[0]


def short(name: str, n: int = 90) -> str:
    name = name.replace("canny::(anonymous namespace)::", "").replace("void ", "")
    return name if len(name) <= n else name[: n - 3] + "..."


def stats(args) -> None:
    rows = list(csv.DictReader(open(_one(os.path.join(args.dir, "*kernel_stats.csv")))))
    print(f"# {args.title}")
    if args.command:
        print(f"# command: {args.command}")
    print(f"{'calls':>6} {'avg_us':>9} {'min_us':>9} {'max_us':>9} {'share%':>7}  kernel")
    for r in rows:
        print(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} "
              f"{float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):7.2f}  {short(r['Name'])}")


def _per_dispatch(d: str, counter: str, substr: str, pick: str = "median"):
    vals = []
    for r in csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))):
        if r["Counter_Name"] == counter and substr in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    if not vals:
        sys.exit(f"no {counter} rows for kernels matching {substr!r} in {d}")
    vals.sort()
    if pick == "max":  # the calibration copy: the largest copy of the run, not an upload
        return vals[-1], len(vals)
    return vals[len(vals) // 2], len(vals)


def traffic(args) -> None:
    kib = 1024.0
    f_k, nf = _per_dispatch(args.fetch_dir, "FETCH_SIZE", args.kernel)
    w_k, nw = _per_dispatch(args.write_dir, "WRITE_SIZE", args.kernel)
    f_c, _ = _per_dispatch(args.fetch_dir, "FETCH_SIZE", COPY_KERNEL, "max")
    w_c, _ = _per_dispatch(args.write_dir, "WRITE_SIZE", COPY_KERNEL, "max")
    fs = args.copy_bytes / (f_c * kib)
    ws = args.copy_bytes / (w_c * kib)
    total = f_k * kib * fs + w_k * kib * ws
    print(f"# HBM traffic of {args.kernel} (hardware counters, per dispatch)")
    for c in args.command or []:
        print(f"# command: {c}")
    print(f"kernel: {args.kernel}")
    print(f"source_sha256: {walk_source_hash()}")
    print(f"dispatches_fetch: {nf}")
    print(f"dispatches_write: {nw}")
    print(f"fetch_kib_per_dispatch: {f_k:.1f}")
    print(f"write_kib_per_dispatch: {w_k:.1f}")
    print(f"copy_bytes: {args.copy_bytes}")
    print(f"copy_fetch_kib: {f_c:.1f}")
    print(f"copy_write_kib: {w_c:.1f}")
    print(f"fetch_scale: {fs:.4f}")
    print(f"write_scale: {ws:.4f}")
    print(f"traffic_bytes_per_launch: {total:.0f}")
    if args.alg_bytes:
        print(f"algorithmic_bytes_per_launch: {args.alg_bytes:.0f}")
        print(f"traffic_over_algorithmic: {total / args.alg_bytes:.3f}")


def traffic_table(args) -> None:
    """HBM bytes per launch of several kernels of one run pair, each counter
    scaled by its reading for the copy kernel, beside the kernel's algorithmic
    bytes (NAME=BYTES; 0 when the kernel has no figure of its own)."""
    kib = 1024.0
    f_c, _ = _per_dispatch(args.fetch_dir, "FETCH_SIZE", COPY_KERNEL, "max")
    w_c, _ = _per_dispatch(args.write_dir, "WRITE_SIZE", COPY_KERNEL, "max")
    fs = args.copy_bytes / (f_c * kib)
    ws = args.copy_bytes / (w_c * kib)
    print(f"# HBM traffic per launch (FETCH_SIZE x {fs:.4f}, WRITE_SIZE x {ws:.4f}: the factors "
          f"that make a {args.copy_bytes:.0f}-byte device copy read and write its size)")
    for c in args.command or []:
        print(f"# command: {c}")
    print(f"{'kernel':48s} {'fetch_MB':>10s} {'write_MB':>10s} {'total_MB':>10s} {'alg_MB':>10s} {'ratio':>7s}")
    for spec in args.kernel:
        name, _, alg = spec.rpartition("=")
        alg = float(alg)
        f_k, _ = _per_dispatch(args.fetch_dir, "FETCH_SIZE", name)
        w_k, _ = _per_dispatch(args.write_dir, "WRITE_SIZE", name)
        fb, wb = f_k * kib * fs, w_k * kib * ws
        ratio = f"{(fb + wb) / alg:7.2f}" if alg > 0 else f"{'-':>7s}"
        alg_s = f"{alg / 1e6:10.1f}" if alg > 0 else f"{'-':>10s}"
        print(f"{name[:48]:48s} {fb / 1e6:10.1f} {wb / 1e6:10.1f} {(fb + wb) / 1e6:10.1f} {alg_s} {ratio}")


def valu(args) -> None:
    insts, n = _per_dispatch(args.dir, "SQ_INSTS_VALU", args.kernel)
    waves, _ = _per_dispatch(args.dir, "SQ_WAVES", args.kernel)
    print(f"# VALU instructions of {args.kernel} (hardware counters, per dispatch)")
    for c in args.command or []:
        print(f"# command: {c}")
    print(f"kernel: {args.kernel}")
    print(f"source_sha256: {walk_source_hash()}")
    print(f"dispatches: {n}")
    print(f"valu_insts_per_launch: {insts:.0f}")
    print(f"waves_per_launch: {waves:.0f}")
    print(f"valu_insts_per_wave: {insts / max(waves, 1):.1f}")


def counters(args) -> None:
    rows = list(csv.DictReader(open(_one(os.path.join(args.dir, "*counter_collection.csv")))))
    names = sorted({r["Counter_Name"] for r in rows})
    print("# hardware counters per dispatch (median over dispatches)")
    for c in args.command or []:
        print(f"# command: {c}")
    print(f"{'kernel':44s} " + " ".join(f"{n:>20s}" for n in names))
    for k in args.kernel:
        vals = []
        for n in names:
            v = sorted(float(r["Counter_Value"]) for r in rows
                       if r["Counter_Name"] == n and k in r["Kernel_Name"])
            vals.append(f"{v[len(v) // 2]:20.0f}" if v else f"{'-':>20s}")
        print(f"{k[:44]:44s} " + " ".join(vals))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--title", default="rocprofv3 kernel statistics")
    s.add_argument("--command", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", default=WALK_KERNEL)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--alg-bytes", type=float, default=0.0)
    t.add_argument("--command", action="append")
    tt = sub.add_parser("traffic-table")
    tt.add_argument("fetch_dir")
    tt.add_argument("write_dir")
    tt.add_argument("--kernel", action="append", required=True, help="NAME=ALG_BYTES")
    tt.add_argument("--copy-bytes", type=float, required=True)
    tt.add_argument("--command", action="append")
    v = sub.add_parser("valu")
    v.add_argument("dir")
    v.add_argument("--kernel", default=WALK_KERNEL)
    v.add_argument("--command", action="append")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--command", action="append")
    a = ap.parse_args(argv)
    {"stats": stats, "traffic": traffic, "traffic-table": traffic_table, "valu": valu,
     "counters": counters}[a.cmd](a)


if __name__ == "__main__":
    main()
