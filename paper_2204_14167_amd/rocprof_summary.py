"""Summaries of rocprofv3 result databases for the profiles/ folder.

  python -m paper_2204_14167_amd.rocprof_summary kernels KT.db --command "..." > out.md
      per-kernel dispatch count and mean / min / max duration (kernel-trace run)
  python -m paper_2204_14167_amd.rocprof_summary traffic FETCH.db WRITE.db --command "..." > out.md
      HBM bytes per dispatch of every kernel from a FETCH_SIZE run and a WRITE_SIZE run,
      each scaled by what the same counter reads for the 1 GiB device copy those runs
      include (bench.py --copy-calibration), with a fenced JSON block that bench.py reads
  python -m paper_2204_14167_amd.rocprof_summary issue SQ.db KT.db --command "..." > out.md
      instructions per wavefront (VALU, SALU, vector memory reads, LDS) from an SQ counter
      run, and the share of VALU issue cycles each kernel fills over its kernel-trace
      duration: a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles, and the
      chip has 1024 SIMDs (256 CUs x 4) at 2.4 GHz

All read only the rocpd SQLite tables `kernels` and `counters_collection`.  The JSON
blocks of the traffic and issue summaries carry the sha256 of every HIP source file and
header at the time of the run, so that a reader can tell which kernels have changed since.
"""
import argparse
import hashlib
import json
import os
import re
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

COPY_BYTES = 1 << 30  # the calibration copy of bench.py --copy-calibration
SIMDS, CLOCK_HZ, CYCLES_PER_VALU = 1024, 2.4e9, 4


def _short(name):
    """Kernel name without namespace, return type and call arguments (template arguments
    kept, so that instantiations stay apart)."""
    name = re.sub(r"\(.*", "", name).replace("discos::", "")
    return re.sub(r"^void ", "", name)


def source_hashes(base=CSRC):
    """{file name: sha256} of the HIP sources and headers."""
    out = {}
    for name in sorted(os.listdir(base)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(base, name), "rb") as f:
                out[name] = hashlib.sha256(f.read()).hexdigest()
    return out


def kernel_files(kernel, base=CSRC):
    """The source files a kernel's timing and traffic depend on: the file that defines it
    (a __global__ function of that name) and every header."""
    stem = re.escape(kernel.split("<", 1)[0])
    pat = re.compile(r"__global__[^;{]*?\b" + stem + r"\s*\(")
    files = []
    for name in sorted(os.listdir(base)):
        if name.endswith(".h"):
            files.append(name)
        elif name.endswith(".hip"):
            with open(os.path.join(base, name)) as f:
                if pat.search(f.read()):
                    files.append(name)
    return files


def sources_unchanged(data, kernel, base=CSRC):
    """True if the profile block `data` was taken on the present sources of `kernel`."""
    then = data.get("source_sha256")
    if not isinstance(then, dict):
        return False
    now = source_hashes(base)
    files = kernel_files(kernel, base)
    return any(f.endswith(".hip") for f in files) and all(then.get(f) == now[f] for f in files)


def kernel_rows(db):
    cur = sqlite3.connect(db).cursor()
    q = ("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
         "from kernels group by name order by sum(duration) desc")
    return [(_short(r[0]),) + tuple(r[1:]) for r in cur.execute(q).fetchall()]


def counter_means(db, counter):
    """{kernel: (dispatches, mean KiB, max KiB)} for one counter."""
    cur = sqlite3.connect(db).cursor()
    q = ("select kernel_name, count(*), avg(value), max(value) from counters_collection "
         "where counter_name = ? group by kernel_name")
    return {_short(r[0]): (r[1], r[2], r[3]) for r in cur.execute(q, (counter,)).fetchall()}


def copy_factor(means):
    """Known bytes / counted bytes of the largest device-copy dispatch (the 1 GiB copy)."""
    best = 0.0
    for k, (_, _, mx) in means.items():
        if "copyBuffer" in k:
            best = max(best, mx)
    if best <= 0.0:
        raise SystemExit("no calibration copy in the counter run (bench.py --copy-calibration)")
    return COPY_BYTES / (best * 1024.0)


def cmd_kernels(args):
    rows = kernel_rows(args.db)
    tot = sum(r[5] for r in rows)
    print(f"# Kernel trace: {args.title}\n")
    print(f"Command:\n\n    {args.command}\n")
    print("| kernel | dispatches | mean us | min us | max us | total ms | % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for name, n, avg, mn, mx, s in rows:
        print(f"| {name[:60]} | {n} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
              f"{s / 1e6:.3f} | {100 * s / tot:.1f} |")


def cmd_traffic(args):
    fetch = counter_means(args.fetch_db, "FETCH_SIZE")
    write = counter_means(args.write_db, "WRITE_SIZE")
    ff, fw = copy_factor(fetch), copy_factor(write)
    kern = {}
    for k in sorted(set(fetch) & set(write)):
        if "rocclr" in k or "at::native" in k:
            continue
        fb = fetch[k][1] * 1024.0 * ff
        wb = write[k][1] * 1024.0 * fw
        kern[k] = {"dispatches": fetch[k][0], "fetch_kib_raw": round(fetch[k][1], 1),
                   "write_kib_raw": round(write[k][1], 1), "hbm_bytes_per_launch": round(fb + wb)}
    print(f"# HBM traffic per dispatch: {args.title}\n")
    print("Commands (one counter per run, each with the 1 GiB calibration copy):\n")
    for c in args.command:
        print(f"    {c}")
    print(f"\nCalibration: the 1 GiB device copy reads {COPY_BYTES / ff / 1024:.1f} KiB of "
          f"FETCH_SIZE (factor {ff:.4f}) and {COPY_BYTES / fw / 1024:.1f} KiB of WRITE_SIZE "
          f"(factor {fw:.4f}).  Traffic = FETCH_SIZE x {ff:.4f} + WRITE_SIZE x {fw:.4f}.\n")
    print("| kernel | dispatches | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | HBM MB / launch |")
    print("|---|---:|---:|---:|---:|")
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"]):
        print(f"| {k} | {v['dispatches']} | {v['fetch_kib_raw']} | {v['write_kib_raw']} | "
              f"{v['hbm_bytes_per_launch'] / 1e6:.1f} |")
    data = {"source_sha256": source_hashes(), "fetch_factor": ff, "write_factor": fw,
            "kernels": {k: {"hbm_bytes_per_launch": v["hbm_bytes_per_launch"]} for k, v in kern.items()}}
    print("\n```json\n" + json.dumps(data, indent=1) + "\n```")


def cmd_issue(args):
    cur = sqlite3.connect(args.db).cursor()
    q = ("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
         "group by kernel_name, counter_name")
    per = {}
    for k, c, v, n in cur.execute(q).fetchall():
        per.setdefault(_short(k), {})[c] = (v, n)
    dur = {r[0]: r[2] for r in kernel_rows(args.trace_db)}  # mean ns
    print(f"# Instruction issue per wavefront: {args.title}\n")
    print("Commands (counters, then the kernel trace whose mean durations are used):\n")
    for c in args.command:
        print(f"    {c}")
    print(f"\nVALU issue share = VALU instructions x {CYCLES_PER_VALU} cycles / ({SIMDS} SIMDs x "
          f"{CLOCK_HZ / 1e9:.1f} GHz x mean duration).\n")
    print("| kernel | dispatches | waves | VALU / wave | SALU / wave | VMEM rd / wave | LDS / wave "
          "| mean us | VALU issue share |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|")
    data = {}
    for k in sorted(per, key=lambda k: -per[k].get("SQ_INSTS_VALU", (0, 0))[0]):
        d = per[k]
        if "SQ_WAVES" not in d or "SQ_INSTS_VALU" not in d or "rocclr" in k or "at::native" in k:
            continue
        waves = d["SQ_WAVES"][0]
        if waves <= 0:
            continue
        pw = {c: d[c][0] / waves for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD",
                                           "SQ_INSTS_LDS") if c in d}
        t = dur.get(k)
        share = (d["SQ_INSTS_VALU"][0] * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ * t * 1e-9)
                 if t else None)
        cell = lambda c: f"{pw[c]:.0f}" if c in pw else "-"
        print(f"| {k} | {d['SQ_WAVES'][1]} | {waves:.0f} | {cell('SQ_INSTS_VALU')} | "
              f"{cell('SQ_INSTS_SALU')} | {cell('SQ_INSTS_VMEM_RD')} | {cell('SQ_INSTS_LDS')} | "
              f"{'-' if t is None else f'{t / 1e3:.2f}'} | {'-' if share is None else f'{share:.2f}'} |")
        data[k] = {"valu_per_wave": round(pw["SQ_INSTS_VALU"], 1),
                   "valu_issue_share": None if share is None else round(share, 3)}
    print("\n```json\n" + json.dumps({"source_sha256": source_hashes(), "kernels": data},
                                      indent=1) + "\n```")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("kernels")
    a.add_argument("db")
    a.add_argument("--command", required=True)
    a.add_argument("--title", default="")
    a.set_defaults(fn=cmd_kernels)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_db")
    b.add_argument("write_db")
    b.add_argument("--command", action="append", required=True)
    b.add_argument("--title", default="")
    b.set_defaults(fn=cmd_traffic)
    c = sub.add_parser("issue")
    c.add_argument("db")
    c.add_argument("trace_db")
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--title", default="")
    c.set_defaults(fn=cmd_issue)
    args = ap.parse_args(argv)
    args.fn(args)


if __name__ == "__main__":
    main(sys.argv[1:])
