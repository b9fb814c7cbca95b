"""Turn rocprofv3 CSV output into the short text summaries kept under profiles/.

Usage (each reads the directory rocprofv3 wrote with ``-d DIR --output-format csv``):

  python -m paper_2105_09671_amd.rocprof_summary trace DIR OUT.txt --command "..."
      kernel table from *_kernel_stats.csv (calls, total, mean, min, max).

  python -m paper_2105_09671_amd.rocprof_summary counters OUT.txt DIR [DIR ...] --kernel NAME ...
      mean per dispatch of every counter of each matching kernel (several
      --pmc runs, one directory each), with per-wave instruction counts.

  python -m paper_2105_09671_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR OUT.txt \\
      --kernel tile2d_kernel --copy-bytes 268435456 --alg-bytes N --src FILE --json OUT.json
      HBM bytes per dispatch of the kernel from FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch).  Each counter is scaled by (copy bytes / counter reading) of the
      largest __amd_rocclr_copyBuffer dispatch in the same run, a device-to-device
      copy of known size.  The JSON records the kernel source's sha256 so a later
      change of the kernel invalidates the figure.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[0]


def _short(name: str, n: int = 70) -> str:
    name = name.replace("void ", "").replace("(anonymous namespace)::", "")
    cut = name.find("(")
    if cut > 0:
        name = name[:cut]
    return name if len(name) <= n else name[: n - 3] + "..."


def trace(d: str, out: str, command: str) -> None:
    rows = list(csv.DictReader(open(_find(d, "_kernel_stats.csv"))))
    lines = ["# rocprofv3 --kernel-trace --stats", "# command: " + command, "",
             "%-72s %8s %12s %11s %11s %11s %7s" % ("kernel", "calls", "total_ms", "mean_us",
                                                    "min_us", "max_us", "pct")]
    for r in rows:
        lines.append("%-72s %8d %12.3f %11.3f %11.3f %11.3f %7.2f" % (
            _short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(d: str, kernel: str):
    rows = list(csv.DictReader(open(_find(d, "_counter_collection.csv"))))
    ker = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]]
    copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    name = rows[0]["Counter_Name"] if rows else "?"
    return name, ker, copies


def sources_sha256(paths) -> str:
    """sha256 over the concatenated bytes of the given source files, in order."""
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic(fetch_dir, write_dir, out, kernel, copy_bytes, alg_bytes, src, out_json, command):
    res = {}
    lines = ["# HBM traffic per dispatch of %s from rocprofv3 --pmc" % kernel,
             "# command: " + command, ""]
    total = 0.0
    for d in (fetch_dir, write_dir):
        name, ker, copies = _counter(d, kernel)
        ref = max(copies)                           # the copy of known size, in KiB
        scale = copy_bytes / (ref * 1024.0)
        mean_kib = statistics.mean(ker)
        b = mean_kib * 1024.0 * scale
        total += b
        res[name] = {"dispatches": len(ker), "mean_kib": mean_kib, "copy_ref_kib": ref,
                     "scale": scale, "bytes_per_dispatch": b}
        lines.append("%-10s dispatches %6d  mean %12.1f KiB  copy ref %12.1f KiB for %d B "
                     "-> scale %.4f  -> %.1f MiB/dispatch" % (name, len(ker), mean_kib, ref,
                                                             copy_bytes, scale, b / 2 ** 20))
    lines.append("HBM bytes per dispatch (scaled FETCH + WRITE): %.1f MiB" % (total / 2 ** 20))
    if alg_bytes:
        lines.append("algorithmic bytes per dispatch: %.1f MiB  (measured / algorithmic = %.3f)"
                     % (alg_bytes / 2 ** 20, total / alg_bytes))
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))
    if out_json:
        sha = sources_sha256(src.split(",")) if src else None
        json.dump({"kernel": kernel, "counters": res, "hbm_bytes_per_launch": int(total),
                   "algorithmic_bytes_per_launch": alg_bytes, "src": ",".join(os.path.basename(x) for x in src.split(",")) if src else "",
                   "src_sha256": sha, "command": command}, open(out_json, "w"), indent=1)


def counters(dirs, out: str, kernels, command: str, fetch_scale: float = 2.0,
             write_scale: float = 1.0) -> None:
    """Mean value per dispatch of every counter collected in the given runs,
    for each kernel whose name contains one of `kernels`, plus derived ratios
    when their inputs are present."""
    per = {}          # kernel -> counter -> [values]
    for d in dirs:
        for r in csv.DictReader(open(_find(d, "_counter_collection.csv"))):
            name = r["Kernel_Name"]
            k = next((k for k in kernels if k in name), None)
            if k is None:
                continue
            per.setdefault(_short(name, 60), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
    lines = ["# rocprofv3 --pmc, mean per dispatch", "# command: " + command, ""]
    for kname in sorted(per):
        c = {n: statistics.mean(v) for n, v in per[kname].items()}
        n_disp = max(len(v) for v in per[kname].values())
        lines.append("%s  (%d dispatches)" % (kname, n_disp))
        for n in sorted(c):
            lines.append("    %-28s %16.1f" % (n, c[n]))
        waves = c.get("SQ_WAVES")
        if waves:
            for n in ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM"):
                if n in c:
                    lines.append("    %-28s %16.2f" % (n + " per wave", c[n] / waves))
        if "FETCH_SIZE" in c and "WRITE_SIZE" in c:
            # KiB per dispatch, scaled as the copy reference of the traffic
            # records reads (FETCH_SIZE counts half of a copy's bytes)
            hb = (c["FETCH_SIZE"] * fetch_scale + c["WRITE_SIZE"] * write_scale) * 1024.0
            lines.append("    %-28s %16.1f" % ("HBM MiB (F x%.1f + W x%.1f)" % (fetch_scale, write_scale),
                                               hb / 2 ** 20))
        if c.get("SQ_WAVE_CYCLES") and "SQ_WAIT_INST_ANY" in c:
            lines.append("    %-28s %16.4f" % ("wait-any / wave cycles", c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"]))
        if c.get("SQ_WAVE_CYCLES") and "SQ_ACTIVE_INST_VALU" in c:
            lines.append("    %-28s %16.4f" % ("VALU active / wave cycles", c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"]))
        if c.get("SQ_INSTS_LDS") and "SQ_LDS_BANK_CONFLICT" in c and c.get("SQ_LDS_IDX_ACTIVE"):
            lines.append("    %-28s %16.4f" % ("LDS bank-conflict / active", c["SQ_LDS_BANK_CONFLICT"] / c["SQ_LDS_IDX_ACTIVE"]))
        lines.append("")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("out")
    t.add_argument("--command", default="")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_dir")
    f.add_argument("write_dir")
    f.add_argument("out")
    f.add_argument("--kernel", required=True)
    f.add_argument("--copy-bytes", type=int, default=256 * 2 ** 20)
    f.add_argument("--alg-bytes", type=int, default=0)
    f.add_argument("--src", default="", help="comma-separated kernel source files")
    f.add_argument("--json", default="")
    f.add_argument("--command", default="")
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--command", default="")
    a = ap.parse_args()
    if a.cmd == "counters":
        counters(a.dirs, a.out, a.kernel, a.command)
        return
    if a.cmd == "trace":
        trace(a.dir, a.out, a.command)
    else:
        traffic(a.fetch_dir, a.write_dir, a.out, a.kernel, a.copy_bytes, a.alg_bytes, a.src,
                a.json, a.command)


if __name__ == "__main__":
    main()
