"""Text summaries of rocprofv3 CSV output, for the ``profiles/`` folder.

Kernel time (from ``--kernel-trace --stats --output-format csv``)::

    python -m paper_2603_11531_amd.profsum stats <dir>/<name>_kernel_stats.csv --cmd "<command>"

Hardware byte counters of one kernel (two ``--pmc`` runs, FETCH_SIZE then WRITE_SIZE,
optionally a third with SQ_* counters), scaled by what the same counters read for the
plain device-to-device copy of known size that ``bench.py --calib-copy-mib`` runs first::

    python -m paper_2603_11531_amd.profsum pmc --fetch <f>/p_counter_collection.csv \
        --write <w>/p_counter_collection.csv [--sq <s>/p_counter_collection.csv] \
        --kernel "split_plan_ordered_kernel;blend_range_kernel;merge_ranges_kernel" --calib-mib 1024 \
        --cmd "<command>"

The pmc summary records a hash of the kernel's sources; ``bench.py`` reports the
measured traffic only while the sources still hash the same.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import sys
from collections import OrderedDict

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")

# sources each profiled kernel group is built from (a summary is valid while they hash the same)
SOURCES = {
    "blend": ("blend.hip", "blend_math.h", "index_math.h", "batch.h", "common.h"),
    "enhance_project": ("project.hip", "proj_math.h", "mlp_math.h", "common.h"),
    "bin": ("bin.hip", "index_math.h", "batch.h", "common.h"),
}
BLEND_SOURCES = SOURCES["blend"]


def source_hash(files=BLEND_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _short(name, n=72):
    return name if len(name) <= n else name[:n - 3] + "..."


def stats(path, cmd, top=24):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"command: {cmd}", "", f"{'kernel':72s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'%':>6s}"]
    for r in rows[:top]:
        out.append(f"{_short(r['Name']):72s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                   f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):6.2f}")
    return "\n".join(out) + "\n"


def _counters(path):
    """{(kernel, counter): [values per dispatch]} from a counter_collection.csv."""
    agg = OrderedDict()
    for r in csv.DictReader(open(path)):
        agg.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    return agg


def _pick(agg, kernel_substr, counter):
    vals = [v for (k, c), vs in agg.items() if kernel_substr in k and c == counter for v in vs]
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {kernel_substr!r} with counter {counter}")
    return vals


def pmc(fetch_csv, write_csv, sq_csv, kernels, calib_mib, cmd, group="blend"):
    """kernels: the kernels one launch of the measured entry point runs (name substrings);
    their per-dispatch means are summed.  sq_csv: one counter CSV or a list of them."""
    fa, wa = _counters(fetch_csv), _counters(write_csv)
    calib_kib = calib_mib * 1024.0
    # the calibration copy is the largest copy dispatch of the run
    cf = max(_pick(fa, "copyBuffer", "FETCH_SIZE"))
    cw = max(_pick(wa, "copyBuffer", "WRITE_SIZE"))
    kf = calib_kib / cf
    kw = calib_kib / cw
    out = [f"command (one run per counter group): {cmd}",
           f"kernels: {', '.join(kernels)}",
           f"source_sha256: {source_hash(SOURCES[group])}",
           f"calibration copy: {calib_mib:g} MiB read + {calib_mib:g} MiB written; FETCH_SIZE read {cf:.1f} KiB, "
           f"WRITE_SIZE read {cw:.1f} KiB -> scale factors fetch {kf:.4f}, write {kw:.4f}"]
    total = 0.0
    for kernel in kernels:
        f = _pick(fa, kernel, "FETCH_SIZE")
        w = _pick(wa, kernel, "WRITE_SIZE")
        fm, wm = sum(f) / len(f), sum(w) / len(w)
        total += (fm * kf + wm * kw) * 1024.0
        out += [f"{kernel}: dispatches {len(f)} (FETCH run), {len(w)} (WRITE run)",
                f"  FETCH_SIZE per dispatch: mean {fm:.1f} KiB (min {min(f):.1f}, max {max(f):.1f}); "
                f"scaled {fm * kf / 1024:.1f} MiB",
                f"  WRITE_SIZE per dispatch: mean {wm:.1f} KiB (min {min(w):.1f}, max {max(w):.1f}); "
                f"scaled {wm * kw / 1024:.1f} MiB"]
    out.append(f"traffic_bytes_per_launch: {total:.0f}")
    if sq_csv:
        sa = OrderedDict()
        for path in ([sq_csv] if isinstance(sq_csv, str) else sq_csv):
            sa.update(_counters(path))
        out.append("")
        out.append("SQ / GRBM counters per dispatch (mean over dispatches; GRBM_GUI_ACTIVE summed over XCDs):")
        for kernel in kernels:
            for (k, c), vs in sa.items():
                if kernel in k:
                    out.append(f"  {kernel.replace(' ', ''):22s} {c:22s} {sum(vs) / len(vs):16.1f}")
    return "\n".join(out) + "\n"


def read_summary(path, files=BLEND_SOURCES):
    """(traffic_bytes_per_launch, {(kernel, counter): mean per dispatch}) of a pmc summary, or
    None if it is missing or the kernels' sources changed since the counters were taken."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    kv = dict(l.split(": ", 1) for l in lines if ": " in l and not l.startswith(" "))
    if kv.get("source_sha256") != source_hash(files):
        return None
    try:
        traffic = float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
    sq = {}
    for l in lines:
        f = l.split()
        if l.startswith("  ") and len(f) == 3 and f[1].isupper():
            try:
                sq[(f[0], f[1])] = float(f[2])
            except ValueError:
                pass
    return traffic, sq


def read_traffic(path, files=BLEND_SOURCES):
    """traffic_bytes_per_launch from a pmc summary, or None if it is missing or the kernel's
    sources changed since the counters were taken."""
    r = read_summary(path, files)
    return None if r is None else r[0]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--top", type=int, default=24, help="kernels listed, by total time")
    p = sub.add_parser("pmc")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--sq", default=None, help="comma-separated counter CSVs of SQ / GRBM passes")
    p.add_argument("--group", default="blend", choices=sorted(SOURCES))
    p.add_argument("--kernel", required=True, help="';'-separated kernel name substrings")
    p.add_argument("--calib-mib", type=float, required=True)
    p.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.mode == "stats":
        sys.stdout.write(stats(a.csv, a.cmd, a.top))
    else:
        sys.stdout.write(pmc(a.fetch, a.write, a.sq.split(",") if a.sq else None, a.kernel.split(";"), a.calib_mib,
                             a.cmd, a.group))


if __name__ == "__main__":
    main()
