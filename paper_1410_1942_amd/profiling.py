"""Summaries of rocprofv3 output (kernel trace statistics and PMC counters).

Reads the CSV files rocprofv3 writes (--output-format csv) and prints short
text summaries: per-kernel launch counts and durations, and per-kernel HBM
bytes from the FETCH_SIZE / WRITE_SIZE counters, calibrated against the plain
copy kernel of known size that the same run launches.

    python -m paper_1410_1942_amd.profiling stats <kernel_stats.csv | kernel_trace.csv>
        [--match S --gap-ms G --segment N]
    python -m paper_1410_1942_amd.profiling counters <counter_collection.csv>... --match S
    python -m paper_1410_1942_amd.profiling traffic <fetch counter_collection.csv>
        <write counter_collection.csv> --cells N --copy-bytes B [--sha S]
"""
from __future__ import annotations

import argparse
import collections
import csv
import statistics
import sys


def _short(name: str, width: int = 70) -> str:
    return name if len(name) <= width else name[: width - 3] + "..."


def _segment(rows, match: str, gap_ms: float, segment: int):
    """The launches whose kernel name contains `match`, in start order, cut
    where the device ran none of them for more than gap_ms; the segment-th
    run of launches (0 = the first)."""
    rows = sorted((r for r in rows if match in r["Kernel_Name"]),
                  key=lambda r: int(r["Start_Timestamp"]))
    runs, cur, last_end = [], [], None
    for r in rows:
        s, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if last_end is not None and s - last_end > gap_ms * 1e6:
            runs.append(cur)
            cur = []
        cur.append(r)
        last_end = e if last_end is None else max(last_end, e)
    if cur:
        runs.append(cur)
    if not 0 <= segment < len(runs):
        raise SystemExit(f"{len(runs)} runs of launches, no run {segment}")
    return runs[segment]


def kernel_stats(path: str, match: str = "", gap_ms: float = 0.0, segment: int = -1) -> str:
    rows = list(csv.DictReader(open(path)))
    out = []
    if segment >= 0:
        rows = _segment(rows, match, gap_ms, segment)
        span = int(rows[-1]["End_Timestamp"]) - int(rows[0]["Start_Timestamp"])
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows)
        out.append(f"# run {segment} of the launches matching '{match}' (cut at idle gaps over "
                   f"{gap_ms} ms): {len(rows)} launches over {span / 1e6:.2f} ms, "
                   f"busy {busy / 1e6:.2f} ms ({busy / span:.0%})")
    if rows and "TotalDurationNs" in rows[0]:          # *_kernel_stats.csv
        out.append(f"{'kernel':70s} {'calls':>7s} {'avg_ms':>10s} {'min_ms':>10s} "
                   f"{'max_ms':>10s} {'total_s':>9s} {'pct':>6s}")
        for r in rows:
            out.append(f"{_short(r['Name']):70s} {int(r['Calls']):7d} "
                       f"{float(r['AverageNs'])/1e6:10.4f} {float(r['MinNs'])/1e6:10.4f} "
                       f"{float(r['MaxNs'])/1e6:10.4f} {float(r['TotalDurationNs'])/1e9:9.3f} "
                       f"{float(r['Percentage']):6.2f}")
        return "\n".join(out)
    # *_kernel_trace.csv: aggregate ourselves; `large` averages the typical
    # launches of the problem launched most (see _large)
    agg = collections.defaultdict(list)
    for r in rows:
        agg[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out.append(f"{'kernel':70s} {'calls':>7s} {'avg_ms':>10s} {'median_ms':>10s} "
               f"{'large_n':>8s} {'large_avg_ms':>12s} {'short_n':>8s} {'short_ms':>9s} "
               f"{'long_n':>7s} {'long_ms':>8s} {'total_s':>9s}")
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        big = _large(v)
        (sn, sm), (ln, lm) = _two_forms(big)
        out.append(f"{_short(k):70s} {len(v):7d} {statistics.mean(v)/1e6:10.4f} "
                   f"{statistics.median(v)/1e6:10.4f} {len(big):8d} "
                   f"{statistics.mean(big)/1e6:12.4f} {sn:8d} {sm/1e6:9.4f} "
                   f"{ln:7d} {lm/1e6:8.4f} {sum(v)/1e9:9.3f}")
    return "\n".join(out)


def _two_forms(values):
    """Count and mean of the two groups that a cut of the sorted values
    leaves with the least summed squared deviation (two-means in one
    dimension): the two forms of the iteration (without and with the x
    update), which a handful of much longer set-up launches cannot pull
    apart as they would a cut at the midpoint of the range."""
    v = sorted(values)
    n = len(v)
    if n < 2:
        return (n, statistics.mean(v)), (n, statistics.mean(v))
    pre = [0.0]
    pre2 = [0.0]
    for x in v:
        pre.append(pre[-1] + x)
        pre2.append(pre2[-1] + x * x)

    def sse(a, b):
        m = b - a
        s = pre[b] - pre[a]
        return pre2[b] - pre2[a] - s * s / m

    cut = min(range(1, n), key=lambda c: sse(0, c) + sse(c, n))
    a, b = v[:cut], v[cut:]
    return (len(a), statistics.mean(a)), (len(b), statistics.mean(b))


def _large(values, lo=0.5, hi=3.0):
    """The values within [lo, hi] times the median of the non-empty ones
    (above a hundredth of the largest): the launches of the problem a run
    launches most, every form of a kernel whose launches alternate (the
    iteration with and without the x update, within a factor of about 2.3
    of each other); not the empty launches at the end of a captured chunk,
    however many, those of much smaller problems, nor the rare set-up and
    residual launches."""
    top = max(values)
    busy = [v for v in values if v > 0.01 * top] or values
    med = statistics.median(busy)
    return [v for v in values if lo * med <= v <= hi * med]


def _counter(path: str):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def traffic(fetch_csv: str, write_csv: str, cells: int, copy_bytes: int,
            sha: str = "") -> str:
    """HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by (true bytes / counted bytes) of the copy kernel, which
    reads and writes copy_bytes per launch."""
    f, w = _counter(fetch_csv), _counter(write_csv)
    copy = [k for k in f if "k_copy" in k]
    if not copy:
        raise SystemExit("no copy kernel in the fetch run")
    f_copy = statistics.median(f[copy[0]]) * 1024
    w_copy = statistics.median(w[copy[0]]) * 1024
    sf, sw = copy_bytes / f_copy, copy_bytes / w_copy
    lines = [f"# FETCH_SIZE scale {sf:.4f}, WRITE_SIZE scale {sw:.4f} "
             f"(copy kernel: {copy_bytes} B read and written per launch)",
             f"# per launch, mean over the launches within half to three times the "
             f"median of the non-empty ones (empty launches at the end of a captured "
             f"chunk, however many, and the rare set-up launches excluded; both forms of "
             f"the iteration, with and without the x update, kept); cells = {cells}"]
    if sha:
        lines.append(f"kernel_source_sha = {sha}")
    lines.append(f"{'kernel':58s} {'n':>4s} {'fetch_B':>14s} {'write_B':>14s} "
                 f"{'fetch/cell':>10s} {'write/cell':>10s}")
    for k in f:
        if k not in w:
            continue
        fb = statistics.mean(_large(f[k])) * 1024 * sf
        wb = statistics.mean(_large(w[k])) * 1024 * sw
        lines.append(f"{_short(k, 58):58s} {len(f[k]):4d} {fb:14.4e} {wb:14.4e} "
                     f"{fb / cells:10.2f} {wb / cells:10.2f}")
        if "k_iter<" in k:
            tag = k[k.index("k_iter<"):k.index(">", k.index("k_iter<")) + 1]
            lines.append(f"bytes[{tag}] = {fb + wb:.6e}")
    return "\n".join(lines)


def counters(paths, match: str) -> str:
    """Per-counter means over the launches of the kernels whose name holds
    `match`, from one or more PMC runs (counter_collection CSVs), each
    counter over the launches within half to three times the median of its
    non-empty values (see _large)."""
    lines = [f"{'kernel':58s} {'counter':28s} {'n':>5s} {'mean':>14s}"]
    for path in paths:
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if match in r["Kernel_Name"]:
                agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
        for (k, c), v in sorted(agg.items()):
            big = _large(v) if max(v) > 0 else v
            lines.append(f"{_short(k, 58):58s} {c:28s} {len(big):5d} {statistics.mean(big):14.6e}")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--match", default="", help="kernel name substring (with --segment)")
    s.add_argument("--gap-ms", type=float, default=2.0,
                   help="idle time that separates runs of launches (with --segment)")
    s.add_argument("--segment", type=int, default=-1,
                   help="summarize only this run of matching launches (trace CSV)")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--match", required=True, help="kernel name substring")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--cells", type=int, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--sha", default="")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(kernel_stats(a.csv, a.match, a.gap_ms, a.segment))
    elif a.cmd == "counters":
        print(counters(a.csv, a.match))
    else:
        print(traffic(a.fetch_csv, a.write_csv, a.cells, a.copy_bytes, a.sha))


if __name__ == "__main__":
    sys.exit(main())
