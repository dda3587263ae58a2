"""Text summaries of rocprofv3 output databases (kernel timings and hardware counters).

    python -m paper_1507_07068_amd.profiling stats DIR          # per-kernel time table
    python -m paper_1507_07068_amd.profiling steps DIR          # per-step breakdown
    python -m paper_1507_07068_amd.profiling pmc DIR [DIR ...]  # counters per kernel

DIR is the output directory of ``rocprofv3 -d DIR -o run ...``; its SQLite database is
found recursively.  Only the standard library and numpy are used.
"""
from __future__ import annotations

import collections
import glob
import re
import sqlite3
import sys

import numpy as np


def _db(d: str) -> str:
    found = sorted(glob.glob(d + "/**/*.db", recursive=True))
    if not found:
        raise SystemExit(f"no rocprofv3 database under {d}")
    return found[-1]


def short_name(n: str) -> str:
    m = re.search(r"md::(k_\w+)(<[^>]*>)?", n)
    return (m.group(1) + (m.group(2) or "")) if m else n.split("(")[0][:48]


def stats(d: str) -> str:
    c = sqlite3.connect(_db(d))
    out = [f"{'kernel':44s} {'calls':>7s} {'total ms':>10s} {'avg us':>9s} {'share':>6s}"]
    for name, calls, total, avg, pct in c.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels limit 30"):
        # the summary table holds durations in microseconds
        out.append(f"{short_name(name):44s} {calls:7d} {total / 1e3:10.3f} {avg:9.2f} {pct:5.1f}%")
    return "\n".join(out)


def steps(d: str) -> str:
    """Kernel durations per step, split into steps with and without a list rebuild (Cr-Cr
    list kernel longer than 20 us).  A step starts at its first build kernel (k_decide, or
    k_bin when the binning blocks take the decision themselves) or at the k_kick_drift launch
    just before it; FP64 runs drift inside the force pass and launch k_kick_drift only after
    steps whose velocities are observed."""
    c = sqlite3.connect(_db(d))
    rows = list(c.execute("select name, start, end from kernels order by start"))
    groups, cur, prev = [], None, ""
    for n, s, e in rows:
        k = short_name(n)
        first_build = k.startswith("k_decide") or (k.startswith("k_bin") and not prev.startswith("k_decide"))
        if k.startswith("k_kick_drift") or (first_build and not prev.startswith("k_kick_drift")):
            cur = []
            groups.append(cur)
        if cur is not None:
            cur.append((k, s, e))
        prev = k
    groups = groups[5:-1]
    out = []
    split = {"rebuild": [], "no rebuild": []}
    for g in groups:
        dur = collections.defaultdict(float)
        for k, s, e in g:
            dur[k] += (e - s) / 1e3
        lst = sum(v for k, v in dur.items() if k.startswith(("k_list_tiles", "k_list_rows")))
        split["rebuild" if lst > 20.0 else "no rebuild"].append((dur, (g[-1][2] - g[0][1]) / 1e3))
    # the rebuilding steps' list-kernel time over the run, in quarters
    reb = [sum(v for k, v in dur.items() if k.startswith(("k_list_tiles", "k_list_rows")))
           for dur, _ in split["rebuild"]]
    if len(reb) >= 4:
        q = np.array_split(np.array(reb), 4)
        out.append("list kernel of rebuilding steps by quarter of the run: "
                   + ", ".join(f"{x.mean():.1f}" for x in q) + " us")
    for name, gs in split.items():
        if not gs:
            continue
        out.append(f"{name}: {len(gs)} steps, first-to-last kernel {np.mean([w for _, w in gs]):.1f} us/step")
        acc = collections.defaultdict(list)
        for dur, _ in gs:
            for k, v in dur.items():
                acc[k].append(v)
        for k, v in sorted(acc.items(), key=lambda kv: -np.mean(kv[1])):
            out.append(f"    {k:40s} {np.mean(v):8.2f} us")
    return "\n".join(out)


def pmc(dirs) -> str:
    """Counters per kernel: the mean over its dispatches, and the mean over its busy
    dispatches (those above the geometric mean of the smallest and largest reading; for the
    build kernels, which return at once in steps without a rebuild, these are the rebuilds)."""
    res = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    for d in dirs:
        c = sqlite3.connect(_db(d))
        cols = [r[1] for r in c.execute("pragma table_info(counters_collection)")]
        key = "dispatch_id" if "dispatch_id" in cols else "rowid"
        for kn, cn, val, did in c.execute(
                f"select kernel_name, counter_name, value, {key} from counters_collection"):
            res[kn][cn][(d, did)] += val
    out = []
    for kn in sorted(res):
        parts = [f"{short_name(kn):40s}"]
        for cn in sorted(res[kn]):
            v = np.array(list(res[kn][cn].values()))
            lo, hi = max(v.min(), 1e-9), max(v.max(), 1e-9)
            busy = v[v > np.sqrt(lo * hi)] if hi > 4 * lo else v
            parts.append(f"{cn}: mean {v.mean():.6g} busy {busy.mean():.6g} (n={v.size}, busy {busy.size})")
        out.append("  ".join(parts))
    return "\n".join(out)


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) < 2 or argv[0] not in ("stats", "steps", "pmc"):
        raise SystemExit(__doc__)
    if argv[0] == "stats":
        print(stats(argv[1]))
    elif argv[0] == "steps":
        print(steps(argv[1]))
    else:
        print(pmc(argv[1:]))


if __name__ == "__main__":
    main()
