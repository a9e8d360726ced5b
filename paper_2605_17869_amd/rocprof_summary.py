"""Summaries of rocprofv3 result databases (SQLite) as short text.

    python -m paper_2605_17869_amd.rocprof_summary trace DB [--group PREFIX ...]
    python -m paper_2605_17869_amd.rocprof_summary dispatches DB FIRST COUNT
    python -m paper_2605_17869_amd.rocprof_summary counters DB COUNTER [--group PREFIX ...]
    python -m paper_2605_17869_amd.rocprof_summary calibrate DB COUNTER KERNEL BYTES_PER_DISPATCH
    python -m paper_2605_17869_amd.rocprof_summary traffic FETCH_DB WRITE_DB CAL_FETCH_DB \
        CAL_WRITE_DB CAL_KERNEL CAL_BYTES PREFIX

``trace`` prints per-kernel calls, total and average duration (from a
``--kernel-trace`` run); ``dispatches`` lists COUNT consecutive dispatches
from the FIRST-th (0-based, in start order) with duration, grid, register
and LDS use, e.g. one launch sequence of a batch; ``counters`` prints the per-dispatch average of one
counter per kernel (from a ``--pmc`` run); ``calibrate`` prints the ratio of a
known per-dispatch byte count to what the counter reports for a plain copy
kernel.  ``traffic`` turns FETCH_SIZE and WRITE_SIZE of the kernels whose
name starts with PREFIX into HBM bytes per launch, each counter scaled by
CAL_BYTES over what it reports per dispatch of the calibration kernel (the
first kernel whose name contains CAL_KERNEL), and prints the digest of the
blur kernel's sources the figure holds for.  ``--group`` sums kernels whose
demangled name starts with PREFIX.
"""
from __future__ import annotations

import argparse
import sqlite3
from collections import OrderedDict


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def kernel_times(db: str) -> "OrderedDict[str, tuple]":
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average from top_kernels").fetchall()
    return OrderedDict((_short(r[0]), (int(r[1]), float(r[2]), float(r[3]))) for r in rows)


def counter_values(db: str, counter: str) -> "OrderedDict[str, tuple]":
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, count(*), sum(value) from counters_collection "
        "where counter_name = ? group by kernel_name order by sum(value) desc", (counter,)).fetchall()
    return OrderedDict((_short(r[0]), (int(r[1]), float(r[2]))) for r in rows)


def grouped(items: "OrderedDict", groups) -> "OrderedDict":
    out: "OrderedDict" = OrderedDict()
    for name, vals in items.items():
        key = next((g + "*" for g in groups if name.startswith(g)), name)
        if key in out:
            out[key] = tuple(a + b for a, b in zip(out[key], vals))
        else:
            out[key] = vals
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "dispatches", "counters", "calibrate", "traffic"])
    ap.add_argument("db")
    ap.add_argument("rest", nargs="*")
    ap.add_argument("--group", action="append", default=[])
    a = ap.parse_args(argv)
    if a.mode == "trace":
        t = kernel_times(a.db)
        total = sum(v[1] for v in t.values())
        rows = [(k, v[0], v[1]) for k, v in t.items()]
        if a.group:
            g = grouped(OrderedDict((k, (c, d)) for k, c, d in rows), a.group)
            rows = [(k, v[0], v[1]) for k, v in g.items()]
        rows.sort(key=lambda r: -r[2])
        print(f"{'kernel':60s} {'calls':>6s} {'total_us':>12s} {'avg_us':>10s} {'pct':>6s}")
        for k, c, d in rows:
            print(f"{k[:60]:60s} {c:6d} {d:12.1f} {d / c:10.2f} {100 * d / total:6.2f}")
    elif a.mode == "dispatches":
        first, count = int(a.rest[0]), int(a.rest[1])
        con = sqlite3.connect(a.db)
        rows = con.execute(
            "select name, duration, grid_x, workgroup_x, vgpr_count, accum_vgpr_count, lds_size "
            "from kernels order by start limit ? offset ?", (count, first)).fetchall()
        print(f"{'kernel':44s} {'us':>9s} {'groups':>8s} {'wg':>4s} {'vgpr':>5s} {'agpr':>5s} {'lds':>6s}")
        for name, dur, gx, wx, vg, ag, lds in rows:
            groups = gx // max(wx, 1)
            print(f"{_short(name)[:44]:44s} {dur / 1000.0:9.1f} {groups:8d} {wx:4d} {vg:5d} {ag:5d} {lds:6d}")
    elif a.mode == "counters":
        counter = a.rest[0]
        v = counter_values(a.db, counter)
        if a.group:
            v = grouped(v, a.group)
        print(f"{'kernel':60s} {'dispatches':>10s} {counter + '_KiB_per_dispatch':>28s}")
        for k, (n, s) in v.items():
            print(f"{k[:60]:60s} {n:10d} {s / n:28.1f}")
    elif a.mode == "traffic":
        fetch_db, write_db, cal_fetch, cal_write, cal_kernel = a.db, *a.rest[:4]
        cal_bytes, prefix = float(a.rest[4]), a.rest[5]
        out = {}
        for counter, db, cal in (("FETCH_SIZE", fetch_db, cal_fetch), ("WRITE_SIZE", write_db, cal_write)):
            cv = counter_values(cal, counter)
            name = next(k for k in cv if cal_kernel in k)
            cn, cs = cv[name]
            scale = cal_bytes / (cs / cn * 1024.0)
            prefixes = tuple(prefix.split(","))
            kv = [(n, s_) for k, (n, s_) in counter_values(db, counter).items() if k.startswith(prefixes)]
            launches = sum(n for n, _ in kv)
            raw = sum(s_ for _, s_ in kv) / launches * 1024.0
            out[counter] = raw * scale
            print(f"{counter}: {raw:.0f} bytes/launch reported over {launches} launches of {prefix}*; "
                  f"calibration {name[:40]}: {cs / cn * 1024.0:.0f} reported for {cal_bytes:.0f}, "
                  f"scale {scale:.4f}; scaled {raw * scale:.0f} bytes/launch")
        from paper_2605_17869_amd.build import kernel_source_hash
        print(f"hbm_bytes_per_launch: {int(round(out['FETCH_SIZE'] + out['WRITE_SIZE']))}")
        print(f"kernel_source_sha256: {kernel_source_hash()}")
    else:
        counter, kernel, expected = a.rest[0], a.rest[1], float(a.rest[2])
        v = counter_values(a.db, counter)
        n, s = v[kernel]
        per = s / n * 1024.0
        print(f"kernel {kernel}: {counter} {per:.0f} bytes/dispatch over {n} dispatches, "
              f"expected {expected:.0f}; scale {expected / per:.4f}")


if __name__ == "__main__":
    main()
