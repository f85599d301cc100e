"""Summaries of rocprofv3 results (rocpd SQLite databases) as short text.

    python -m paper_2507_15277_amd.profsum stats TRACE.db
    python -m paper_2507_15277_amd.profsum traffic --kernel NAME FETCH.db WRITE.db \\
           COPY_FETCH.db COPY_WRITE.db --copy-mib 1024

``stats`` lists per-kernel dispatch counts and durations from a
``--kernel-trace`` run.  ``traffic`` averages FETCH_SIZE and WRITE_SIZE
(KiB per dispatch) over the named kernel's dispatches and scales each by the
factor that makes the same counter read the true byte count of a plain
device copy of known size (one copy dispatch reads and writes --copy-mib MiB).
"""
from __future__ import annotations

import argparse
import sqlite3
import sys


def kernel_stats(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                       "max(duration) from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1.0
    return [{"name": r[0], "calls": r[1], "total_us": r[2] / 1e3, "avg_us": r[3] / 1e3,
             "min_us": r[4] / 1e3, "max_us": r[5] / 1e3, "pct": 100.0 * r[2] / total} for r in rows]


def counter_avg(db, counter, kernel=None, name_like=None):
    con = sqlite3.connect(db)
    q = "select kernel_name, count(*), avg(value) from counters_collection where counter_name = ?"
    args = [counter]
    if kernel is not None:
        q += " and kernel_name = ?"
        args.append(kernel)
    if name_like is not None:
        q += " and kernel_name like ?"
        args.append(name_like)
    q += " group by kernel_name"
    return con.execute(q, args).fetchall()


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--top", type=int, default=20)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("copy_fetch_db")
    t.add_argument("copy_write_db")
    t.add_argument("--copy-mib", type=float, default=1024.0)
    t.add_argument("--copy-kernel-like", default="%copyBuffer%")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print("| kernel | calls | total us | avg us | min us | max us | % |")
        print("|---|---:|---:|---:|---:|---:|---:|")
        for r in kernel_stats(args.db)[:args.top]:
            print(f"| {r['name']} | {r['calls']} | {r['total_us']:.1f} | {r['avg_us']:.3f} | "
                  f"{r['min_us']:.3f} | {r['max_us']:.3f} | {r['pct']:.1f} |")
        return
    kib = args.copy_mib * 1024.0
    cf = counter_avg(args.copy_fetch_db, "FETCH_SIZE", name_like=args.copy_kernel_like)
    cw = counter_avg(args.copy_write_db, "WRITE_SIZE", name_like=args.copy_kernel_like)
    if not cf or not cw:
        sys.exit("copy kernel not found in the calibration runs")
    f_fetch = kib / cf[0][2]
    f_write = kib / cw[0][2]
    kf = counter_avg(args.fetch_db, "FETCH_SIZE", kernel=args.kernel)
    kw = counter_avg(args.write_db, "WRITE_SIZE", kernel=args.kernel)
    if not kf or not kw:
        sys.exit(f"kernel {args.kernel} not found")
    fetch_b = kf[0][2] * 1024.0 * f_fetch
    write_b = kw[0][2] * 1024.0 * f_write
    print(f"copy calibration: FETCH_SIZE {cf[0][2]:.1f} KiB and WRITE_SIZE {cw[0][2]:.1f} KiB per "
          f"{args.copy_mib:.0f} MiB copy -> factors fetch {f_fetch:.4f}, write {f_write:.4f}")
    print(f"kernel {args.kernel}: {kf[0][1]} dispatches; FETCH_SIZE {kf[0][2]:.1f} KiB, "
          f"WRITE_SIZE {kw[0][2]:.1f} KiB per dispatch")
    print(f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}")
    print(f"fetch_bytes_per_launch: {fetch_b:.0f}")
    print(f"write_bytes_per_launch: {write_b:.0f}")


if __name__ == "__main__":
    main()
