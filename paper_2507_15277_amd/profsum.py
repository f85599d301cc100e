"""Summaries of rocprofv3 results (rocpd SQLite databases) as short text.

    python -m paper_2507_15277_amd.profsum stats TRACE.db
    python -m paper_2507_15277_amd.profsum traffic --kernel NAME FETCH.db WRITE.db \\
           COPY_FETCH.db COPY_WRITE.db --copy-mib 1024
    python -m paper_2507_15277_amd.profsum mfma PASS1.db PASS2.db TRACE.db NAME:M:N:K:REPS ...

``stats`` lists per-kernel dispatch counts and durations from a
``--kernel-trace`` run.  ``traffic`` averages FETCH_SIZE and WRITE_SIZE
(KiB per dispatch) over the named kernel's dispatches and scales each by the
factor that makes the same counter read the true byte count of a plain
device copy of known size (one copy dispatch reads and writes --copy-mib MiB).
``mfma`` combines two SQ counter passes and a kernel trace of the same
``kernel_drive`` launches into per-launch MFMA utilisation, effective clock
and wait shares.
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


def _dispatch_counters(db, prefix):
    """{dispatch_id: (kernel, {counter: value})} for kernels whose name starts with prefix."""
    con = sqlite3.connect(db)
    out = {}
    for did, name, cname, val in con.execute(
            "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
        if name.startswith(prefix):
            out.setdefault(did, (name, {}))[1][cname] = val
    return out


def _dispatch_durations(db, prefix):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    return [(n, d / 1e3) for n, d in rows if n.startswith(prefix)]


def mfma_table(pass1, pass2, trace, launches, ses=32, simds=1024, peak_ghz=2.4):
    """Per kernel_drive argument NAME:M:N:K:REPS (one warm-up launch, then
    REPS timed ones, in order): counters averaged over the timed launches."""
    c1, c2 = _dispatch_counters(pass1, "sgemm"), _dispatch_counters(pass2, "sgemm")
    d1, d2 = [c1[k] for k in sorted(c1)], [c2[k] for k in sorted(c2)]
    tr = _dispatch_durations(trace, "sgemm")
    rows, pos = [], 0
    for arg in launches:
        name, M, N, K, reps = arg.split(":")
        M, N, K, reps = int(M), int(N), int(K), int(reps)
        idx = range(pos + 1, pos + 1 + reps)
        pos += 1 + reps
        assert all(d1[i][0] == name and d2[i][0] == name and tr[i][0] == name for i in idx), arg
        avg = lambda d, c: sum(d[i][1][c] for i in idx) / reps  # noqa: E731
        dur = sum(tr[i][1] for i in idx) / reps
        busy = avg(d1, "SQ_BUSY_CYCLES") / ses
        mfma = avg(d1, "SQ_VALU_MFMA_BUSY_CYCLES") / simds
        wave = avg(d1, "SQ_WAVE_CYCLES")
        rows.append({"kernel": name, "shape": f"{M}x{N}x{K}", "duration_us": dur,
                     "tflops": 2.0 * M * N * K / dur / 1e6,
                     "clock_ghz": busy / dur / 1e3, "mfma_busy": mfma / busy,
                     "mfma_at_peak_clock": mfma / (dur * peak_ghz * 1e3),
                     "issue_wait": avg(d2, "SQ_WAIT_INST_ANY") / wave, "any_wait": avg(d2, "SQ_WAIT_ANY") / wave,
                     "lds_bank_conflicts": avg(d1, "SQ_LDS_BANK_CONFLICT"),
                     "check": mfma / (2.0 * M * N * K / simds / 64.0)})
    return rows


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
    m = sub.add_parser("mfma")
    m.add_argument("pass1_db")
    m.add_argument("pass2_db")
    m.add_argument("trace_db")
    m.add_argument("launches", nargs="+", help="the kernel_drive arguments of the three runs")
    args = ap.parse_args(argv)
    if args.cmd == "mfma":
        print("| kernel | shape | duration us | TFLOP/s | clock GHz | MFMA busy / busy cycles | at 2.4 GHz | "
              "issue-wait / wave cycles | any-wait / wave cycles | LDS bank conflicts | check |")
        print("|---|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
        for r in mfma_table(args.pass1_db, args.pass2_db, args.trace_db, args.launches):
            print(f"| {r['kernel']} | {r['shape']} | {r['duration_us']:.1f} | {r['tflops']:.1f} | {r['clock_ghz']:.2f} | "
                  f"{r['mfma_busy']:.2f} | {r['mfma_at_peak_clock']:.2f} | {r['issue_wait']:.2f} | "
                  f"{r['any_wait']:.2f} | {r['lds_bank_conflicts']:.0f} | {r['check']:.2f} |")
        return
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
