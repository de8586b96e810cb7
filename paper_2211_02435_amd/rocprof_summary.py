"""Summaries of rocprofv3 output (rocpd SQLite databases) for the library's kernels.

  python -m paper_2211_02435_amd.rocprof_summary stats <run_results.db> [--match sweep_kernel]
      per-kernel calls, total and average duration (the --kernel-trace --stats view)

  python -m paper_2211_02435_amd.rocprof_summary traffic --fetch <db> --write <db>
      --kernel <substring> --copy-bytes <bytes> --workload <name> [--layout planes|rows] [--out <json>]
      HBM bytes per launch of the kernel from FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
      each scaled by what the same counter reads for the plain copy kernel of known size,
      together with the hash of the sources and build flags the counters were taken on.

  python -m paper_2211_02435_amd.rocprof_summary counters <db> [<db> ...] [--match sweep]
      median value per dispatch of every PMC counter in the databases, per kernel

  python -m paper_2211_02435_amd.rocprof_summary memory <db> [<db> ...] (--copy-bytes <bytes> | --scales F,W)
      the memory-interface view of every sweep and copy kernel from the passes FETCH_SIZE;
      WRITE_SIZE; TCC_EA0_{RD,WR}REQ{,_LEVEL}_sum with GRBM_GUI_ACTIVE;
      TCC_EA0_WRREQ_64B_sum, TCC_EA0_WRREQ_STALL_sum, TCC_EA0_{RD,WR}REQ_DRAM_CREDIT_STALL_sum
      with GRBM_GUI_ACTIVE: bytes moved, bytes per request, average request latency and
      requests in flight (Little's law: level / requests, level / cycles), stall fractions
"""
import argparse
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = "paper_2211_02435_amd/csrc"


def kernel_sources():
    """Every file that decides what the measured kernels do and how they are launched: the
    device code, the runtime (launch shapes, tile tables, LDS reserve), the instantiation
    units and the build script with its compiler flags."""
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(os.path.join(ROOT, CSRC))
                   if f.endswith((".hpp", ".hip", ".inc", ".cpp")))
    return files + ["paper_2211_02435_amd/build.py", "include/lbm.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in kernel_sources():
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_rows(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration, dispatch_id from kernels order by start").fetchall()
    con.close()
    return rows


def stats(db, match=None, last=None):
    """Per-kernel call count and total / average / min / max duration; with `last`, only the
    last `last` dispatches of every kernel (the timed region of a bench run that autotuned
    or warmed up first)."""
    per = {}
    for name, dur, _ in kernel_rows(db):
        if match and match not in name:
            continue
        per.setdefault(name, []).append(dur)
    agg = {}
    for name, durs in per.items():
        if last:
            durs = durs[-last:]
        agg[name] = [len(durs), float(sum(durs)), float(min(durs)), float(max(durs))]
    out = []
    for name, (n, tot, mn, mx) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append({"kernel": name, "calls": n, "total_us": tot / 1e3, "avg_us": tot / n / 1e3,
                    "min_us": mn / 1e3, "max_us": mx / 1e3})
    return out


def counter_per_dispatch(db, counter):
    """{kernel name: [value per dispatch]} for one PMC counter (summed over instances)."""
    con = sqlite3.connect(db)
    q = """select k.name, k.dispatch_id, sum(p.value) from pmc_events p
           join kernels k on p.event_id = k.id
           join pmc_info i on p.pmc_id = i.id
           where i.name = ? group by k.id order by k.start"""
    try:
        rows = con.execute(q, (counter,)).fetchall()
    except sqlite3.OperationalError:
        rows = []
    if not rows:  # fall back to the counters_collection view
        cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
        name_col = "kernel_name" if "kernel_name" in cols else "name"
        rows = con.execute("select %s, dispatch_id, sum(value) from counters_collection where counter_name = ? "
                           "group by dispatch_id order by dispatch_id" % name_col, (counter,)).fetchall()
    con.close()
    out = {}
    for name, _, v in rows:
        out.setdefault(name, []).append(float(v))
    return out


def all_counters(db):
    """{counter name: {kernel name: [value per dispatch]}} for every PMC counter in db."""
    con = sqlite3.connect(db)
    try:
        names = [r[0] for r in con.execute("select distinct name from pmc_info")]
    except sqlite3.OperationalError:
        names = [r[0] for r in con.execute("select distinct counter_name from counters_collection")]
    con.close()
    return {n: counter_per_dispatch(db, n) for n in names}


def counters_table(dbs, match=None):
    """Median per dispatch of every counter of every database, per kernel."""
    rows = {}
    for db in dbs:
        for name, per_kernel in all_counters(db).items():
            for k, vals in per_kernel.items():
                if match and match not in k:
                    continue
                vals = sorted(vals)
                rows.setdefault(k, {})[name] = vals[len(vals) // 2]
    return rows


XCDS = 8           # GRBM_GUI_ACTIVE is summed over the XCDs
TCC_CHANNELS = 128  # the _sum counters are summed over 16 L2 channels on each of the 8 XCDs


def memory_view(dbs, copy_bytes=None, clock_ghz=2.1, scales=None):
    """Derived memory-interface figures per kernel (see the module docstring).  FETCH_SIZE and
    WRITE_SIZE are scaled by the copy kernel of copy_bytes each way in the same databases, or,
    for runs without it, by the given (fetch, write) factors."""
    t = counters_table(dbs)
    copy = [v for k, v in t.items() if "copy_kernel" in k]
    if copy and copy_bytes:
        sf = copy_bytes / (copy[0]["FETCH_SIZE"] * 1024.0)
        sw = copy_bytes / (copy[0]["WRITE_SIZE"] * 1024.0)
    elif scales:
        sf, sw = scales
    else:
        raise SystemExit("no copy_kernel dispatch (with --copy-bytes) or --scales to scale FETCH_SIZE / WRITE_SIZE")
    out = []
    for k, v in t.items():
        if not ("sweep" in k or "copy_kernel" in k):
            continue
        cyc = v["GRBM_GUI_ACTIVE"] / XCDS
        rd, wr = v["TCC_EA0_RDREQ_sum"], v["TCC_EA0_WRREQ_sum"]
        fb, wb = v["FETCH_SIZE"] * 1024.0 * sf, v["WRITE_SIZE"] * 1024.0 * sw
        out.append({"kernel": k, "fetch_GB": fb / 1e9, "write_GB": wb / 1e9,
                    "bytes_per_read_req": fb / rd, "bytes_per_write_req": wb / wr,
                    "write_64B_fraction": v["TCC_EA0_WRREQ_64B_sum"] / wr,
                    "read_latency_cycles": v["TCC_EA0_RDREQ_LEVEL_sum"] / rd,
                    "write_latency_cycles": v["TCC_EA0_WRREQ_LEVEL_sum"] / wr,
                    "reads_in_flight": v["TCC_EA0_RDREQ_LEVEL_sum"] / cyc,
                    "writes_in_flight": v["TCC_EA0_WRREQ_LEVEL_sum"] / cyc,
                    "write_stall_fraction": v["TCC_EA0_WRREQ_STALL_sum"] / cyc / TCC_CHANNELS,
                    "read_credit_stall_fraction": v["TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum"] / cyc / TCC_CHANNELS,
                    "write_credit_stall_fraction": v["TCC_EA0_WRREQ_DRAM_CREDIT_STALL_sum"] / cyc / TCC_CHANNELS,
                    "ms": cyc / (clock_ghz * 1e6)})
    return out


def traffic(fetch_db, write_db, kernel, copy_bytes, workload, layout=None, last=None):
    """HBM bytes per launch of the kernel matching `kernel`: the median over its dispatches
    (with `last`, over its last `last` dispatches only: the timed region of a bench run whose
    autotuner launched the same kernel in other shapes first)."""
    f = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    w = counter_per_dispatch(write_db, "WRITE_SIZE")

    def pick(d, sub, n=None):
        vals = [v for k, vs in d.items() if sub in k for v in vs]
        if not vals:
            raise SystemExit("no dispatch of a kernel matching %r" % sub)
        if n:
            vals = vals[-n:]
        vals.sort()
        return vals[len(vals) // 2]  # median over dispatches

    f_copy, w_copy = pick(f, "copy_kernel"), pick(w, "copy_kernel")
    f_k, w_k = pick(f, kernel, last), pick(w, kernel, last)
    sf, sw = copy_bytes / (f_copy * 1024.0), copy_bytes / (w_copy * 1024.0)
    return {"workload": workload, "layout": layout, "kernel_match": kernel, "last_dispatches": last,
            "kernel_source_sha": kernel_source_hash(),
            "fetch_kib_per_launch_raw": f_k, "write_kib_per_launch_raw": w_k,
            "copy_fetch_kib_raw": f_copy, "copy_write_kib_raw": w_copy, "copy_bytes_each_way": copy_bytes,
            "fetch_scale": sf, "write_scale": sw,
            "bytes_per_launch": f_k * 1024.0 * sf + w_k * 1024.0 * sw,
            "fetch_bytes_per_launch": f_k * 1024.0 * sf, "write_bytes_per_launch": w_k * 1024.0 * sw}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--match", default=None)
    s.add_argument("--last", type=int, default=None, help="only the last N dispatches of every kernel")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--layout", default=None, help="storage layout of the profiled run (planes / rows)")
    t.add_argument("--out", default=None)
    t.add_argument("--last", type=int, default=None, help="only the kernel's last N dispatches")
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--match", default=None)
    m = sub.add_parser("memory")
    m.add_argument("dbs", nargs="+")
    m.add_argument("--copy-bytes", type=float, default=None)
    m.add_argument("--scales", default=None,
                   help="fetch,write factors for databases without the copy kernel (e.g. 2,1 on gfx950)")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        rows = stats(a.db, a.match, a.last)
        print("%-110s %6s %12s %10s %10s %10s" % ("kernel", "calls", "total_us", "avg_us", "min_us", "max_us"))
        for r in rows:
            print("%-110s %6d %12.1f %10.1f %10.1f %10.1f" % (r["kernel"][:110], r["calls"], r["total_us"],
                                                               r["avg_us"], r["min_us"], r["max_us"]))
    elif a.cmd == "memory":
        print("%-72s %7s %7s %5s %5s %5s %7s %6s %7s %7s %6s %6s %7s" % (
            "kernel", "rd GB", "wr GB", "B/rd", "B/wr", "wr64", "rd lat", "wr lat", "rd fly", "wr fly",
            "wstall", "rcred", "busy ms"))
        scales = tuple(float(v) for v in a.scales.split(",")) if a.scales else None
        for r in memory_view(a.dbs, a.copy_bytes, scales=scales):
            print("%-72s %7.2f %7.2f %5.0f %5.0f %5.2f %7.0f %6.0f %7.0f %7.0f %6.3f %6.3f %7.3f" % (
                r["kernel"][:72], r["fetch_GB"], r["write_GB"], r["bytes_per_read_req"], r["bytes_per_write_req"],
                r["write_64B_fraction"], r["read_latency_cycles"], r["write_latency_cycles"], r["reads_in_flight"],
                r["writes_in_flight"], r["write_stall_fraction"], r["read_credit_stall_fraction"], r["ms"]))
    elif a.cmd == "counters":
        for k, vals in counters_table(a.dbs, a.match).items():
            print(k[:150])
            for n in sorted(vals):
                print("    %-40s %20.1f" % (n, vals[n]))
    else:
        res = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.workload, a.layout, a.last)
        txt = json.dumps(res, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(txt + "\n")
        print(txt)


if __name__ == "__main__":
    sys.exit(main())
