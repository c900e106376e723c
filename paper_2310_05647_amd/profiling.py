"""Text summaries of rocprofv3 output, and the reader that turns a counter summary into HBM bytes.

rocprofv3 writes its results as an SQLite database (``<dir>/<host>/<pid>_results.db`` or
``<dir>/<prefix>_results.db``); the tables used here are ``kernels`` (one row per dispatch, with its
duration in ns) and ``counters_collection`` (one row per dispatch and counter).

    python -m paper_2310_05647_amd.profiling stats --db DIR --out FILE --command "..."
    python -m paper_2310_05647_amd.profiling traffic --fetch DIR --write DIR --kernel LABEL \\
        --out FILE --command-fetch "..." --command-write "..."
    python -m paper_2310_05647_amd.profiling counters --db DIR [--db DIR ...] --kernels SUBSTR,... \\
        --out FILE --command "..." [--command "..."]

The traffic summary scales each counter by what it reads for a plain streaming kernel of known
size in the same run (bench.py launches one: 256 MiB read, 256 MiB written), and records the
SHA-256 of the kernel's source file so that a reader can tell when the counters have gone stale.
"""
import argparse
import glob
import hashlib
import os
import sqlite3

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# launch label (as timed by the library) -> (kernel symbol substring, source file in csrc/)
KERNELS = {
    "llr_gram": ("k_gram_cells", "llr.hip"),
    "llr_tridiag": ("k_tridiag", "llr.hip"),
    "llr_coef": ("k_coef_strip", "llr.hip"),
    "llr_xupdate": ("k_xupdate_mfma<10, true, true>", "llr.hip"),
    "llr_backxf": ("k_backxf", "llr.hip"),
    "lap_quad": ("k_qc_trace", "graph.hip"),
    "lap_quad_far": ("k_qc_far", "graph.hip"),
    "graph_qc_lists": ("k_qc_lists", "graph.hip"),
    "llr_eig": ("k_eig_val", "llr.hip"),
    "llr_eigvec": ("k_eig_vec", "llr.hip"),
    "match_full": ("k_match_top4", "match.hip"),
    "match_rerank": ("k_rerank", "match.hip"),
    "mlp_gemm": ("k_gemm", "mlp.hip"),
    "mlp_synth": ("k_synth", "mlp.hip"),
    "nufft_col_adj": ("k_col_adj", "nufft.hip"),
    "nufft_col_fwd": ("k_col_fwd", "nufft.hip"),
    "nufft_row_fwd": ("k_row_fwd", "nufft.hip"),
    "nufft_row_adj": ("k_row_adj", "nufft.hip"),
    "match_subspace": ("k_match_sub", "subspace.hip"),
    "graph_knn_dist": ("k_knn_dist", "graph.hip"),
    "graph_knn_select": ("k_knn_select", "graph.hip"),
}
CALIBRATION = "neg_kernel"          # the streaming kernel's symbol substring
CALIBRATION_BYTES = 1 << 28         # read, and the same written


def _db(path):
    if os.path.isfile(path):
        return sqlite3.connect(path)
    hits = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
    if not hits:
        raise FileNotFoundError("no rocprofv3 *_results.db under " + path)
    return sqlite3.connect(hits[0])


def _short(name, n=70):
    name = name.split("(")[0]
    for pre in ("void ", "mrf::"):
        name = name.replace(pre, "")
    return name if len(name) <= n else name[:n - 3] + "..."


def kernel_stats(db):
    """[(name, calls, total_ms, avg_us, min_us, max_us)] by total time, descending."""
    c = _db(db)
    rows = c.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                     "from kernels group by name").fetchall()
    out = [(n, k, t / 1e6, a / 1e3, lo / 1e3, hi / 1e3) for n, k, t, a, lo, hi in rows]
    return sorted(out, key=lambda r: -r[2])


def counter_per_dispatch(db, counter):
    """{kernel name: (mean value per dispatch, dispatches)} for one counter."""
    c = _db(db)
    rows = c.execute("select kernel_name, avg(value), count(*) from counters_collection where counter_name = ? "
                     "group by kernel_name", (counter,)).fetchall()
    return {n: (v, k) for n, v, k in rows}


def _match(table, sub):
    hits = [(n, v) for n, v in table.items() if sub in n]
    if not hits:
        raise KeyError("no kernel matching %r" % sub)
    if len(hits) > 1:
        hits.sort(key=lambda nv: len(nv[0]))
    return hits[0]


def source_sha(src):
    with open(os.path.join(CSRC, src), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def write_stats(db, out, command, top=30):
    rows = kernel_stats(db)
    total = sum(r[2] for r in rows)
    lines = ["# rocprofv3 kernel trace statistics", "command: " + command, "",
             "%-72s %7s %10s %10s %10s %10s %6s" % ("kernel", "calls", "total_ms", "avg_us", "min_us", "max_us", "pct")]
    for n, k, t, a, lo, hi in rows[:top]:
        lines.append("%-72s %7d %10.3f %10.2f %10.2f %10.2f %6.2f" % (_short(n), k, t, a, lo, hi, 100.0 * t / total))
    lines.append("")
    with open(out, "w") as f:
        f.write("\n".join(lines))


def write_traffic(fetch_db, write_db, label, out, command_fetch, command_write):
    sym, src = KERNELS[label]
    fetch = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(write_db, "WRITE_SIZE")
    kname, (fk, nd) = _match(fetch, sym)
    _, (wk, _) = _match(write, sym)
    _, (cfk, _) = _match(fetch, CALIBRATION)
    _, (cwk, _) = _match(write, CALIBRATION)
    fscale = CALIBRATION_BYTES / (cfk * 1024.0)
    wscale = CALIBRATION_BYTES / (cwk * 1024.0)
    hbm = fk * 1024.0 * fscale + wk * 1024.0 * wscale
    lines = ["# HBM traffic of one launch from rocprofv3 counters (KiB per dispatch)",
             "kernel: " + label, "symbol: " + _short(kname, 120), "source: csrc/" + src,
             "source_sha256: " + source_sha(src), "dispatches: %d" % nd,
             "fetch_kib_per_dispatch: %.1f" % fk, "write_kib_per_dispatch: %.1f" % wk,
             "calibration_kernel: torch neg (%d bytes read, %d written)" % (CALIBRATION_BYTES, CALIBRATION_BYTES),
             "calibration_fetch_kib: %.1f" % cfk, "calibration_write_kib: %.1f" % cwk,
             "fetch_scale: %.4f" % fscale, "write_scale: %.4f" % wscale,
             "hbm_bytes_per_launch: %.0f" % hbm,
             "command_fetch: " + command_fetch, "command_write: " + command_write, ""]
    with open(out, "w") as f:
        f.write("\n".join(lines))


def read_summary(path):
    d = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                d[k.strip()] = v.strip()
    return d


def traffic_bytes(profiles_dir, label):
    """HBM bytes per launch of `label` from profiles/<label>__*_traffic.txt, or None if absent or
    if the kernel's source has changed since the counters were taken."""
    if label not in KERNELS:
        return None
    hits = sorted(glob.glob(os.path.join(profiles_dir, label + "__*_traffic.txt")))
    if not hits:
        return None
    d = read_summary(hits[0])
    if d.get("source_sha256") != source_sha(KERNELS[label][1]):
        return None
    return float(d["hbm_bytes_per_launch"])


def counter_table(dbs):
    """{kernel name: {counter: (mean per dispatch, dispatches)}} over one or more counter runs."""
    out = {}
    for db in dbs:
        c = _db(db)
        rows = c.execute("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                         "group by kernel_name, counter_name").fetchall()
        for n, cn, v, k in rows:
            out.setdefault(n, {})[cn] = (v, k)
    return out


N_XCD, N_SIMD, CLOCK_HZ = 8, 1024, 2.4e9   # MI355X: GRBM_GUI_ACTIVE reads as the sum over its 8 XCDs


def derived(c):
    """Derived per-dispatch figures from whichever counters are present: busy time, MFMA
    utilisation (busy MFMA cycles over SIMD cycles), MFMA flops (512 per MOP), LDS bank-conflict
    share of LDS-active cycles, L2 hit rate."""
    g = lambda k: c[k][0] if k in c else None
    out = []
    gui = g("GRBM_GUI_ACTIVE")
    if gui:
        out.append(("busy_ms", gui / N_XCD / CLOCK_HZ * 1e3))
        if g("SQ_VALU_MFMA_BUSY_CYCLES") is not None:
            out.append(("mfma_util_pct", 100.0 * g("SQ_VALU_MFMA_BUSY_CYCLES") / (gui / N_XCD * N_SIMD)))
    mops = sum(g(k) or 0.0 for k in ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16",
                                     "SQ_INSTS_VALU_MFMA_MOPS_F8"))
    if mops:
        out.append(("mfma_gflop", mops * 512 / 1e9))
    if g("SQ_LDS_IDX_ACTIVE"):
        out.append(("lds_bank_conflict_pct", 100.0 * g("SQ_LDS_BANK_CONFLICT") / g("SQ_LDS_IDX_ACTIVE")))
    if g("TCC_REQ_sum"):
        out.append(("l2_hit_pct", 100.0 * g("TCC_HIT_sum") / g("TCC_REQ_sum")))
    return out


def write_counters(dbs, kernels, out, commands):
    """Mean value per dispatch of every collected counter, for each kernel whose symbol contains one
    of the given substrings (all instantiations listed), with the source hashes of their files."""
    table = counter_table(dbs)
    lines = ["# rocprofv3 hardware counters, mean per dispatch"] + ["command: " + c for c in commands]
    for src in sorted({v[1] for v in KERNELS.values()}):
        lines.append("source_sha256 csrc/%s: %s" % (src, source_sha(src)))
    for sub in kernels:
        hits = sorted(n for n in table if sub in n)
        for n in hits:
            lines.append("")
            lines.append("kernel: " + _short(n, 160))
            for cn in sorted(table[n]):
                v, k = table[n][cn]
                lines.append("  %-40s %18.1f   (%d dispatches)" % (cn, v, k))
            for dn, dv in derived(table[n]):
                lines.append("  = %-38s %18.3f" % (dn, dv))
    lines.append("")
    with open(out, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--db", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--command", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--command-fetch", required=True)
    b.add_argument("--command-write", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--db", required=True, action="append")
    c.add_argument("--kernels", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True, action="append")
    args = ap.parse_args()
    if args.cmd == "stats":
        write_stats(args.db, args.out, args.command)
    elif args.cmd == "counters":
        write_counters(args.db, args.kernels.split(","), args.out, args.command)
    else:
        write_traffic(args.fetch, args.write, args.kernel, args.out, args.command_fetch, args.command_write)


if __name__ == "__main__":
    main()
