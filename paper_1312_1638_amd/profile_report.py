"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_1312_1638_amd.profile_report stats DIR
        Markdown table of the kernel statistics (``*_kernel_stats.csv``) that
        ``rocprofv3 --kernel-trace --stats --output-format csv -d DIR`` wrote.

    python -m paper_1312_1638_amd.profile_report trace DIR --kernel SUBSTRING [--last N]
        Average duration (and VGPR count) of the dispatches of the kernels
        whose name contains SUBSTRING in ``*_kernel_trace.csv`` (the last N
        of them: the launches a timing loop made after set-up and tuning).

    python -m paper_1312_1638_amd.profile_report traffic FETCH_DIR WRITE_DIR \\
            --workload NAME --step NAME --kernel SUBSTRING [--last N]
        HBM traffic per dispatch of the kernels whose name contains SUBSTRING
        (the last N such dispatches),
        from one ``rocprofv3 --pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE``
        run (KiB per dispatch), each scaled by what the same counter reads for
        the library's triad kernel (fr_measure_ceiling kind 0: reads 4 GiB and
        writes 2 GiB per dispatch).  Prints one table row in the format
        bench.py reads, with the hash of the library sources it was taken on.

    python -m paper_1312_1638_amd.profile_report gemm-sweep
        Times every instantiated (row blocks, column strips) plan of the
        matrix-core operator kernel on the operator shapes of hex p=3 (16^3
        and 48^3 elements) and hex p=4 (48^3), FP64 and FP32, with the
        measured ceilings, and prints the fastest and slowest plans per shape
        (needs a HIP device; the set-up autotuner makes the same choice per
        mesh).
"""
import argparse
import csv
import glob
import hashlib
import os
import sys

TRIAD_FETCH_KIB = 4 * 1024 * 1024
TRIAD_WRITE_KIB = 2 * 1024 * 1024
TRIAD_NAME = "triad_kernel"


def source_hash(root=None):
    """Hash of every source of the native library (kernels and host code)."""
    root = root or os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(root)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(root, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _csv_rows(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        sys.exit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(names)


def stats(d):
    rows = _csv_rows(d, "_kernel_stats.csv")
    rows.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
    print("| kernel | calls | avg us | min us | max us | total ms | % |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        name = _col(r, "Name", "KernelName")
        print(f"| `{name[:110]}` | {_col(r, 'Calls')} | {float(_col(r, 'AverageNs')) / 1e3:.2f} | "
              f"{float(_col(r, 'MinNs')) / 1e3:.2f} | {float(_col(r, 'MaxNs')) / 1e3:.2f} | "
              f"{float(_col(r, 'TotalDurationNs')) / 1e6:.3f} | {float(_col(r, 'Percentage')):.1f} |")


def trace(d, kernel, last=0):
    rows = [r for r in _csv_rows(d, "_kernel_trace.csv") if kernel in _col(r, "Kernel_Name")]
    if not rows:
        sys.exit(f"no dispatch of a kernel matching {kernel!r}")
    rows.sort(key=lambda r: int(_col(r, "Dispatch_Id")))
    if last > 0:
        rows = rows[-last:]
    dur = [(int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3 for r in rows]
    names = sorted({_col(r, "Kernel_Name") for r in rows})
    print(f"kernel(s): {'; '.join(n[:120] for n in names)}")
    print(f"dispatches: {len(dur)}  average {sum(dur) / len(dur):.2f} us  min {min(dur):.2f} us  "
          f"max {max(dur):.2f} us  VGPR {_col(rows[-1], 'VGPR_Count')}")


def _per_dispatch(d, counter):
    """{kernel name: [value per dispatch]} for one counter (summed over the
    counter's instances within a dispatch)."""
    rows = _csv_rows(d, "_counter_collection.csv")
    acc = {}
    for r in rows:
        if _col(r, "Counter_Name") != counter:
            continue
        key = (_col(r, "Kernel_Name"), _col(r, "Dispatch_Id"))
        acc[key] = acc.get(key, 0.0) + float(_col(r, "Counter_Value"))
    out = {}
    for (name, disp), v in acc.items():
        out.setdefault(name, []).append((int(disp), v))
    return out


def _mean_for(per, sub, last=0):
    """Mean over the dispatches of kernels whose name contains `sub` (the
    last `last` of them if > 0, in dispatch order)."""
    vals = [(i, v) for name, vs in per.items() if sub in name for i, v in vs]
    vals.sort()
    if last > 0:
        vals = vals[-last:]
    vals = [v for _, v in vals]
    if not vals:
        sys.exit(f"no dispatch of a kernel matching {sub!r}")
    return sum(vals) / len(vals), len(vals)


def traffic(fetch_dir, write_dir, workload, step, kernel, last=0):
    fe = _per_dispatch(fetch_dir, "FETCH_SIZE")
    wr = _per_dispatch(write_dir, "WRITE_SIZE")
    tf, _ = _mean_for(fe, TRIAD_NAME)
    tw, _ = _mean_for(wr, TRIAD_NAME)
    kf, nf = _mean_for(fe, kernel, last)
    kw, nw = _mean_for(wr, kernel, last)
    ff, fw = TRIAD_FETCH_KIB / tf, TRIAD_WRITE_KIB / tw
    total = (kf * ff + kw * fw) * 1024.0
    print("| workload | step | kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | "
          "fetch scale | write scale | HBM bytes per launch | sources |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    print(f"| {workload} | {step} | `{kernel}` | {nf}/{nw} | {kf:.1f} | {kw:.1f} | {ff:.4f} | "
          f"{fw:.4f} | {total:.0f} | {source_hash()} |")


def counters(dirs, kernel, last=0):
    """Every counter of one or more --pmc runs, averaged over the last
    `last` dispatches of the kernels whose name contains `kernel`."""
    print(f"| counter | per dispatch (`{kernel}`) | dispatches |")
    print("|---|---|---|")
    for d in dirs:
        names = sorted({_col(r, "Counter_Name") for r in _csv_rows(d, "_counter_collection.csv")})
        for c in names:
            mean, n = _mean_for(_per_dispatch(d, c), kernel, last)
            print(f"| {c} | {mean:.4g} | {n} |")


def read_traffic_table(path, workload, step):
    """HBM bytes per launch for (workload, step) from a table written by
    `traffic`: the row taken on the current library sources, or None (rows
    of earlier sources stay in the table as a record)."""
    if not os.path.exists(path):
        return None
    h = source_hash()
    with open(path) as fh:
        for line in fh:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) == 10 and cells[0] == workload and cells[1] == step and cells[9] == h:
                return float(cells[8])
    return None


SWEEP_SHAPES = [(1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (3, 1), (3, 2), (3, 4), (4, 1),
                (4, 2), (4, 4), (6, 1), (6, 2), (6, 4), (8, 1), (8, 2), (12, 1), (12, 2)]
# (name, M, K1, K2, N, batch)
SWEEP_CASES = [("M0 p3", 96, 64, 0, 20480, 1), ("S3 p3", 192, 96, 64, 20480, 1),
               ("M5 p3", 96, 64, 0, 20480, 3), ("S8 p3", 64, 96, 192, 20480, 1),
               ("M0 p4 L", 150, 125, 0, 552960, 1), ("S8 p4 L", 125, 150, 375, 552960, 1),
               ("S3 p3 L", 192, 96, 64, 552960, 1)]


def gemm_sweep():
    from . import binding as B
    print("ceilings: HBM GB/s %.0f  FP64 MFMA TF %.1f  FP32 MFMA TF %.1f" % (
        B.measure_ceiling(0), B.measure_ceiling(1), B.measure_ceiling(2)), flush=True)
    for prec in ("fp64", "fp32"):
        for name, M, K1, K2, N, batch in SWEEP_CASES:
            MB = -(-M // 16)
            res = []
            for mbw, nc in SWEEP_SHAPES:
                wm = -(-MB // mbw)
                if mbw * (wm - 1) >= MB:
                    continue
                ms = B.bench_gemm(prec, M, K1, K2, N, (mbw, nc, wm), batch, 10)
                tf = 2.0 * M * (K1 + K2) * N * batch / (ms * 1e-3) / 1e12
                res.append((ms, mbw, nc, wm, tf))
            res.sort()
            print(prec, name, " ".join("[%d,%d,%d] %.1fus %.1fTF" % (m, n, w, ms * 1e3, tf)
                                       for ms, m, n, w, tf in res[:6]), flush=True)
            print("   worst", " ".join("[%d,%d,%d] %.1fus" % (m, n, w, ms * 1e3)
                                       for ms, m, n, w, tf in res[-3:]), flush=True)


# Dense triangle operators of the batched 512-problem vortex mesh (2-D,
# 4 fields, element counts per order as in that mesh): interpolation M0
# (Nf x Nu) and the divergence [M3 | M1'] (Nu x (Nf + 2 Nu)).
TRI_CASES = [(p, n) for p, n in ((2, 115552), (3, 134900), (4, 129744))]
BF16_LDS_SHAPES = [(1, 4, 64), (2, 4, 64), (3, 4, 64), (4, 4, 64), (6, 4, 64),
                   (1, 2, 64), (2, 2, 64), (3, 2, 64), (4, 2, 64), (6, 2, 64), (8, 2, 64),
                   (1, 1, 64), (2, 1, 64), (3, 1, 64), (4, 1, 64), (6, 1, 64), (8, 1, 64),
                   (12, 1, 64), (1, 4, 128), (2, 4, 128), (1, 2, 128), (2, 2, 128),
                   (3, 2, 128), (4, 2, 128), (1, 1, 128), (2, 1, 128), (4, 1, 128),
                   (6, 1, 128), (8, 1, 128)]


def tri_sweep():
    """Best plan per precision for the dense triangle operators: FP64 and
    FP32 matrix-core tiles, BF16x3 register and LDS-staged tiles."""
    from . import binding as B
    print("| operator | M x K | N | FP64 us (plan) | FP32 us (plan) | BF16x3 us (plan) | "
          "BF16x3 / FP32 | FP32 GB/s |")
    print("|---|---|---|---|---|---|---|---|")
    for p, nel in TRI_CASES:
        nu, nf = (p + 1) * (p + 2) // 2, 3 * (p + 1)
        N = 4 * (-(-nel // 64) * 64)
        for name, M, K1, K2 in (("M0", nf, nu, 0), ("div", nu, nf, 2 * nu)):
            MB = -(-M // 16)
            best = {}
            for prec in ("fp64", "fp32", "bf16x3"):
                plans = []
                for mbw, nc in SWEEP_SHAPES:
                    wm = -(-MB // mbw)
                    if mbw * (wm - 1) < MB:
                        plans.append((mbw, nc, wm))
                if prec == "bf16x3":
                    plans += [(mbw, tw, wm) for mbw, wm, tw in BF16_LDS_SHAPES
                              if mbw * wm >= MB and mbw * (wm - 1) < MB]
                res = []
                for plan in plans:
                    try:
                        ms = B.bench_gemm(prec, M, K1, K2, N, plan, 1, 10)
                    except B.FRError:
                        continue
                    res.append((ms, plan))
                best[prec] = min(res)
            es = {"fp64": 8, "fp32": 4}
            gbs = ((K1 + K2) + M) * N * es["fp32"] / (best["fp32"][0] * 1e-3) / 1e9
            print(f"| tri p={p} {name} | {M} x {K1 + K2} | {N} | "
                  + " | ".join("%.1f (%s)" % (best[q][0] * 1e3, ",".join(map(str, best[q][1])))
                               for q in ("fp64", "fp32", "bf16x3"))
                  + f" | {best['bf16x3'][0] / best['fp32'][0]:.2f} | {gbs:.0f} |", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--workload", required=True)
    b.add_argument("--step", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--last", type=int, default=0,
                   help="use only the last N matching dispatches")
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--last", type=int, default=0)
    k = sub.add_parser("counters")
    k.add_argument("dirs", nargs="+")
    k.add_argument("--kernel", required=True)
    k.add_argument("--last", type=int, default=0)
    sub.add_parser("hash")
    sub.add_parser("gemm-sweep")
    sub.add_parser("tri-sweep")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        stats(args.dir)
    elif args.cmd == "trace":
        trace(args.dir, args.kernel, args.last)
    elif args.cmd == "traffic":
        traffic(args.fetch_dir, args.write_dir, args.workload, args.step, args.kernel, args.last)
    elif args.cmd == "gemm-sweep":
        gemm_sweep()
    elif args.cmd == "tri-sweep":
        tri_sweep()
    elif args.cmd == "counters":
        counters(args.dirs, args.kernel, args.last)
    else:
        print(source_hash())


if __name__ == "__main__":
    main()
