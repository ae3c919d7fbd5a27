"""Short text summaries of rocprofv3 runs (rocpd SQLite databases).

    python -m paper_2603_28770_amd.rocprof_summary \
        --trace T.db --fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db \
        --copy-bytes 268435456 --kernel bfgs_kernel --workload rastrigin_d10_n65536 \
        --command "..." [--command "..."] -o profiles/bfgs_kernel_rastrigin_d10_n65536.md

The trace database comes from ``rocprofv3 --kernel-trace --stats``; the four
counter databases from ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``
of the workload and of a plain device-to-device copy of ``--copy-bytes`` bytes.
The copy fixes what the counters read per byte actually moved: its reads and
writes are both exactly ``copy-bytes``, so each counter of the workload is
scaled by copy-bytes / (what the counter read for the copy).

Optional ``--mix`` databases come from ``rocprofv3 --pmc`` passes of SQ
instruction counters on the same workload; from them the summary adds the
kernel's instruction mix and its FP64 rate as the counters see it:
64 lanes x (2 FMA + ADD + MUL + transcendental) FP64 wave instructions per
dispatch over the average duration (padding lanes included).  The VALU busy
share is 4 SQ_ACTIVE_INST_VALU / (32 SQ_BUSY_CYCLES): the wave counters count
in units of four cycles, and each of the 32 SQs serves 32 SIMDs.

The summary ends with a JSON block (kernel, workload, average duration,
scaled HBM bytes per dispatch, and a SHA-256 of the kernel's sources at
summary time), which ``bench.py`` reads to report measured traffic only while
the sources still match.
"""
import argparse
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# Sources that define each kernel's code.
KERNEL_SOURCES = {
    "bfgs_kernel": ["csrc/zeus_bfgs_kernels.h", "csrc/zeus_bfgs_common.h", "csrc/zeus_group.h",
                    "csrc/zeus_device.h", "csrc/zeus_internal.h"],
    "pso_kernel": ["csrc/zeus_pso_kernels.h", "csrc/zeus_group.h", "csrc/zeus_device.h",
                   "csrc/zeus_internal.h"],
    "lbfgs_kernel": ["csrc/zeus_lbfgs_kernels.h", "csrc/zeus_bfgs_common.h", "csrc/zeus_group.h",
                     "csrc/zeus_device.h", "csrc/zeus_internal.h"],
    "bfgs_tile_kernel": ["csrc/zeus_bfgs_tile_kernels.h", "csrc/zeus_block.h", "csrc/zeus_bfgs_common.h",
                         "csrc/zeus_group.h", "csrc/zeus_device.h", "csrc/zeus_internal.h"],
    "bfgs_hybrid_kernel": ["csrc/zeus_bfgs_hybrid_kernels.h", "csrc/zeus_block.h", "csrc/zeus_bfgs_common.h",
                           "csrc/zeus_group.h", "csrc/zeus_device.h", "csrc/zeus_internal.h"],
    "bfgs_wide_kernel": ["csrc/zeus_bfgs_wide.hip", "csrc/zeus_block.h", "csrc/zeus_bfgs_common.h",
                         "csrc/zeus_group.h", "csrc/zeus_device.h", "csrc/zeus_internal.h"],
}


def sources_sha256(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    name = name.replace("zeus::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0]


def kernel_stats(db: str):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                     "group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1.0
    return [{"kernel": _short(r[0]), "calls": r[1], "total_ms": r[2] / 1e6,
             "avg_us": r[3] / 1e3, "pct": 100.0 * r[2] / total} for r in rows]


def counter_per_dispatch(db: str, counter: str):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, count(*), avg(value) from counters_collection "
                     "where counter_name = ? group by kernel_name", (counter,)).fetchall()
    return {_short(r[0]): (r[1], r[2]) for r in rows}


def copy_factor(db: str, counter: str, nbytes: int) -> float:
    per = counter_per_dispatch(db, counter)
    kib = [v for k, (n, v) in per.items() if "copyBuffer" in k]
    if not kib:
        raise SystemExit(f"{db}: no copy kernel found for {counter}")
    return nbytes / (kib[0] * 1024.0)


def main(argv=None):
    ap = argparse.ArgumentParser()
    for a in ("trace", "fetch", "write", "copy-fetch", "copy-write", "kernel", "workload", "o"):
        ap.add_argument("--" + a if len(a) > 1 else "-" + a, required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--note", default="")
    ap.add_argument("--mix", action="append", default=[],
                    help="rocprofv3 --pmc database with SQ instruction counters (repeatable)")
    args = ap.parse_args(argv)

    stats = kernel_stats(args.trace)
    fetch = counter_per_dispatch(args.fetch, "FETCH_SIZE")
    write = counter_per_dispatch(args.write, "WRITE_SIZE")
    ff = copy_factor(args.copy_fetch, "FETCH_SIZE", args.copy_bytes)
    wf = copy_factor(args.copy_write, "WRITE_SIZE", args.copy_bytes)
    main_k = [s for s in stats if s["kernel"].split("<")[0].endswith(args.kernel)]
    if not main_k:
        raise SystemExit(f"kernel {args.kernel} not in the trace")
    mk = main_k[0]

    def scaled(name):
        fk = next((v for k, (n, v) in fetch.items() if k == name), None)
        wk = next((v for k, (n, v) in write.items() if k == name), None)
        if fk is None or wk is None:
            return None, None, None, None
        return fk, wk, fk * 1024.0 * ff, wk * 1024.0 * wf

    lines = [f"# {args.kernel} -- {args.workload}", ""]
    if args.note:
        lines += [args.note, ""]
    lines += ["Commands (run from the repository root on one MI355X, `TMPDIR=/tmp`):", "", "```"]
    lines += args.command + ["```", "", "## Kernel trace", "",
                             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for s in stats:
        lines.append(f"| `{s['kernel']}` | {s['calls']} | {s['total_ms']:.3f} | "
                     f"{s['avg_us']:.2f} | {s['pct']:.1f} |")
    lines += ["", "## HBM traffic per dispatch (PMC)", "",
              f"Copy calibration: a {args.copy_bytes} B device copy reads {args.copy_bytes / ff / 1024:.1f} KiB "
              f"in FETCH_SIZE and {args.copy_bytes / wf / 1024:.1f} KiB in WRITE_SIZE, so FETCH_SIZE is scaled "
              f"by {ff:.4f} and WRITE_SIZE by {wf:.4f}.", "",
              "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB (scaled) | written MB (scaled) |",
              "|---|---|---|---|---|"]
    for s in stats:
        fk, wk, fb, wb = scaled(s["kernel"])
        if fk is None:
            continue
        lines.append(f"| `{s['kernel']}` | {fk:.1f} | {wk:.1f} | {fb / 1e6:.3f} | {wb / 1e6:.3f} |")
    fk, wk, fb, wb = scaled(mk["kernel"])
    summary = {"kernel": args.kernel, "instance": mk["kernel"], "workload": args.workload,
               "avg_duration_us": mk["avg_us"], "calls": mk["calls"],
               "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
               "fetch_factor": ff, "write_factor": wf,
               "read_bytes": fb, "write_bytes": wb,
               "traffic_bytes": (fb + wb) if fb is not None else None,
               "sources_sha256": sources_sha256(args.kernel)}
    if args.mix:
        mix = {}
        for db in args.mix:
            c = sqlite3.connect(db)
            for kn, cn, v in c.execute("select kernel_name, counter_name, avg(value) "
                                       "from counters_collection group by kernel_name, counter_name"):
                if _short(kn) == mk["kernel"]:
                    mix[cn] = v
        lines += ["", "## Instruction mix of the main kernel per dispatch (PMC)", "",
                  "| counter | value |", "|---|---|"]
        lines += [f"| {k} | {v:.4g} |" for k, v in sorted(mix.items())]
        f64 = [mix.get("SQ_INSTS_VALU_" + k) for k in ("FMA_F64", "ADD_F64", "MUL_F64")]
        if all(v is not None for v in f64):
            flops = 64.0 * (2.0 * f64[0] + f64[1] + f64[2] + mix.get("SQ_INSTS_VALU_TRANS_F64", 0.0))
            summary["counter_fp64_flops"] = flops
            summary["counter_fp64_tflops"] = flops / (mk["avg_us"] * 1e-6) / 1e12
        if "SQ_ACTIVE_INST_VALU" in mix and "SQ_BUSY_CYCLES" in mix:
            summary["valu_busy"] = 4.0 * mix["SQ_ACTIVE_INST_VALU"] / (32.0 * mix["SQ_BUSY_CYCLES"])
        summary["mix"] = mix
    lines += ["", "## Figures used by bench.py", "", "```json", json.dumps(summary, indent=1), "```", ""]
    os.makedirs(os.path.dirname(os.path.abspath(args.o)), exist_ok=True)
    with open(args.o, "w") as f:
        f.write("\n".join(lines))
    print(args.o)


def load(path: str):
    """The JSON block of a summary written by main(), or None."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    a = text.rfind("```json")
    if a < 0:
        return None
    b = text.find("```", a + 7)
    return json.loads(text[a + 7:b])


if __name__ == "__main__":
    sys.exit(main())
