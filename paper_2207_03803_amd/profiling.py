"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2207_03803_amd.profiling trace DB [--top N]
      per-kernel launches / total / average time from a --kernel-trace database
      (markdown table on stdout)

  python -m paper_2207_03803_amd.profiling kernels --trace DB --sq CSV --fetch CSV --write CSV
         --copy-fetch CSV --copy-write CSV --out PREFIX
      per-kernel table over every kernel of a run: time, MFMA busy share,
      MFMA flops executed, LDS bank conflicts, HBM bytes and GB/s (PREFIX.json,
      PREFIX.table.md)

  python -m paper_2207_03803_amd.profiling traffic --fit-fetch CSV --fit-write CSV
         --copy-fetch CSV --copy-write CSV --out PREFIX
      HBM traffic of the K_NM launch of knm_kernel: FETCH_SIZE and WRITE_SIZE
      (KiB per dispatch) scaled by what the same counters read for a plain
      device copy of known size (bench.py --copy-calibration: 1 GiB read and
      1 GiB written per launch).  Writes PREFIX.json (read by bench.py, keyed
      by a hash of the kernel's sources) and PREFIX.md.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
KNM_SOURCES = ("knm.hip", "knm.h", "common.h")
COPY_BYTES = 8 << 27  # one copy launch of bench.py --copy-calibration, each direction


def source_hash():
    h = hashlib.sha256()
    for f in KNM_SOURCES:
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    return h.hexdigest()


def _short(name):
    return name.split("(")[0].replace("void ", "").strip()


def trace_table(db, top=40):
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(kernels)")]
    name_col = "kernel_name" if "kernel_name" in cols else "name"
    agg = collections.defaultdict(list)
    for name, start, end in con.execute(f"select {name_col}, start, end from kernels"):
        agg[_short(name)].append((end - start) / 1e3)
    lines = ["| kernel | launches | total ms | avg us | min us | max us |", "|---|---:|---:|---:|---:|---:|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"| `{k[:80]}` | {len(v)} | {sum(v) / 1e3:.2f} | {sum(v) / len(v):.1f} | {min(v):.1f} | "
                     f"{max(v):.1f} |")
    return "\n".join(lines)


def _counter_rows(path, counter):
    out = []
    for row in csv.DictReader(open(path)):
        if row["Counter_Name"] == counter:
            out.append((_short(row["Kernel_Name"]), int(row["Grid_Size"]), float(row["Counter_Value"])))
    return out


def _knm_launch(path, counter):
    """The K_NM launch: the knm_kernel dispatch with the largest reading."""
    vals = [v for n, g, v in _counter_rows(path, counter) if n.startswith("gap::knm_kernel")]
    if not vals:
        raise SystemExit(f"no knm_kernel dispatch in {path}")
    return max(vals)


def _copy_launch(path, counter):
    vals = sorted(v for n, g, v in _counter_rows(path, counter) if "copyBuffer" in n)
    if not vals:
        raise SystemExit(f"no copy dispatch in {path}")
    return vals[len(vals) // 2]


def traffic(args):
    fetch = _knm_launch(args.fit_fetch, "FETCH_SIZE")
    write = _knm_launch(args.fit_write, "WRITE_SIZE")
    cf = _copy_launch(args.copy_fetch, "FETCH_SIZE")
    cw = _copy_launch(args.copy_write, "WRITE_SIZE")
    ff = COPY_BYTES / (cf * 1024.0)
    wf = COPY_BYTES / (cw * 1024.0)
    rd = fetch * 1024.0 * ff
    wr = write * 1024.0 * wf
    rec = {
        "kernel": "knm_kernel",
        "workload": "realistic_fp64 (K_NM launch: N=1e5 configs, 3,998,181 atoms, d=400, M=1e4)",
        "fetch_size_kib_per_launch": fetch,
        "write_size_kib_per_launch": write,
        "copy_calibration": {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES, "fetch_size_kib": cf,
                             "write_size_kib": cw, "fetch_factor": ff, "write_factor": wf},
        "hbm_read_bytes_per_launch": rd,
        "hbm_write_bytes_per_launch": wr,
        "source_sha256": source_hash(),
        "traffic_bytes_per_launch": rd + wr,
    }
    json.dump(rec, open(args.out + ".json", "w"), indent=1)
    d_ff, d_fw = os.path.dirname(args.fit_fetch), os.path.dirname(args.fit_write)
    d_cf, d_cw = os.path.dirname(args.copy_fetch), os.path.dirname(args.copy_write)
    md = f"""# HBM traffic of `knm_kernel`, realistic workload (K_NM launch)

Counters from two `rocprofv3 --pmc` passes over one benchmark run, then the same two
counters over a plain 1 GiB device-to-device copy (bench.py --copy-calibration) to
calibrate what each counter reads for a known byte count.  Produced by
`python -m paper_2207_03803_amd.profiling traffic ...` from these runs (repository root,
one MI355X):
```
rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d_ff} -o fit -- python3 bench.py {args.bench_args}
rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d_fw} -o fit -- python3 bench.py {args.bench_args}
rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d_cf} -o copy -- python3 bench.py --copy-calibration
rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d_cw} -o copy -- python3 bench.py --copy-calibration
```

| quantity | counter reading (KiB) | calibration factor | bytes |
|---|---:|---:|---:|
| copy, 1 GiB read | FETCH_SIZE {cf:.4e} | {ff:.3f} | {COPY_BYTES:.4e} |
| copy, 1 GiB written | WRITE_SIZE {cw:.4e} | {wf:.3f} | {COPY_BYTES:.4e} |
| knm_kernel (K_NM launch) read | FETCH_SIZE {fetch:.4e} | {ff:.3f} | {rd:.4e} |
| knm_kernel (K_NM launch) written | WRITE_SIZE {write:.4e} | {wf:.3f} | {wr:.4e} |

Algorithmic bytes of the K_NM launch: descriptors read once (3,998,181 x 400 x 8 =
12.8 GB), sparse points (32 MB), the N x M output written once (8.0 GB): about 20.8 GB.
Traffic past L2 well above that is the sparse set re-read by every atom tile, which the
256 MB Infinity Cache serves for the most part.
"""
    open(args.out + ".md", "w").write(md)
    print(json.dumps(rec, indent=1))


def _sums(path, counters):
    """{kernel: {counter: (sum over dispatches, dispatches)}} from a --pmc CSV."""
    out = collections.defaultdict(dict)
    seen = collections.defaultdict(set)
    for row in csv.DictReader(open(path)):
        c = row["Counter_Name"]
        if c not in counters:
            continue
        k = _short(row["Kernel_Name"])
        v, n = out[k].get(c, (0.0, 0))
        did = row.get("Dispatch_Id") or row.get("Correlation_Id") or str(len(seen[(k, c)]))
        new = did not in seen[(k, c)]
        seen[(k, c)].add(did)
        out[k][c] = (v + float(row["Counter_Value"]), n + (1 if new else 0))
    return out


def _durations(db):
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(kernels)")]
    name_col = "kernel_name" if "kernel_name" in cols else "name"
    agg = collections.defaultdict(list)
    for name, start, end in con.execute(f"select {name_col}, start, end from kernels"):
        agg[_short(name)].append((end - start) * 1e-9)
    return agg


def kernels(args):
    """Per-kernel table: time (kernel trace), MFMA busy share of the SIMD cycles,
    MFMA flops executed, LDS bank conflicts per LDS instruction, HBM bytes read /
    written (FETCH_SIZE / WRITE_SIZE scaled by the copy calibration) and GB/s."""
    dur = _durations(args.trace)
    mops_counters = ("SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16",
                     "SQ_INSTS_VALU_MFMA_MOPS_F16", "SQ_INSTS_VALU_MFMA_MOPS_I8")
    sq = _sums(args.sq, {"SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS",
                         *mops_counters})
    fe = _sums(args.fetch, {"FETCH_SIZE"})
    wr = _sums(args.write, {"WRITE_SIZE"})
    cf = _copy_launch(args.copy_fetch, "FETCH_SIZE")
    cw = _copy_launch(args.copy_write, "WRITE_SIZE")
    ff, wf = COPY_BYTES / (cf * 1024.0), COPY_BYTES / (cw * 1024.0)
    rows = []
    for k, ds in sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:args.top]:
        t = sum(ds)
        q = sq.get(k, {})
        busy = q.get("SQ_VALU_MFMA_BUSY_CYCLES", (0.0, 0))[0]
        grbm = q.get("GRBM_GUI_ACTIVE", (0.0, 0))[0]
        # GRBM_GUI_ACTIVE is summed over the XCDs; MFMA busy cycles over every SIMD
        util = busy / (grbm / args.xcds * args.simds) if grbm > 0 else float("nan")
        # MFMA operations the counters saw (a pass holds only some of the MOPS counters)
        mops = sum(q.get(c, (0.0, 0))[0] for c in mops_counters)
        lds = q.get("SQ_INSTS_LDS", (0.0, 0))[0]
        conf = q.get("SQ_LDS_BANK_CONFLICT", (0.0, 0))[0]
        rd = fe.get(k, {}).get("FETCH_SIZE", (0.0, 0))[0] * 1024.0 * ff
        wb = wr.get(k, {}).get("WRITE_SIZE", (0.0, 0))[0] * 1024.0 * wf
        rows.append(dict(kernel=k, launches=len(ds), total_ms=t * 1e3, mfma_busy=util,
                         mfma_tflops=mops * 512 / t / 1e12 if t > 0 else 0.0,
                         lds_conflict_per_inst=conf / lds if lds > 0 else 0.0,
                         read_gb=rd / 1e9, write_gb=wb / 1e9, gbps=(rd + wb) / t / 1e9 if t > 0 else 0.0))
    json.dump(dict(rows=rows, copy_calibration=dict(fetch_factor=ff, write_factor=wf)),
              open(args.out + ".json", "w"), indent=1)
    lines = ["| kernel | launches | total ms | MFMA busy | MFMA TFLOP/s (TOP/s) | LDS conflicts / inst | HBM read GB | "
             "HBM write GB | GB/s |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{r['kernel'][:60]}` | {r['launches']} | {r['total_ms']:.2f} | {100 * r['mfma_busy']:.1f} % | "
                     f"{r['mfma_tflops']:.1f} | {r['lds_conflict_per_inst']:.2f} | {r['read_gb']:.2f} | "
                     f"{r['write_gb']:.2f} | {r['gbps']:.0f} |")
    table = "\n".join(lines)
    open(args.out + ".table.md", "w").write(table + "\n")
    print(table)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=40)
    f = sub.add_parser("traffic")
    for k in ("fit-fetch", "fit-write", "copy-fetch", "copy-write", "out"):
        f.add_argument("--" + k, required=True)
    f.add_argument("--bench-args", default="--steps 1 --warmup 0 --no-cpu-baseline --forms mixed,bf16 --inputs device",
                   help="the bench.py arguments of the profiled run (quoted in the summary)")
    k = sub.add_parser("kernels")
    for a in ("trace", "sq", "fetch", "write", "copy-fetch", "copy-write", "out"):
        k.add_argument("--" + a, required=True)
    k.add_argument("--top", type=int, default=30)
    k.add_argument("--xcds", type=int, default=8)
    k.add_argument("--simds", type=int, default=1024)
    args = ap.parse_args()
    if args.cmd == "trace":
        print(trace_table(args.db, args.top))
    elif args.cmd == "kernels":
        kernels(args)
    else:
        traffic(args)


if __name__ == "__main__":
    main()
