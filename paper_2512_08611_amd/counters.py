"""Summaries of rocprofv3 runs of bench.py: kernel durations and HBM bytes.

A summary (a short markdown file under profiles/) records, per kernel of one
workload: the mean duration from a --kernel-trace --stats run, and the HBM
bytes per launch from two counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per
dispatch).  Each counter is scaled by what it reads for a plain device copy of
known size in the same run (the copy bench.py --copy-calibration issues), so
bytes = FETCH_SIZE * 1024 * copied/FETCH_SIZE(copy) and likewise for writes.
An optional third counter run (SQ_INSTS_VALU_FMA_F64, _ADD_F64, _MUL_F64,
_TRANS_F64: wave instructions per dispatch) gives the hardware FP64 operations
per launch, (2 FMA + ADD + MUL) * 64 lanes, with the transcendental ones
(square roots, reciprocals) listed beside.  An optional fourth run counts the
L2-to-fabric read requests by size (TCC_EA0_RDREQ_32B/_64B/_128B): their bytes
need no calibration and check the scaled FETCH_SIZE kernel by kernel.

The summary carries a digest of the kernel sources (csrc/*, include/lwfr.h,
comments removed); bench.py reports the measured traffic only while the digest matches the
current sources, and null otherwise.

  python -m paper_2512_08611_amd.counters --stats KT_STATS.csv --fetch FETCH.csv \\
      --write WRITE.csv --copy-bytes 268435456 --match MHD2D --out profiles/NAME.md \\
      --command "..." [--command "..."]
"""
import argparse
import csv
import glob
import hashlib
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)


def code_only(text):
    """C/C++ source without its comments, trailing blanks and empty lines: what
    the compiler sees, so that a comment edit leaves the digest unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, copied whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (line.rstrip() for line in "".join(out).splitlines())
    return "\n".join(line for line in lines if line) + "\n"


def sources_digest(root=ROOT):
    """sha256 over the kernel sources and the C ABI header (code only, comments
    removed), in name order."""
    files = sorted(glob.glob(os.path.join(root, "paper_2512_08611_amd", "csrc", "*")))
    files.append(os.path.join(root, "include", "lwfr.h"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()


def _short(name):
    """'void lwfr::k_stages<lwfr::MHD2D, 4, 5>(...)' -> 'k_stages<MHD2D, 4, 5>'."""
    n = name.split("(")[0].replace("void ", "").replace("lwfr::", "")
    return n.strip()


def _counter_means(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(_short(r["Kernel_Name"]), []).append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return vals


def _copy_factor(vals, copy_bytes):
    """bytes per counter KiB from the calibration copy: the last of the run's
    device copies with the largest grid (bench.py makes it after every other
    launch; an upload of a larger state earlier in the run has the same grid)."""
    copies = [v for k, lst in vals.items() if "copyBuffer" in k for v in lst]
    if not copies:
        raise ValueError("no device copy in the counter run (run bench.py with --copy-calibration)")
    gmax = max(g for g, _ in copies)
    kib = [c for g, c in copies if g == gmax][-1]
    return copy_bytes / kib


RDREQ_COUNTERS = (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64), ("TCC_EA0_RDREQ_128B_sum", 128))
FP64_COUNTERS = ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64")


def summarize(stats_csv, fetch_csv, write_csv, copy_bytes, match, fp64_csv=None, rdreq_csv=None):
    """{kernel: {mean_us, calls, fetch_bytes, write_bytes[, fp64_ops, fp64_trans][, read_bytes_req]}}
    for kernels whose name contains `match`, and the two calibration factors."""
    out = {}
    for r in csv.DictReader(open(stats_csv)):
        k = _short(r["Name"])
        if match in k:
            out[k] = {"mean_us": float(r["AverageNs"]) / 1e3, "calls": int(r["Calls"])}
    fv = _counter_means(fetch_csv, "FETCH_SIZE")
    wv = _counter_means(write_csv, "WRITE_SIZE")
    ff = _copy_factor(fv, copy_bytes)
    fw = _copy_factor(wv, copy_bytes)
    for k in out:
        f = [v for _, v in fv.get(k, [])]
        w = [v for _, v in wv.get(k, [])]
        out[k]["fetch_bytes"] = ff * sum(f) / len(f) if f else None
        out[k]["write_bytes"] = fw * sum(w) / len(w) if w else None
    if fp64_csv:
        cm = {c: _counter_means(fp64_csv, c) for c in FP64_COUNTERS}

        def mean(c, k):
            vals = [v for _, v in cm[c].get(k, [])]
            return sum(vals) / len(vals) if vals else None

        for k in out:
            fma, add, mul, tr = (mean(c, k) for c in FP64_COUNTERS)
            if None not in (fma, add, mul):
                out[k]["fp64_ops"] = (2 * fma + add + mul) * 64
                out[k]["fp64_trans"] = (tr or 0.0) * 64
    if rdreq_csv:
        rm = {c: _counter_means(rdreq_csv, c) for c, _ in RDREQ_COUNTERS}
        for k in out:
            tot = 0.0
            for c, size in RDREQ_COUNTERS:
                vals = [v for _, v in rm[c].get(k, [])]
                if not vals:
                    break
                tot += size * sum(vals) / len(vals)
            else:
                out[k]["read_bytes_req"] = tot
    return out, ff, fw


def write_md(path, title, summary, ff, fw, commands, digest):
    lines = [f"# {title}", "", "Commands (run from the repository root R; the counter passes are separate runs):", ""]
    lines += ["```"] + list(commands) + ["```", ""]
    lines += [f"Calibration (256 MiB device copy in the same runs): FETCH_SIZE x {ff / 1024:.3f} KiB, "
              f"WRITE_SIZE x {fw / 1024:.3f} KiB per counted KiB.", ""]
    lines += ["| kernel | calls | mean (us) | HBM read (MB/launch) | HBM write (MB/launch) | GB/s | % of 8 TB/s | "
              "FP64 hw ops (G/launch) | TFLOP/s | % of 78.6 |", "|---|---|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(summary.items(), key=lambda kv: -kv[1]["mean_us"] * kv[1]["calls"]):
        rd = v["fetch_bytes"] or 0.0
        wr = v["write_bytes"] or 0.0
        bw = (rd + wr) / (v["mean_us"] * 1e-6) / 1e9 if v["mean_us"] else 0.0
        ops = v.get("fp64_ops")
        fl = ops / (v["mean_us"] * 1e-6) / 1e12 if ops is not None and v["mean_us"] else None
        fcols = f"{ops / 1e9:.2f} | {fl:.1f} | {100 * fl / 78.6:.1f}" if fl is not None else "- | - | -"
        lines.append(f"| `{k}` | {v['calls']} | {v['mean_us']:.1f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {bw:.0f} | "
                     f"{100 * bw / 8000:.1f} | {fcols} |")
    lines += ["", "FP64 hw ops = (2 FMA + ADD + MUL) x 64 lanes from the SQ_INSTS_VALU_*_F64 counters "
              "(transcendental instructions not counted).", ""]
    req = [(k, v) for k, v in sorted(summary.items()) if v.get("read_bytes_req") and v["fetch_bytes"]]
    if req:
        lines += ["Read bytes from the request-size counters (no calibration) against the scaled FETCH_SIZE:", ""]
        lines += [f"- `{k}`: {v['read_bytes_req'] / 1e6:.1f} MB by request counts, {v['fetch_bytes'] / 1e6:.1f} MB "
                  f"by FETCH_SIZE (ratio {v['read_bytes_req'] / v['fetch_bytes']:.4f})" for k, v in req]
        lines += [""]
    lines += [f"kernel sources sha256: {digest}", ""]
    for k, v in sorted(summary.items()):
        if v["fetch_bytes"] is not None and v["write_bytes"] is not None:
            lines.append(f"traffic_bytes {k} {v['fetch_bytes'] + v['write_bytes']:.0f} mean_us {v['mean_us']:.3f}")
        if v.get("fp64_ops") is not None:
            lines.append(f"fp64_ops {k} {v['fp64_ops']:.0f} trans {v['fp64_trans']:.0f}")
    open(path, "w").write("\n".join(lines) + "\n")


def read_traffic(path, kernel_prefix, digest=None):
    """(bytes per launch, mean us) of the first kernel whose name starts with kernel_prefix in the
    summary at path, or (None, None) if missing or if the summary's source digest differs."""
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    m = re.search(r"kernel sources sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != (digest or sources_digest()):
        return None, None
    for line in text.splitlines():
        if line.startswith("traffic_bytes "):
            parts = line.split()
            # traffic_bytes <name with spaces> <bytes> mean_us <us>
            name = " ".join(parts[1:-3])
            if name.startswith(kernel_prefix):
                return float(parts[-3]), float(parts[-1])
    return None, None


def read_table(path, digest=None):
    """{kernel name: {"bytes": HBM bytes per launch, "mean_us": ..., "fp64_ops": ...}} from a
    summary, or {} if it is missing or its source digest differs from the sources."""
    if not os.path.exists(path):
        return {}
    text = open(path).read()
    m = re.search(r"kernel sources sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != (digest or sources_digest()):
        return {}
    out = {}
    for line in text.splitlines():
        parts = line.split()
        if line.startswith("traffic_bytes "):
            name = " ".join(parts[1:-3])
            out.setdefault(name, {}).update(bytes=float(parts[-3]), mean_us=float(parts[-1]))
        elif line.startswith("fp64_ops "):
            name = " ".join(parts[1:-3])
            out.setdefault(name, {}).update(fp64_ops=float(parts[-3]), fp64_trans=float(parts[-1]))
    return out


def trace_summary(trace_csv, steps, match="lwfr::"):
    """Per-kernel durations of the last `steps` steps of a --kernel-trace run whose last
    launches are one graph replay of `steps` steps (bench.py --graph-trace), the
    span from the first start to the last end of those launches, and the summed
    kernel time: {kernel: [durations ns]}, span_ns, busy_ns."""
    rows = [r for r in csv.DictReader(open(trace_csv)) if match in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    # a step ends with its update kernel (chained steps have no k_pre): the last
    # `steps` steps are the launches after the update of the step before them
    names = [_short(r["Kernel_Name"]) for r in rows]
    ups = [i for i, n in enumerate(names) if n.startswith("k_update<")]
    last = rows[ups[-steps - 1] + 1:] if len(ups) > steps else rows
    out = {}
    for r in last:
        out.setdefault(_short(r["Kernel_Name"]), []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    span = int(last[-1]["End_Timestamp"]) - int(last[0]["Start_Timestamp"])
    busy = sum(sum(v) for v in out.values())
    return out, span, busy


def write_trace_md(path, title, trace_csv, steps, commands, ms_per_step):
    ker, span, busy = trace_summary(trace_csv, steps)
    lines = [f"# {title}", "", "Command (run from the repository root R):", "", "```"] + list(commands) + ["```", ""]
    lines += [f"The last {steps} steps of the run are one replay of the HIP graph that bench.py times "
              f"(the timed region).  Per step: kernel span {span / steps / 1e3:.1f} us, summed kernel time "
              f"{busy / steps / 1e3:.1f} us; the same run's bench line: {ms_per_step * 1e3:.1f} us per step.", ""]
    lines += ["| kernel | launches | mean (us) | min (us) | max (us) | us per step | % of step |",
              "|---|---|---|---|---|---|---|"]
    for k, v in sorted(ker.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{k}` | {len(v)} | {sum(v) / len(v) / 1e3:.1f} | {min(v) / 1e3:.1f} | {max(v) / 1e3:.1f} | "
                     f"{sum(v) / steps / 1e3:.1f} | {100 * sum(v) / busy:.1f} |")
    lines += ["", f"kernel sources sha256: {sources_digest()}", ""]
    open(path, "w").write("\n".join(lines) + "\n")


def launches_by_grid(trace_csv, match="lwfr::"):
    """{(kernel, grid threads): [durations ns]} from a --kernel-trace run: launches
    of one kernel on problems of different sizes apart."""
    out = {}
    for r in csv.DictReader(open(trace_csv)):
        if match not in r["Kernel_Name"]:
            continue
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        out.setdefault((_short(r["Kernel_Name"]), grid), []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def write_stats_md(path, title, stats_csv, commands, top=40, trace_csv=None):
    """The per-kernel table of a rocprofv3 --stats run (every launch of the run);
    with the run's kernel trace, also the library's kernels per launch grid."""
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# {title}", "", "Command (run from the repository root R):", "", "```"] + list(commands) + ["```", ""]
    lines += ["| kernel | calls | total (us) | average (us) | min (us) | max (us) | % |",
              "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    if trace_csv:
        by = launches_by_grid(trace_csv)
        lines += ["", "The library's kernels per launch grid (one grid size per problem size), from the same "
                  "run's kernel trace:", "",
                  "| kernel | grid (threads) | launches | mean (us) | min (us) | max (us) |", "|---|---|---|---|---|---|"]
        for (k, g), v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:top]:
            lines.append(f"| `{k}` | {g} | {len(v)} | {sum(v) / len(v) / 1e3:.1f} | {min(v) / 1e3:.1f} | "
                         f"{max(v) / 1e3:.1f} |")
    lines += ["", f"kernel sources sha256: {sources_digest()}", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def pipes_summary(csvs, match="lwfr::", min_waves=10000):
    """Per kernel and launch grid, the per-launch means of every counter in the
    counter_collection.csv files of several rocprofv3 --pmc passes (each pass a
    run of the same command), and the launch duration of those passes."""
    agg, cnt, dur = {}, {}, {}
    for path in csvs:
        for r in csv.DictReader(open(path)):
            if match not in r["Kernel_Name"]:
                continue
            k = (_short(r["Kernel_Name"]), int(r["Grid_Size"]))
            c = r["Counter_Name"]
            agg.setdefault(k, {}).setdefault(c, 0.0)
            agg[k][c] += float(r["Counter_Value"])
            cnt.setdefault(k, {}).setdefault(c, 0)
            cnt[k][c] += 1
            dur.setdefault(k, {}).setdefault(c, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = {}
    for k, d in agg.items():
        mean = {c: v / cnt[k][c] for c, v in d.items()}
        if mean.get("SQ_WAVES", 0.0) < min_waves:
            continue
        ds = [x for v in dur[k].values() for x in v]
        g = dur[k].get("GRBM_GUI_ACTIVE", ds)
        # the clock takes the durations of the pass that counted GRBM_GUI_ACTIVE
        out[k] = dict(mean, duration_ns=sum(ds) / len(ds), grbm_duration_ns=sum(g) / len(g))
    return out


def write_pipes_md(path, title, csvs, commands, xcds=8, cus=256, lds_bytes_per_clk=128):
    """VALU issue and LDS activity per kernel: instructions per wave, the clock from
    GRBM_GUI_ACTIVE (cycles summed over the XCDs) over the launch, VALU busy as
    4 cycles per wave instruction over the waves of one SIMD, LDS bytes per wave
    from the LDS bandwidth counters (64-byte units), LDS busy from SQ_LDS_IDX_ACTIVE
    over SQ_BUSY_CU_CYCLES and the bank-conflict share of it."""
    s = pipes_summary(csvs)
    lines = [f"# {title}", "", "Commands (run from the repository root R; one counter pass per run):", "", "```"]
    lines += list(commands) + ["```", ""]
    lines += ["| kernel | grid | waves | us | clock (GHz) | VALU / wave | VALU busy | LDS instr / wave | LDS KB / wave | "
              "LDS busy | bank conflicts (of LDS busy) |", "|---|---|---|---|---|---|---|---|---|---|---|"]
    for (k, g), m in sorted(s.items(), key=lambda kv: -kv[1]["duration_ns"]):
        w = m["SQ_WAVES"]
        cyc = m.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        ghz = cyc / m["grbm_duration_ns"] if m["grbm_duration_ns"] else 0.0
        valu = m.get("SQ_INSTS_VALU", 0.0) / w
        valu_busy = 4 * m.get("SQ_INSTS_VALU", 0.0) / (4 * cus) / cyc if cyc else 0.0
        lds_i = m.get("SQ_INSTS_LDS", 0.0) / w
        lds_kb = 64 * (m.get("SQ_INSTS_LDS_LOAD_BANDWIDTH", 0.0) + m.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0.0)) / w / 1024
        busy_cu = m.get("SQ_BUSY_CU_CYCLES", 0.0)
        lds_busy = m.get("SQ_LDS_IDX_ACTIVE", 0.0) / busy_cu if busy_cu else 0.0
        conf = m.get("SQ_LDS_BANK_CONFLICT", 0.0) / m["SQ_LDS_IDX_ACTIVE"] if m.get("SQ_LDS_IDX_ACTIVE") else 0.0
        lines.append(f"| `{k}` | {g} | {w:.0f} | {m['duration_ns'] / 1e3:.1f} | {ghz:.2f} | {valu:.0f} | "
                     f"{100 * valu_busy:.0f} % | {lds_i:.0f} | {lds_kb:.1f} | {100 * lds_busy:.0f} % | {100 * conf:.0f} % |")
    lines += ["", "Per-launch means of every counter:", ""]
    names = sorted({c for m in s.values() for c in m if not c.endswith("duration_ns")})
    lines += ["| kernel | grid | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for (k, g), m in sorted(s.items(), key=lambda kv: -kv[1]["duration_ns"]):
        lines.append(f"| `{k}` | {g} | " + " | ".join(f"{m.get(c, float('nan')):.4g}" for c in names) + " |")
    lines += ["", f"kernel sources sha256: {sources_digest()}", ""]
    open(path, "w").write("\n".join(lines) + "\n")


def main():
    if len(os.sys.argv) > 1 and os.sys.argv[1] == "pipes":
        pp = argparse.ArgumentParser(description="VALU and LDS activity per kernel from rocprofv3 --pmc passes")
        pp.add_argument("cmd")
        pp.add_argument("--pmc", action="append", required=True, help="counter_collection.csv of one pass")
        pp.add_argument("--title", default="VALU and LDS activity")
        pp.add_argument("--command", action="append", default=[])
        pp.add_argument("--out", required=True)
        a = pp.parse_args()
        write_pipes_md(a.out, a.title, a.pmc, a.command)
        return
    if len(os.sys.argv) > 1 and os.sys.argv[1] == "stats":
        sp = argparse.ArgumentParser(description="table of a rocprofv3 --stats kernel summary")
        sp.add_argument("cmd")
        sp.add_argument("--stats", required=True, help="rocprofv3 --stats kernel_stats.csv")
        sp.add_argument("--trace", default=None, help="the same run's kernel_trace.csv (per-grid table)")
        sp.add_argument("--title", default="Kernel statistics")
        sp.add_argument("--command", action="append", default=[])
        sp.add_argument("--out", required=True)
        a = sp.parse_args()
        write_stats_md(a.out, a.title, a.stats, a.command, trace_csv=a.trace)
        return
    if len(os.sys.argv) > 1 and os.sys.argv[1] == "trace":
        tp = argparse.ArgumentParser(description="summary of a graph-replay kernel trace")
        tp.add_argument("cmd")
        tp.add_argument("--trace", required=True, help="rocprofv3 --kernel-trace kernel_trace.csv")
        tp.add_argument("--steps", type=int, required=True)
        tp.add_argument("--ms-per-step", type=float, required=True, help="ms_per_step of the same run's bench line")
        tp.add_argument("--title", default="Kernel trace of the graph-replayed steps")
        tp.add_argument("--command", action="append", default=[])
        tp.add_argument("--out", required=True)
        a = tp.parse_args()
        write_trace_md(a.out, a.title, a.trace, a.steps, a.command, a.ms_per_step)
        return
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--stats", required=True, help="rocprofv3 --stats kernel_stats.csv")
    ap.add_argument("--fetch", required=True, help="counter_collection.csv of the FETCH_SIZE run")
    ap.add_argument("--write", required=True, help="counter_collection.csv of the WRITE_SIZE run")
    ap.add_argument("--fp64", default=None, help="counter_collection.csv of the SQ_INSTS_VALU_*_F64 run")
    ap.add_argument("--rdreq", default=None, help="counter_collection.csv of the TCC_EA0_RDREQ_{32B,64B,128B} run")
    ap.add_argument("--copy-bytes", type=int, default=256 * 1024 * 1024)
    ap.add_argument("--match", default="MHD2D")
    ap.add_argument("--title", default="Kernel durations and HBM traffic")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    s, ff, fw = summarize(a.stats, a.fetch, a.write, a.copy_bytes, a.match, a.fp64, a.rdreq)
    write_md(a.out, a.title, s, ff, fw, a.command, sources_digest())


if __name__ == "__main__":
    main()
