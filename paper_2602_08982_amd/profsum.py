"""Summaries of rocprofv3 output as short Markdown text.

    python -m paper_2602_08982_amd.profsum stats  RUN_kernel_stats.csv OUT.md --command "..."
    python -m paper_2602_08982_amd.profsum counters FETCH.csv WRITE.csv OUT.md --command "..."

`stats` tabulates calls / total / average duration per kernel.  `counters`
turns the per-dispatch FETCH_SIZE and WRITE_SIZE readings (KiB) into HBM
bytes per launch: each counter is scaled by the factor that maps its reading
for the run's 4 GiB device-to-device copy (the largest dispatch of the
library's k_stream_copy, or of the runtime's __amd_rocclr_copyBuffer, 2^32
bytes read and 2^32 bytes written) onto those known sizes.
The counters summary records a digest of the 3D kernel sources and build
flags so that a reader (bench.py) can tell whether the figures still describe
the kernels as built.
"""
import argparse
import collections
import csv
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources of the 3D kernels that the recorded counters cover
KERNEL_SOURCES = ["csrc/kernels3d.h", "csrc/kernels3d_gen.h", "csrc/engine3d.h", "csrc/bufio.h", "csrc/fft.h", "build.py"]
COPY_BYTES = 1 << 32

LAP2_MODES = {0: "lap2_h", 1: "lap2_f", 2: "lap2_corr", 3: "lap2_full", 4: "lap2_taylor"}
PW_MODES = {0: "norm", 1: "pred"}


def sources_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def role(name):
    """Short role of a 3D-path kernel (the names bench.py reports), else None."""
    m = re.search(r"k_lap2<(\w+), \d+, \d+, \d+, (\d)", name)
    if m:
        return LAP2_MODES[int(m.group(2))]
    m = re.search(r"k_pointwise<(\w+), \d+, \d+, \d+, (\d)", name)
    if m:
        return PW_MODES.get(int(m.group(2)), "scale")
    m = re.search(r"q_lap2<\w+, \d+, \d+, (\d)", name)
    if m:
        return "q1d_" + LAP2_MODES[int(m.group(1))]
    m = re.search(r"q_gen<\w+, \d+, \d+, (\d)", name)
    if m:
        return "q1dgen_" + {**LAP2_MODES, 5: "lap1"}[int(m.group(1))]
    m = re.search(r"k_opline<\w+, \d+, \d+, \d+, (\d)", name)
    if m:
        return "gen3d_opline_" + "xyz"[int(m.group(1))]
    m = re.search(r"k_pw_gen<\w+, \d+, \d+, \d+, (\d)", name)
    if m:
        return "gen3d_" + LAP2_MODES[int(m.group(1))]
    m = re.search(r"q2_lap<\w+, \d+, \d+, (\d)", name)
    if m:
        return "q2d_" + {**LAP2_MODES, 5: "lap1"}[int(m.group(1))]
    m = re.search(r"q_pointwise<\w+, \d+, \d+, (\d)", name)
    if m:
        return "q1d_" + PW_MODES.get(int(m.group(1)), "scale")
    for pat, r in (("k_lap1<", "lap1"), ("k_dens_sum<", "dens"), ("k_dens<", "dens_kin"),
                   ("k_reduce_pot", "reduce_pot"), ("k_finalize", "finalize"), ("q_lap1<", "q1d_lap1"),
                   ("q_dens<", "q1d_dens_kin"), ("q_corr_split<", "q1d_lap2_corr"), ("q_fric<", "q1d_friction"),
                   ("q_densj<", "q1dgen_dens"), ("q_reduce_gen<", "q1dgen_reduce_pot"),
                   ("q_jz<", "q1dgen_dens"), ("q_taujs<", "q1das_dens"), ("q_reduce_aslda<", "q1das_reduce_pot"),
                   ("q2_kz_tau<", "q2d_grad"), ("k_jline<", "gen3d_jline"), ("k_reduce_gen3d<", "gen3d_reduce_pot"),
                   ("k_taujline<", "as3d_taujline"), ("k_reduce_aslda3d<", "as3d_reduce_pot"),
                   ("k_bpline<", "fric3d_bpline"),
                   ("k_grad_axis<", "grad"), ("k_grad_reduce", "grad_reduce"),
                   ("k_stream_copy", "stream_copy"), ("k_stream_read", "stream_read")):
        if pat in name:
            return r
    return None


def precision(name):
    m = re.search(r"<(double|float)\b", name)
    return m.group(1) if m else ""


def key(name):
    """precision:extent:role of a path kernel (extent = the first integer
    template argument: x extent of the 3D kernels, A of the quasi-1D ones,
    the state-group size of the density-sum pass), else None."""
    rl = role(name)
    if rl is None:
        return None
    m = re.search(r"<(?:double|float), (\d+)", name)
    nx = m.group(1) if m and rl not in ("reduce_pot", "finalize") else "-"
    return f"{precision(name)}:{nx}:{rl}"


def short(name, width=72):
    n = name.replace("tdslda::", "").replace("void ", "")
    return n if len(n) <= width else n[:width - 3] + "..."


def cmd_stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    out = [f"# {args.title}", "", "Command (from the repository root, on one MI355X):", "",
           "    " + args.command, "", "| kernel | role | calls | total ms | avg ms | % |",
           "|---|---|---:|---:|---:|---:|"]
    # every kernel of the path (those with a role), and the others down to
    # the args.others-th by total time
    others, skipped, skipped_ms = 0, 0, 0.0
    for r in rows:
        nm = r["Name"]
        rl = role(nm)
        small = float(r["Percentage"]) < args.min_pct
        if rl is None:
            others += 1
        if (rl is None and others > args.others) or small:
            skipped += 1
            skipped_ms += int(r["TotalDurationNs"]) / 1e6
            continue
        rl = f"{rl} ({precision(nm)})" if rl else ""
        out.append(f"| `{short(nm)}` | {rl} | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e6:.3f} | {r['Percentage']} |")
    if skipped:
        out += ["", f"{skipped} further kernels (outside the path, or below {args.min_pct}% of the time; "
                    f"{skipped_ms:.1f} ms in total) are not listed."]
    if args.note:
        out += ["", args.note]
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")


def _per_kernel(path):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    return agg


def _copy_factor(agg):
    """The library's streaming copy of 4 GiB (its largest k_stream_copy
    dispatch; else the runtime's largest copyBuffer dispatch)."""
    for pat in ("k_stream_copy", "copyBuffer"):
        copies = [v for k, vals in agg.items() if pat in k for v in vals]
        if copies:
            return COPY_BYTES / max(copies)
    raise SystemExit("no 4 GiB copy dispatch in the counter file")


def cmd_counters(args):
    fetch, write = _per_kernel(args.fetch), _per_kernel(args.write)
    ff, fw = _copy_factor(fetch), _copy_factor(write)
    out = [f"# {args.title}", "", "Commands (from the repository root, on one MI355X):", ""]
    out += ["    " + c for c in args.command]
    out += ["", f"Calibration: the 4 GiB device-to-device copy reads {COPY_BYTES} bytes and writes "
                f"{COPY_BYTES}; its FETCH_SIZE reading x {ff:.4f} and its WRITE_SIZE reading x {fw:.4f} "
                "give those sizes, and every kernel's readings are scaled by the same factors.", "",
            "| kernel | role | dispatches | HBM read GB / launch | HBM written GB / launch |",
            "|---|---|---:|---:|---:|"]
    machine = []
    for nm in sorted(fetch, key=lambda k: -sum(fetch[k]) / len(fetch[k])):
        rl = role(nm)
        if rl is None:
            continue
        rd = ff * sum(fetch[nm]) / len(fetch[nm])
        wr = fw * sum(write.get(nm, [0.0])) / max(1, len(write.get(nm, [])))
        out.append(f"| `{short(nm)}` | {rl} ({precision(nm)}) | {len(fetch[nm])} | {rd / 1e9:.3f} | "
                   f"{wr / 1e9:.3f} |")
        machine.append(f"traffic {key(nm)} {rd + wr:.6e}")
    out += ["", "Machine-readable lines (bytes per launch, read + written; sources digest of the "
                "kernel sources and build flags the counters were taken with):", ""]
    out += ["    " + m for m in machine]
    out += [f"    sources {sources_digest()}"]
    if args.note:
        out += ["", args.note]
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")


def read_traffic(md_path, prec, nx, kernel):
    """Bytes per launch recorded for the kernel (precision "double" / "float",
    x extent, role), or None when the file is missing or the kernel sources
    changed since it was written."""
    if not os.path.exists(md_path):
        return None
    val, src = None, None
    want = f"{prec}:{nx}:{kernel}"
    for line in open(md_path):
        p = line.split()
        if len(p) == 3 and p[0] == "traffic" and p[1] == want:
            val = float(p[2])
        if len(p) == 2 and p[0] == "sources":
            src = p[1]
    return val if src == sources_digest() else None


SQ_ROLES = ("lap2_corr", "lap2_full", "lap1", "dens", "stream_copy")


def cmd_sq(args):
    """Per-kernel SQ counters of one --pmc pass (waves, wave-cycles, VALU and
    LDS activity, LDS bank conflicts, GRBM_GUI_ACTIVE), summed over the
    dispatches of each role and normalised by the dispatches' own durations.
    The wave-cycle and active-instruction counters count quad-cycles (x4);
    GRBM_GUI_ACTIVE sums the 8 XCDs."""
    rows = list(csv.DictReader(open(args.csv)))
    agg, dur, disp, name = {}, {}, {}, {}
    seen = set()
    for r in rows:
        k = key(r["Kernel_Name"])
        if k is None or k.split(":")[2] not in SQ_ROLES:
            continue
        a = agg.setdefault(k, {})
        a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        if (k, r["Dispatch_Id"]) not in seen:
            seen.add((k, r["Dispatch_Id"]))
            dur[k] = dur.get(k, 0) + int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            disp[k] = disp.get(k, 0) + 1
            name[k] = r["Kernel_Name"]
    out = [f"# {args.title}", "", "Commands (from the repository root, on one MI355X):", ""]
    out += ["    " + c for c in args.command]
    out += ["", "Per role: the counters summed over its dispatches; cycles = the dispatches' durations x the "
            "GRBM_GUI_ACTIVE clock (GRBM_GUI_ACTIVE / 8 XCDs / duration). waves/CU = 4 SQ_WAVE_CYCLES / (256 CUs "
            "cycles); VALU busy = 4 SQ_ACTIVE_INST_VALU / (1024 SIMDs cycles); LDS busy = 4 SQ_ACTIVE_INST_LDS / "
            "(256 CUs cycles); bank-conflict rate = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS.", "",
            "| kernel | role | dispatches | avg ms | clock GHz | waves/CU | VALU busy | VALU instr/wave | LDS busy | "
            "LDS bank-conflict rate |", "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(agg, key=lambda k: (k.split(":")[2], k)):
        a, n, t = agg[k], disp[k], dur[k] * 1e-9
        clk = a.get("GRBM_GUI_ACTIVE", 0.0) / 8 / t  # cycles per second
        cyc = clk * t
        wav = 4 * a.get("SQ_WAVE_CYCLES", 0.0) / (256 * cyc)
        valu = 4 * a.get("SQ_ACTIVE_INST_VALU", 0.0) / (1024 * cyc)
        lds = 4 * a.get("SQ_ACTIVE_INST_LDS", 0.0) / (256 * cyc)
        ipw = a.get("SQ_INSTS_VALU", 0.0) / max(1.0, a.get("SQ_WAVES", 0.0))
        bc = a.get("SQ_LDS_BANK_CONFLICT", 0.0) / a["SQ_ACTIVE_INST_LDS"] if a.get("SQ_ACTIVE_INST_LDS") else 0.0
        out.append(f"| `{short(name[k])}` | {k.split(':')[2]} ({k.split(':')[0]}) | {n} | {1e3 * t / n:.3f} | "
                   f"{clk / 1e9:.2f} | {wav:.1f} | {valu:.2f} | {ipw:.0f} | {lds:.3f} | {bc:.3f} |")
    if args.note:
        out += ["", args.note]
    open(args.out, "w").write("\n".join(out) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="Kernel trace")
    s.add_argument("--note", default="")
    s.add_argument("--others", type=int, default=12, help="kernels outside the path to list")
    s.add_argument("--min-pct", type=float, default=0.05, help="list no kernel below this share of the time")
    c = sub.add_parser("counters")
    c.add_argument("fetch")
    c.add_argument("write")
    c.add_argument("out")
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--title", default="HBM traffic counters")
    c.add_argument("--note", default="")
    q = sub.add_parser("sq")
    q.add_argument("csv")
    q.add_argument("out")
    q.add_argument("--command", action="append", required=True)
    q.add_argument("--title", default="SQ counters")
    q.add_argument("--note", default="")
    a = ap.parse_args()
    {"stats": cmd_stats, "counters": cmd_counters, "sq": cmd_sq}[a.cmd](a)


if __name__ == "__main__":
    main()
