"""Short text summaries of rocprofv3 output, for the profiles/ folder.

  python -m paper_2403_12820_amd.profile_summary stats KERNEL_STATS.csv OUT.txt --command "..."
      per-kernel calls, average and total duration (from --kernel-trace --stats)

  python -m paper_2403_12820_amd.profile_summary sq --kernel NAME --nodes N --a A.csv --b B.csv \
      --command-a "..." --command-b "..." OUT.txt
      SQ and GRBM counters of one kernel (two --pmc passes), mean per dispatch, with derived
      rates: VALU lane-op slots per node, MFMA per 16 nodes, VALU and MFMA busy fractions and
      where the waves spend their time.

  python -m paper_2403_12820_amd.profile_summary traffic --kernel NAME[,NAME...] --nodes N \
      --fetch FETCH.csv --write WRITE.csv --copy-fetch CF.csv --copy-write CW.csv \
      --copy-bytes B OUT.txt --command-fetch "..." (and the other three commands)
      HBM bytes per launch of one kernel (or of each of several) from two --pmc runs (FETCH_SIZE,
      WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for a plain device
      copy of B bytes.

The traffic summary carries a hash of the kernel's sources; bench.py reports its figure only
while the sources still hash the same.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {
    "cnn_fwd_bf16": ("cnn_fwd_bf16.hip", "cnn_common.hpp", "common.hpp", "row_pieces.hpp"),
    "ms_step": ("ms_step.hip", "common.hpp", "row_pieces.hpp"),
    "cnn_bwd": ("cnn_bwd.hip", "cnn_bwd_tile.hip", "cnn_bwd_table.hpp", "cnn_common.hpp", "common.hpp"),
}


def source_hash(kind: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_summary(path: str) -> dict:
    """key: value lines of a summary file (other lines ignored)."""
    out = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def _stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["rocprofv3 kernel statistics", "command: " + args.command, "",
             "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[: args.top]:
        lines.append("| %s | %s | %.2f | %.3f | %.1f |" % (
            r["Name"].split("(")[0][:90], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, 100 * float(r["TotalDurationNs"]) / tot))
    if args.trace and args.tail_kernel:
        # the launches bench.py times alone with HIP events are the last ones of the kernel
        tr = sorted((r for r in csv.DictReader(open(args.trace)) if args.tail_kernel in r["Kernel_Name"]),
                    key=lambda r: int(r["Start_Timestamp"]))
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tr]
        if d:
            tail = d[-args.tail:]
            lines += ["", "last %d launches of %s (the event-timed repetitions): avg %.2f us; all %d: avg %.2f us, "
                      "min %.2f, max %.2f" % (len(tail), args.tail_kernel, sum(tail) / len(tail), len(d),
                                                sum(d) / len(d), min(d), max(d))]
    open(args.out, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path: str, name: str, counter: str):
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if name in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit("no %s dispatches of %s in %s" % (counter, name, path))
    return sum(vals) / len(vals), len(vals)


def _traffic(args):
    # the copy kernel: take its largest dispatch (the 1 GiB copy)
    cf = max(float(r["Counter_Value"]) for r in csv.DictReader(open(args.copy_fetch)) if r["Counter_Name"] == "FETCH_SIZE")
    cw = max(float(r["Counter_Value"]) for r in csv.DictReader(open(args.copy_write)) if r["Counter_Name"] == "WRITE_SIZE")
    kf, kw = args.copy_bytes / (cf * 1024), args.copy_bytes / (cw * 1024)
    kernels = args.kernel.split(",")
    head = [
        "command_fetch: " + args.command_fetch,
        "command_write: " + args.command_write,
        "command_copy_fetch: " + args.command_copy_fetch,
        "command_copy_write: " + args.command_copy_write,
    ]
    calib = [
        "copy_calibration: a %d-byte device copy reads FETCH_SIZE %.1f KiB and WRITE_SIZE %.1f KiB" % (
            args.copy_bytes, cf, cw),
        "fetch_factor: %.4f" % kf,
        "write_factor: %.4f" % kw,
    ]
    if len(kernels) == 1:
        f_kib, nf = _per_dispatch(args.fetch, args.kernel, "FETCH_SIZE")
        w_kib, nw = _per_dispatch(args.write, args.kernel, "WRITE_SIZE")
        fetch_b, write_b = f_kib * 1024 * kf, w_kib * 1024 * kw
        lines = ["HBM traffic per launch of %s (rocprofv3 --pmc)" % args.kernel] + head + [
            "kernel: %s" % args.kernel,
            "nodes: %d" % args.nodes,
            "dispatches: %d fetch, %d write" % (nf, nw),
            "fetch_kib_per_dispatch: %.1f" % f_kib,
            "write_kib_per_dispatch: %.1f" % w_kib,
        ] + calib + [
            "fetch_bytes: %.0f" % fetch_b,
            "write_bytes: %.0f" % write_b,
            "bytes_per_launch: %.0f" % (fetch_b + write_b),
            "bytes_per_node: %.2f" % ((fetch_b + write_b) / args.nodes),
        ]
    else:
        lines = ["HBM traffic per launch of each kernel of %s on %d nodes (rocprofv3 --pmc FETCH_SIZE and "
                 "WRITE_SIZE, each scaled by the same counter on a plain device copy)" % (args.what or args.kind,
                                                                                         args.nodes)] + head + calib
        total = 0.0
        for k in kernels:
            f_kib, _ = _per_dispatch(args.fetch, k, "FETCH_SIZE")
            w_kib, _ = _per_dispatch(args.write, k, "WRITE_SIZE")
            fb, wb = f_kib * 1024 * kf, w_kib * 1024 * kw
            total += fb + wb
            lines.append("%s: fetch %.0f B, write %.0f B, %.1f B per node" % (k, fb, wb, (fb + wb) / args.nodes))
        lines.append("bytes_per_node_all_kernels: %.1f" % (total / args.nodes))
    lines += ["note: " + n for n in args.note] + ["source_hash: %s" % source_hash(args.kind)]
    open(args.out, "w").write("\n".join(lines) + "\n")


def _sq(args):
    vals = {}
    for path in (args.a, args.b):
        per = {}
        for r in csv.DictReader(open(path)):
            if args.kernel in r["Kernel_Name"]:
                per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for k, v in per.items():
            vals[k] = sum(v) / len(v)
    n = args.nodes
    simds = args.simds
    act = vals["GRBM_GUI_ACTIVE"] / args.xcds
    lines = ["SQ and GRBM counters of %s (%s)" % (args.kernel, args.what),
             "command_a: " + args.command_a, "command_b: " + args.command_b,
             "note: mean over the dispatches of the kernel; SQ wave-cycle counters are in units of 4 cycles; "
             "%d XCDs x %d SIMDs" % (args.xcds, simds // args.xcds), ""]
    lines += ["%s: %.6g" % (k, vals[k]) for k in sorted(vals)]
    lines += ["", "derived:",
              "valu_lane_op_slots_per_node: %.0f  (SQ_INSTS_VALU x 64 / nodes)" % (vals["SQ_INSTS_VALU"] * 64 / n),
              "mfma_per_16_nodes: %.2f" % (vals["SQ_INSTS_MFMA"] * 16 / n),
              "valu_cycles_per_simd: %.0f  (SQ_INSTS_VALU x 4 / %d SIMDs)" % (vals["SQ_INSTS_VALU"] * 4 / simds, simds),
              "gpu_active_cycles_per_xcd: %.0f  (GRBM_GUI_ACTIVE / %d)" % (act, args.xcds),
              "valu_busy_fraction: %.2f" % (vals["SQ_INSTS_VALU"] * 4 / simds / act),
              "mfma_busy_fraction: %.2f  (SQ_VALU_MFMA_BUSY_CYCLES / %d SIMDs / active cycles)" % (
                  vals["SQ_VALU_MFMA_BUSY_CYCLES"] / simds / act, simds),
              "wave_time_waiting_on_waitcnt: %.2f  (SQ_WAIT_ANY / SQ_WAVE_CYCLES)" % (vals["SQ_WAIT_ANY"] / vals["SQ_WAVE_CYCLES"]),
              "wave_time_issuing: %.2f  (SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES)" % (
                  vals["SQ_ACTIVE_INST_ANY"] / vals["SQ_WAVE_CYCLES"]),
              "wave_time_waiting_for_issue: %.2f  (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES)" % (
                  vals["SQ_WAIT_INST_ANY"] / vals["SQ_WAVE_CYCLES"]),
              "source_hash: %s" % source_hash(args.kind)]
    open(args.out, "w").write("\n".join(lines) + "\n")


def _markers(args):
    """roctx ranges of a run (host time from push to pop), by name, in order of first use."""
    per, order = {}, []
    for r in csv.DictReader(open(args.csv)):
        name = r["Function"]
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        if name not in per:
            per[name] = []
            order.append(name)
        per[name].append(d)
    lines = ["roctx ranges (host time from push to pop)", "command: " + args.command, "",
             "| range | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for name in order:
        d = per[name]
        lines.append("| %s | %d | %.1f | %.1f | %.1f |" % (name, len(d), sum(d) / len(d), min(d), max(d)))
    lines += ["note: " + n for n in args.note]
    open(args.out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=16)
    s.add_argument("--trace", default=None, help="kernel_trace.csv of the same run")
    s.add_argument("--tail-kernel", default=None, help="kernel name substring for the tail average")
    s.add_argument("--tail", type=int, default=20)
    t = sub.add_parser("traffic")
    t.add_argument("out")
    t.add_argument("--kind", choices=sorted(KERNEL_SOURCES), required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--nodes", type=int, required=True)
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        t.add_argument("--" + k, required=True)
        t.add_argument("--command-" + k, required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--what", default="", help="workload named in the header of a several-kernel summary")
    t.add_argument("--note", action="append", default=[], help="a line of context (repeatable)")
    q = sub.add_parser("sq")
    q.add_argument("out")
    q.add_argument("--kind", choices=sorted(KERNEL_SOURCES), required=True)
    q.add_argument("--kernel", required=True)
    q.add_argument("--what", default="")
    q.add_argument("--nodes", type=int, required=True)
    q.add_argument("--a", required=True)
    q.add_argument("--b", required=True)
    q.add_argument("--command-a", required=True)
    q.add_argument("--command-b", required=True)
    q.add_argument("--simds", type=int, default=1024)
    q.add_argument("--xcds", type=int, default=8)
    m = sub.add_parser("markers")
    m.add_argument("csv", help="marker_api_trace.csv")
    m.add_argument("out")
    m.add_argument("--command", required=True)
    m.add_argument("--note", action="append", default=[], help="a line of context (repeatable)")
    a = ap.parse_args()
    {"stats": _stats, "traffic": _traffic, "sq": _sq, "markers": _markers}[a.cmd](a)


if __name__ == "__main__":
    main()
