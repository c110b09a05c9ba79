"""Turn rocprofv3 CSV output into the short text summaries kept with the project.

  python -m paper_1807_03749_amd.profile_summary stats <run>_kernel_stats.csv --command "..." --out FILE
      per-kernel dispatch statistics (calls, total / average / min / max duration, share)

  python -m paper_1807_03749_amd.profile_summary trace <run>_kernel_trace.csv --steps K --command "..." --out FILE
      the same statistics from a per-dispatch kernel trace, over the last K steps only (a step
      ends with its k_final_part dispatch), so that the growth of the population before the
      timed steps does not enter them

  python -m paper_1807_03749_amd.profile_summary traffic --kernel k_generate --name generate
      --workload W --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv
      --copy-bytes N --command "..." --out FILE [--last K]
      HBM bytes per dispatch of one kernel: FETCH_SIZE and WRITE_SIZE (KiB per dispatch,
      averaged over its dispatches, or over its last K dispatches: the steps at the workload's
      population, after the growth phase), each scaled by expected / measured of the same
      counter on device copies of N bytes (a read of N and a write of N bytes per copy).  With
      a comma-separated --kernel list the figure is per step: the listed kernels' bytes summed
      over their dispatches of the last K steps (one step = one dispatch of the first kernel).

  python -m paper_1807_03749_amd.profile_summary valu --pmc P.csv --kernels k_items,k_generate
      --simds 1024 --xcds 8 --workload W --command "..." --out FILE
      vector-ALU use per kernel from one counter pass (SQ_WAVES, SQ_INSTS_VALU,
      SQ_ACTIVE_INST_VALU, SQ_WAVE_CYCLES, SQ_WAIT_INST_ANY, GRBM_GUI_ACTIVE): VALU instructions
      per wave, VALU busy = 4 SQ_ACTIVE_INST_VALU / (SIMDs x GRBM_GUI_ACTIVE / XCDs) (the
      active-instruction counter counts in units of four cycles, the wave64 issue time on a
      16-lane SIMD; GRBM_GUI_ACTIVE arrives summed over the XCDs), and the fraction of wave
      time spent waiting.

  python -m paper_1807_03749_amd.profile_summary gaps <run>_kernel_trace.csv --steps K
      [--api <run>_hip_api_trace.csv] --command "..." --out FILE
      the idle time of the GPU between consecutive kernels over the last K steps (median per
      pair of kernels, and the sum per step), and with an API trace the host's time per
      hipLaunchKernel call: where the host issues launches more slowly than the kernels run,
      the GPU waits between them

The summaries record the hash of the HIP sources they were taken on; bench.py uses a
traffic figure only while that hash still matches.
"""
from __future__ import annotations

import argparse
import csv
import datetime
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    n = name.replace("void ", "").replace("ccmc::", "")
    depth, out = 0, []
    for ch in n:  # drop the parameter list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _source_hash() -> str:
    sys.path.insert(0, ROOT)
    import bench  # noqa: E402  (the hash function lives with its only reader)
    return bench.source_hash()


def stats(args):
    rows = _rows(args.csv)
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics  ({datetime.date.today().isoformat()})",
             f"# command: {args.command}",
             f"# source_hash = {_source_hash()}",
             f"# {'kernel':58s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'share':>6s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        t = float(r["TotalDurationNs"])
        lines.append(f"  {_short(r['Name'])[:58]:58s} {int(r['Calls']):7d} {t / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {100 * t / tot:5.1f}%")
    _write(args.out, lines)


def trace(args):
    rows = _rows(args.csv)
    for r in rows:
        r["_s"], r["_e"] = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
    rows.sort(key=lambda r: r["_s"])
    ends = [r["_e"] for r in rows if "k_final_part" in r["Kernel_Name"]]
    if len(ends) < args.steps + 1:
        raise SystemExit(f"trace: {len(ends)} steps in the trace, fewer than {args.steps} + 1")
    t0 = ends[-args.steps - 1]
    agg = {}
    for r in rows:
        if r["_s"] < t0:
            continue
        d = r["_e"] - r["_s"]
        a = agg.setdefault(_short(r["Kernel_Name"]), [0, 0, 1 << 62, 0])
        a[0] += 1
        a[1] += d
        a[2] = min(a[2], d)
        a[3] = max(a[3], d)
    tot = sum(a[1] for a in agg.values())
    lines = [f"# rocprofv3 kernel statistics over the last {args.steps} steps  ({datetime.date.today().isoformat()})",
             f"# command: {args.command}",
             f"# source_hash = {_source_hash()}",
             f"# {'kernel':58s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'share':>6s}",]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"  {k[:58]:58s} {a[0]:7d} {a[1] / 1e6:10.3f} {a[1] / a[0] / 1e3:9.2f} {a[2] / 1e3:9.2f} "
                     f"{a[3] / 1e3:9.2f} {100 * a[1] / tot:5.1f}%")
    lines.append(f"# per step: {tot / 1e3 / args.steps:.1f} us of kernel time")
    _write(args.out, lines)


def gaps(args):
    rows = _rows(args.csv)
    for r in rows:
        r["_s"], r["_e"] = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
    rows.sort(key=lambda r: r["_s"])
    ends = [r["_e"] for r in rows if "k_final_part" in r["Kernel_Name"]]
    if len(ends) < args.steps + 1:
        raise SystemExit(f"gaps: {len(ends)} steps in the trace, fewer than {args.steps} + 1")
    t0 = ends[-args.steps - 1]
    rows = [r for r in rows if r["_s"] >= t0 and not r["Kernel_Name"].startswith("__amd")]
    pairs, idle = {}, 0
    for a, b in zip(rows, rows[1:]):
        g = max(0, b["_s"] - a["_e"])
        idle += g
        key = (_short(a["Kernel_Name"]).split("<")[0], _short(b["Kernel_Name"]).split("<")[0])
        pairs.setdefault(key, []).append(g)
    lines = [f"# idle GPU time between kernels over the last {args.steps} steps  ({datetime.date.today().isoformat()})",
             f"# command: {args.command}",
             f"# source_hash = {_source_hash()}",
             f"# {'kernel':>20s} -> {'next kernel':20s} {'count':>6s} {'median_gap_us':>14s}"]
    for (x, y), v in sorted(pairs.items(), key=lambda kv: -sorted(kv[1])[len(kv[1]) // 2]):
        v = sorted(v)
        lines.append(f"  {x:>20s} -> {y:20s} {len(v):6d} {v[len(v) // 2] / 1e3:14.2f}")
    lines.append(f"# per step: {idle / 1e3 / args.steps:.1f} us idle between kernels")
    if args.api:
        launch = {}
        for r in _rows(args.api):
            if r["Function"] == "hipLaunchKernel" and int(r["Start_Timestamp"]) >= t0 - 10**9:
                launch[r["Correlation_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        d = sorted(launch[r["Correlation_Id"]] for r in rows if r.get("Correlation_Id") in launch)
        if d:
            lines.append(f"# hipLaunchKernel host time per launch (under the API tracer): median {d[len(d) // 2] / 1e3:.2f} us "
                         f"over {len(d)} launches")
    _write(args.out, lines)


def _per_dispatch(path, counter, match):
    vals = {}
    for r in _rows(path):
        if r["Counter_Name"] != counter or not match(r["Kernel_Name"]):
            continue
        vals[r["Dispatch_Id"]] = vals.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return [vals[k] for k in sorted(vals, key=int)]  # in dispatch order


def traffic(args):
    names = [k for k in args.kernel.split(",") if k]
    copy = lambda n: "copy" in n.lower()
    cf = _per_dispatch(args.copy_fetch, "FETCH_SIZE", copy)
    cw = _per_dispatch(args.copy_write, "WRITE_SIZE", copy)
    exp_kib = args.copy_bytes * args.copy_reps / 1024.0
    if not (cf and cw):
        raise SystemExit("traffic: a copy counter file holds no copy dispatch")
    sf, sw = exp_kib / sum(cf), exp_kib / sum(cw)
    f, w = [], []
    steps = None
    for i, k in enumerate(names):
        fk = _per_dispatch(args.fetch, "FETCH_SIZE", lambda n, k=k: k in n)
        wk = _per_dispatch(args.write, "WRITE_SIZE", lambda n, k=k: k in n)
        if not (fk and wk):
            raise SystemExit(f"traffic: no dispatch of {k}")
        if len(names) > 1:  # per step: the last K steps' dispatches of each kernel
            if i == 0:
                steps = min(args.last or len(fk), len(fk))
            per = max(1, round(len(fk) / len(_per_dispatch(args.fetch, "FETCH_SIZE", lambda n: names[0] in n))))
            fk, wk = fk[-steps * per:], wk[-steps * per:]
        elif args.last:
            fk, wk = fk[-args.last:], wk[-args.last:]
        f.append(fk)
        w.append(wk)
    if len(names) > 1:
        fk = sum(sum(x) for x in f) / steps
        wk = sum(sum(x) for x in w) / steps
        f, w = [None] * steps, [None] * steps
    else:
        f, w = f[0], w[0]
        fk, wk = sum(f) / len(f), sum(w) / len(w)
    hbm = (fk * sf + wk * sw) * 1024.0
    lines = [f"# HBM traffic of {args.kernel} ({args.name}) on {args.workload}  ({datetime.date.today().isoformat()})",
             f"# command: {args.command}",
             f"source_hash = {_source_hash()}",
             f"{'steps' if len(names) > 1 else 'dispatches'}_fetch = {len(f)}",
             f"{'steps' if len(names) > 1 else 'dispatches'}_write = {len(w)}",
             f"fetch_kib_per_{'step' if len(names) > 1 else 'dispatch'} = {fk:.1f}",
             f"write_kib_per_{'step' if len(names) > 1 else 'dispatch'} = {wk:.1f}",
             f"copy_bytes = {args.copy_bytes} x {args.copy_reps} copies",
             f"copy_fetch_kib_measured = {sum(cf):.1f}  (expected {exp_kib:.1f}, scale {sf:.4f})",
             f"copy_write_kib_measured = {sum(cw):.1f}  (expected {exp_kib:.1f}, scale {sw:.4f})",
             f"hbm_bytes_per_{'step' if len(names) > 1 else 'launch'} = {hbm:.0f}"]
    _write(args.out, lines)


def valu(args):
    names = [k for k in args.kernels.split(",") if k]
    counters = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY",
                "GRBM_GUI_ACTIVE")
    lines = [f"# vector-ALU use on {args.workload}  ({datetime.date.today().isoformat()})"
             + (f", last {args.last} dispatches of each kernel" if args.last else ""),
             f"# command: {args.command}",
             f"source_hash = {_source_hash()}",
             f"simds = {args.simds}, xcds = {args.xcds} (GRBM_GUI_ACTIVE is divided by the XCDs)",
             f"# {'kernel':12s} {'dispatches':>10s} {'waves':>9s} {'valu_insts/wave':>16s} {'valu_busy':>10s} {'wait/wave_cycles':>17s}"]
    for k in names:
        per = {c: _per_dispatch(args.pmc, c, lambda n, k=k: k in n) for c in counters}
        if not per["SQ_WAVES"]:
            raise SystemExit(f"valu: no dispatch of {k}")
        if args.last:  # the last K dispatches of the kernel (the timed steps)
            per = {c: v[-args.last:] for c, v in per.items()}
        av = {c: sum(v) / len(v) for c, v in per.items() if v}
        busy = 4.0 * av["SQ_ACTIVE_INST_VALU"] / (args.simds * av["GRBM_GUI_ACTIVE"] / args.xcds)
        lines.append(f"  {k:12s} {len(per['SQ_WAVES']):10d} {av['SQ_WAVES']:9.0f} "
                     f"{av['SQ_INSTS_VALU'] / av['SQ_WAVES']:16.1f} {100 * busy:9.1f}% "
                     f"{100 * av['SQ_WAIT_INST_ANY'] / av['SQ_WAVE_CYCLES']:16.1f}%")
    _write(args.out, lines)


def _write(out, lines):
    text = "\n".join(lines) + "\n"
    if out:
        with open(out, "w") as f:
            f.write(text)
    print(text, end="")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--out")
    t = sub.add_parser("traffic")
    for a in ("--kernel", "--name", "--workload", "--fetch", "--write", "--copy-fetch", "--copy-write", "--command"):
        t.add_argument(a, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--copy-reps", type=int, default=5)
    t.add_argument("--last", type=int, default=0)
    t.add_argument("--out")
    r = sub.add_parser("trace")
    r.add_argument("csv")
    r.add_argument("--steps", type=int, required=True)
    r.add_argument("--command", required=True)
    r.add_argument("--out")
    g = sub.add_parser("gaps")
    g.add_argument("csv")
    g.add_argument("--steps", type=int, required=True)
    g.add_argument("--api")
    g.add_argument("--command", required=True)
    g.add_argument("--out")
    v = sub.add_parser("valu")
    for a in ("--pmc", "--kernels", "--workload", "--command"):
        v.add_argument(a, required=True)
    v.add_argument("--simds", type=int, default=1024)
    v.add_argument("--xcds", type=int, default=8)
    v.add_argument("--last", type=int, default=0)
    v.add_argument("--out")
    args = ap.parse_args()
    {"stats": stats, "trace": trace, "traffic": traffic, "valu": valu, "gaps": gaps}[args.cmd](args)


if __name__ == "__main__":
    main()
