"""Turn rocprofv3 output into short text summaries and the measured-traffic table.

Runs on the host, on CSV files that ``rocprofv3 --output-format csv`` wrote:

  stats    kernel-trace summary of one command: the busiest kernels, and the
           average duration of the dominant stencil launch (the same launches
           that the benchmark times with HIP events)
  counters per-dispatch averages of any counter sets for chosen kernels
  traffic  HBM bytes per launch of the dominant stencil from two counter runs
           (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by
           what the same counter reads for a plain copy kernel of known size
           run in the same process

    python -m paper_0704_2341_amd.profiling stats --trace DIR --bench-log LOG --command CMD
    python -m paper_0704_2341_amd.profiling traffic --fetch DIR --write DIR \
        --fetch-log LOG --write-log LOG --command CMD [--out JSON]

The benchmark's JSON line (in LOG) names the dominant launch (kernel symbol,
work-items per dispatch, launches in the timed region); the counter runs
select exactly those dispatches.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(PKG, "csrc", f)
                  for f in ("kernels_dslash.hip", "kernels_eo.hip", "stencil.h", "common.h")]
TRAFFIC_FILE = os.path.join(os.path.dirname(PKG), "profiles", "dslash_traffic.json")
COPY_KERNEL = "neg_kernel"  # torch's negation: reads N bytes, writes N bytes


def kernel_source_hash() -> str:
    """Fingerprint of the stencil sources; counter data taken on other
    sources is stale."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_key(prec: str, nrhs: int, dims, shape=None) -> str:
    """Name of a stencil launch in the traffic table: precision, RHS count,
    lattice and (optionally) the launch shape, since the bytes a launch moves
    depend on its shape."""
    key = f"{prec}_nrhs{nrhs}_{'x'.join(map(str, dims))}"
    return key + "_" + shape_tag(shape) if shape else key


def shape_tag(shape) -> str:
    return "_".join(f"{k}{shape[k]}" for k in ("SB", "RG", "split", "grid", "chunk", "march"))


def measured_traffic(key: str, path: str = TRAFFIC_FILE):
    """HBM bytes per launch of the stencil `key` (traffic_key) from the
    committed counter runs, or None when the stencil sources changed since
    they were taken."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    e = t.get("kernels", {}).get(key)
    return None if e is None else e.get("hbm_bytes_per_launch")


def _csv(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def bench_line(log: str) -> dict:
    """The benchmark's JSON line (the last line of LOG that parses as one)."""
    out = None
    with open(log) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                out = json.loads(line)
    if out is None:
        raise SystemExit(f"no benchmark JSON line in {log}")
    return out


def _grid_size(r) -> int:
    """Work-items of a dispatch (counter rows: Grid_Size; trace rows: X*Y*Z)."""
    if "Grid_Size" in r:
        return int(r["Grid_Size"])
    return int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])


def _select(rows, launch, key_id="Dispatch_Id"):
    """The last `launches` dispatches of the dominant launch (its symbol may
    name several kernel instances joined by ' + ', launched alternately)."""
    syms = [x.strip() for x in launch["symbol"].split(" + ")]
    gs, n = int(launch["grid_size"]), int(launch["launches"])
    hit = [r for r in rows if any(x in r["Kernel_Name"] for x in syms) and _grid_size(r) == gs]
    hit.sort(key=lambda r: int(r[key_id]))
    if not hit:
        raise SystemExit(f"no dispatch of {sym} with {gs} work-items")
    return hit[-n:]


def step_breakdown(tr, marker: str, steps: int, top: int = 12):
    """Per-step kernel time over the last `steps` steps of a trace, a step
    ending with the dispatch of the kernel named by `marker` (substring)."""
    tr = sorted(tr, key=lambda r: int(r["Start_Timestamp"]))
    ends = [i for i, r in enumerate(tr) if marker in r["Kernel_Name"]]
    if len(ends) < steps + 1:
        return None
    lo, hi = ends[-steps - 1] + 1, ends[-1] + 1
    agg = {}
    for r in tr[lo:hi]:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("|", "\\|")
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        n, t = agg.get(name, (0, 0))
        agg[name] = (n + 1, t + d)
    busy = sum(t for _, t in agg.values())
    wall = int(tr[hi - 1]["End_Timestamp"]) - int(tr[lo]["Start_Timestamp"])
    lines = [f"Per step over the last {steps} steps (a step ends with `{marker}`): "
             f"{busy / steps / 1e6:.2f} ms of kernels in {wall / steps / 1e6:.2f} ms.", "",
             "| kernel | launches per step | avg us | ms per step | % of kernel time |",
             "|---|---:|---:|---:|---:|"]
    for name, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"| `{name}` | {n / steps:.0f} | {t / n / 1e3:.1f} | {t / steps / 1e6:.2f} | "
                     f"{100 * t / busy:.1f} |")
    return lines


def stats_summary(trace_dir: str, bench_log: str, command: str, top: int = 15, marker: str = "") -> str:
    b = bench_line(bench_log)
    launch = b["roofline"]["launch"]
    st = _csv(trace_dir, "_kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in st)
    lines = ["# rocprofv3 kernel trace: " + b["config"]["workload"], "",
             "Command (from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", "",
             "    " + command, "",
             f"Bench line of this run: {b['value']:.1f} {b['unit']}, {b['ms_per_step']:.2f} ms/step "
             f"({b['steps']} steps); the run also includes the stencil autotuner"
             + (" and the FP64 GCR leg." if b.get("fp64_gcr") else "."), "",
             f"| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(st, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        name = r["Name"].split("(")[0].replace("void ", "").replace("|", "\\|")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    lines.append(f"| (all kernels) | | | {tot / 1e6:.1f} | 100 |")
    tr = _csv(trace_dir, "_kernel_trace.csv")
    sel = _select(tr, launch)
    avg = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in sel) / len(sel) / 1e6
    live = b["roofline"]["avg_launch_ms"]
    lines += ["", f"Dominant launch `{launch['symbol']}` ({launch['grid_size']} work-items, "
                  f"launch {launch['shape']}): last {len(sel)} dispatches (the timed region) "
                  f"average {avg * 1e3:.1f} us in the trace; the benchmark's HIP events on the "
                  f"launch stream measured {live * 1e3:.1f} us per launch in the same run "
                  f"({100 * (avg / live - 1):+.1f} %).",
              f"Algorithmic bytes per launch {b['roofline']['alg_bytes_per_launch']:,}: "
              f"{b['roofline']['alg_bytes_per_launch'] / avg / 1e6:.0f} GB/s on the trace's average."]
    if marker:
        steps = step_breakdown(tr, marker, int(b["steps"]))
        if steps:
            lines += [""] + steps
    return "\n".join(lines) + "\n"


def _copy_factor(rows, copy_bytes: int, counter: str):
    hit = [r for r in rows if COPY_KERNEL in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not hit:
        raise SystemExit(f"no {COPY_KERNEL} dispatch with {counter}")
    gs = max(_grid_size(r) for r in hit)
    vals = [float(r["Counter_Value"]) for r in hit if _grid_size(r) == gs]
    kib = sum(vals) / len(vals)
    return copy_bytes / (kib * 1024.0), kib, len(vals)


def _counter_avg(rows, launch, counter: str):
    rows = [r for r in rows if r["Counter_Name"] == counter]
    sel = _select(rows, launch)
    return sum(float(r["Counter_Value"]) for r in sel) / len(sel), len(sel)


def traffic_table(fetch_dir, write_dir, fetch_log, write_log, command, out=TRAFFIC_FILE):
    bf, bw = bench_line(fetch_log), bench_line(write_log)
    launch = bf["roofline"]["launch"]
    if bw["roofline"]["launch"] != launch:
        raise SystemExit("the two counter runs timed different launches")
    cb = int(bf["calibration_copy_bytes"])
    fr, wr = _csv(fetch_dir, "_counter_collection.csv"), _csv(write_dir, "_counter_collection.csv")
    ff, fk, fn = _copy_factor(fr, cb, "FETCH_SIZE")
    wf, wk, wn = _copy_factor(wr, cb, "WRITE_SIZE")
    fetch, nf = _counter_avg(fr, launch, "FETCH_SIZE")
    write, nw = _counter_avg(wr, launch, "WRITE_SIZE")
    hbm = fetch * 1024 * ff + write * 1024 * wf
    key = bf["roofline"]["traffic_key"]
    tag = shape_tag(launch["shape"])
    if not key.endswith(tag):
        key += "_" + tag
    alg = bf["roofline"]["alg_bytes_per_launch"]
    entry = {"symbol": launch["symbol"], "grid_size": launch["grid_size"], "shape": launch["shape"],
             "dispatches": [nf, nw], "fetch_kib": fetch, "write_kib": write,
             "hbm_bytes_per_launch": hbm, "alg_bytes_per_launch": alg, "ratio_to_alg": hbm / alg,
             "command": command}
    table = {"kernel_source_sha256": kernel_source_hash(),
             "calibration": {"kernel": COPY_KERNEL, "bytes_read": cb, "bytes_written": cb,
                             "fetch_kib": fk, "write_kib": wk, "fetch_factor": ff, "write_factor": wf,
                             "dispatches": [fn, wn]},
             "kernels": {}}
    if os.path.exists(out):
        with open(out) as f:
            old = json.load(f)
        if old.get("kernel_source_sha256") == table["kernel_source_sha256"]:
            table["kernels"] = old.get("kernels", {})
    table["kernels"][key] = entry
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    return table, key


def counters_summary(dirs, kernels, command_lines, title, note=""):
    """Average of every counter per dispatch, per kernel (name substring)
    and grid, over the counter runs in `dirs` (one counter set per run)."""
    rows = []
    for d in dirs:
        rows.extend(_csv(d, "_counter_collection.csv"))
    agg = {}
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        if not any(k in name for k in kernels):
            continue
        key = (name, _grid_size(r), r["Counter_Name"])
        agg.setdefault(key, []).append(float(r["Counter_Value"]))
    lines = ["# " + title, "", "Commands (from the repository root, `cd /tmp && export TMPDIR=/tmp` "
             "first), one counter set per run:", ""]
    lines += ["    " + c for c in command_lines]
    lines += ["", note, "", "| kernel | work-items | dispatches | counter | average |", "|---|---:|---:|---|---:|"]
    for (name, gs, cn), v in sorted(agg.items()):
        lines.append(f"| `{name.replace('|', '/')}` | {gs} | {len(v)} | {cn} | {sum(v) / len(v):.4g} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--bench-log", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--step-marker", default="",
                   help="kernel name (substring) whose dispatch ends a step: adds a per-step breakdown")
    s.add_argument("--out")
    t = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--fetch-log", "--write-log", "--command"):
        t.add_argument(k, required=True)
    t.add_argument("--out", default=TRAFFIC_FILE)
    c = sub.add_parser("counters")
    c.add_argument("--dirs", nargs="+", required=True)
    c.add_argument("--kernels", nargs="+", required=True)
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--note", default="")
    c.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        text = counters_summary(a.dirs, a.kernels, a.command, a.title, a.note)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
        return
    if a.cmd == "stats":
        text = stats_summary(a.trace, a.bench_log, a.command, marker=a.step_marker)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
    else:
        table, key = traffic_table(a.fetch, a.write, a.fetch_log, a.write_log, a.command, a.out)
        e, c = table["kernels"][key], table["calibration"]
        print(f"{key}: {e['hbm_bytes_per_launch'] / 1e9:.3f} GB per launch "
              f"({e['ratio_to_alg']:.2f}x algorithmic); copy factors fetch {c['fetch_factor']:.3f}, "
              f"write {c['write_factor']:.3f}")


if __name__ == "__main__":
    main()
