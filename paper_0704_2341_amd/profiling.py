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
  stencil-table  the same for every launch of the benchmark's stencil table

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
        raise SystemExit(f"no dispatch of {launch['symbol']} with {gs} work-items")
    return hit[-n:]


def step_breakdown(tr, marker: str, steps: int, top: int = 12):
    """Per-step kernel time over the last `steps` steps of a trace, a step
    ending with the dispatch of the kernel named by `marker` (substring)."""
    tr = sorted(tr, key=lambda r: int(r["Start_Timestamp"]))
    name, _, gs = marker.partition(":")
    ends = [i for i, r in enumerate(tr) if name in r["Kernel_Name"] and (not gs or _grid_size(r) == int(gs))]
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


def stats_summary(trace_dir: str, bench_log: str, command: str, top: int = 15, marker: str = "",
                  steps: int = 0, title: str = "") -> str:
    b = bench_line(bench_log)
    launch = b["roofline"]["launch"]
    st = _csv(trace_dir, "_kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in st)
    lines = ["# rocprofv3 kernel trace: " + (title or b["config"]["workload"]), "",
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
        st = step_breakdown(tr, marker, steps or int(b["steps"]))
        if st:
            lines += [""] + st
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


def _first_copy(rows, counter):
    ids = [int(r["Dispatch_Id"]) for r in rows if COPY_KERNEL in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not ids:
        raise SystemExit(f"no {COPY_KERNEL} dispatch with {counter}")
    return min(ids)


def _window_avg(rows, launch, counter, after):
    """Average of `counter` over the `launches` timed dispatches of `launch`
    that follow its warm-up dispatch, the first match after dispatch `after`;
    returns (average, id of the last dispatch taken)."""
    syms = [x.strip() for x in launch["symbol"].split(" + ")]
    gs, n = int(launch["grid_size"]), int(launch["launches"])
    hit = sorted((r for r in rows if r["Counter_Name"] == counter and int(r["Dispatch_Id"]) > after
                  and any(x in r["Kernel_Name"] for x in syms) and _grid_size(r) == gs),
                 key=lambda r: int(r["Dispatch_Id"]))[1:n + 1]
    if len(hit) < n:
        raise SystemExit(f"only {len(hit)} dispatches of {launch['symbol']} ({gs} work-items) after {after}")
    return sum(float(r["Counter_Value"]) for r in hit) / n, int(hit[-1]["Dispatch_Id"])


def stencil_table_traffic(fetch_dir, write_dir, fetch_log, write_log, command, out=TRAFFIC_FILE,
                          time_log=None, time_command=None):
    """HBM bytes per launch of every stencil of the benchmark's stencil table
    (full masked D_rr stencil per precision and RHS count, each in its tuned
    launch), from the same two counter runs and copy calibration as the
    dominant launch; adds them to the traffic table and returns a summary."""
    bf, bw = bench_line(fetch_log), bench_line(write_log)
    tab = bf.get("stencils_32")
    if not tab:
        raise SystemExit("the counter runs have no stencil table")
    # the times come from a run without counters (counter runs serialise the
    # dispatches) whose launches must be the ones the counters saw
    timed = bench_line(time_log)["stencils_32"] if time_log else tab
    for name, e in tab.items():
        if timed[name]["launch"]["shape"] != e["launch"]["shape"]:
            raise SystemExit(f"{name}: the timed run and the counter runs used different launches")
    cb = int(bf["calibration_copy_bytes"])
    fr, wr = _csv(fetch_dir, "_counter_collection.csv"), _csv(write_dir, "_counter_collection.csv")
    ff, fk, _ = _copy_factor(fr, cb, "FETCH_SIZE")
    wf, wk, _ = _copy_factor(wr, cb, "WRITE_SIZE")
    dims = bf["config"]["lattice"]
    with open(out) as f:
        table = json.load(f)
    if table.get("kernel_source_sha256") != kernel_source_hash():
        raise SystemExit("the traffic table is stale: write the dominant launch's entry first")
    lines = ["# Full D_rr stencil at " + "x".join(map(str, dims)) + ": time and HBM traffic per launch", "",
             "Commands (from the repository root, `cd /tmp && export TMPDIR=/tmp` first), one counter per run:", "",
             "    " + command, ""] + (["Times from the same benchmark without counters:", "",
                                   "    " + time_command, ""] if time_command else []) + [
             "Each row is the masked D_rr stencil (rest rows and columns of the Type I partition) in the",
             "launch the autotuner picks for that precision and RHS count.  Time: HIP events on the",
             "library's stream around each launch (bench run without counters).  Traffic: FETCH_SIZE and",
             "WRITE_SIZE per dispatch, scaled by what they read for torch's negation of 1 GiB in the same",
             f"process (fetch factor {ff:.3f}, write factor {wf:.3f}).  Algorithmic bytes: every site reads",
             "its input spinors and 4 links and writes its output spinors once.", "",
             "FETCH_SIZE counts the reads that miss L2, which the last-level cache (256 MB) may serve",
             "rather than HBM: rates above the copy ceiling show such hits.", "",
             "| precision | RHS | kernel (launch) | avg us | alg. GB | alg. GB/s | frac of 8 TB/s | traffic GB (counters) | traffic / alg. | traffic GB/s |",
             "|---|---:|---|---:|---:|---:|---:|---:|---:|---:|"]
    # the table's launches follow the copy ceiling's (the first copy
    # dispatches of the run), row after row: each row takes its warm-up and
    # timed dispatches from a window that starts after the previous row's
    ends = {"FETCH_SIZE": _first_copy(fr, "FETCH_SIZE"), "WRITE_SIZE": _first_copy(wr, "WRITE_SIZE")}
    for name, e in tab.items():
        prec, nrhs = name.split("_nrhs")
        launch = e["launch"]
        fetch, ends["FETCH_SIZE"] = _window_avg(fr, launch, "FETCH_SIZE", ends["FETCH_SIZE"])
        write, ends["WRITE_SIZE"] = _window_avg(wr, launch, "WRITE_SIZE", ends["WRITE_SIZE"])
        hbm = fetch * 1024 * ff + write * 1024 * wf
        alg, ms = e["alg_bytes_per_launch"], timed[name]["avg_ms"]
        key = traffic_key(prec, int(nrhs), dims, launch["shape"])
        table["kernels"][key] = {"symbol": launch["symbol"], "grid_size": launch["grid_size"],
                                 "shape": launch["shape"], "fetch_kib": fetch, "write_kib": write,
                                 "hbm_bytes_per_launch": hbm, "alg_bytes_per_launch": alg,
                                 "ratio_to_alg": hbm / alg, "command": command}
        lines.append(f"| {prec} | {nrhs} | `{launch['symbol']}` {shape_tag(launch['shape'])} | {ms * 1e3:.1f} | "
                     f"{alg / 1e9:.3f} | {alg / ms / 1e6:.0f} | {alg / ms / 1e6 / 8000:.3f} | {hbm / 1e9:.3f} | "
                     f"{hbm / alg:.2f} | {hbm / ms / 1e6:.0f} |")
    ceil = bench_line(time_log).get("copy_ceiling") if time_log else bf.get("copy_ceiling")
    if ceil:
        lines += ["", f"Copy ceiling in the timed run: {ceil['kernel']}, {ceil['GBps']:.0f} GB/s "
                      f"({ceil['frac_of_peak']:.2f} of peak)."]
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    return "\n".join(lines) + "\n"


def _between(rows, marker):
    """The rows dispatched between the last two dispatches of the kernel
    `marker` = 'NAME:WORK_ITEMS' (one step of a run), per counter run."""
    name, gs = marker.rsplit(":", 1)
    ids = sorted({int(r["Dispatch_Id"]) for r in rows if name in r["Kernel_Name"] and _grid_size(r) == int(gs)})
    if len(ids) < 2:
        raise SystemExit(f"fewer than two dispatches of {marker}")
    return [r for r in rows if ids[-2] < int(r["Dispatch_Id"]) < ids[-1]]


def counters_summary(dirs, kernels, command_lines, title, note="", copy_bytes=0, between=""):
    """Average of every counter per dispatch, per kernel (name substring)
    and grid, over the counter runs in `dirs` (one counter set per run);
    with copy_bytes (a copy kernel of that size ran in each run), FETCH_SIZE
    and WRITE_SIZE also scaled to HBM bytes by the copy's reading; with
    between, only the dispatches of the last step of each run (see _between)."""
    rows = []
    factors = {}
    for d in dirs:
        rd = _csv(d, "_counter_collection.csv")
        for cn in ("FETCH_SIZE", "WRITE_SIZE"):
            if copy_bytes and any(r["Counter_Name"] == cn and COPY_KERNEL in r["Kernel_Name"] for r in rd):
                factors[cn] = _copy_factor(rd, copy_bytes, cn)[0]
        rows.extend(_between(rd, between) if between else rd)
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
    if factors:
        note += " " + ", ".join(f"{cn} scale {f:.3f} (copy of {copy_bytes} bytes)" for cn, f in factors.items())
    lines += ["", note, "", "| kernel | work-items | dispatches | counter | average | HBM bytes (scaled) |",
              "|---|---:|---:|---|---:|---:|"]
    for (name, gs, cn), v in sorted(agg.items()):
        avg = sum(v) / len(v)
        scaled = f"{avg * 1024 * factors[cn]:.4g}" if cn in factors else ""
        lines.append(f"| `{name.replace('|', '/')}` | {gs} | {len(v)} | {cn} | {avg:.4g} | {scaled} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--bench-log", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--step-marker", default="",
                   help="kernel name (substring), optionally :WORK_ITEMS, whose dispatch ends a step: "
                        "adds a per-step breakdown")
    s.add_argument("--steps", type=int, default=0, help="steps of the breakdown (default: the bench's)")
    s.add_argument("--title", default="")
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
    c.add_argument("--copy-bytes", type=int, default=0)
    c.add_argument("--between", default="", metavar="KERNEL:WORK_ITEMS",
                   help="only the dispatches between the last two dispatches of this kernel")
    c.add_argument("--out")
    tt = sub.add_parser("stencil-table")
    for k in ("--fetch", "--write", "--fetch-log", "--write-log", "--command", "--out-md"):
        tt.add_argument(k, required=True)
    tt.add_argument("--out", default=TRAFFIC_FILE)
    tt.add_argument("--time-log")
    tt.add_argument("--time-command")
    a = ap.parse_args(argv)
    if a.cmd == "stencil-table":
        text = stencil_table_traffic(a.fetch, a.write, a.fetch_log, a.write_log, a.command, a.out,
                                     a.time_log, a.time_command)
        with open(a.out_md, "w") as f:
            f.write(text)
        sys.stdout.write(text)
        return
    if a.cmd == "counters":
        text = counters_summary(a.dirs, a.kernels, a.command, a.title, a.note, a.copy_bytes, a.between)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
        return
    if a.cmd == "stats":
        text = stats_summary(a.trace, a.bench_log, a.command, marker=a.step_marker, steps=a.steps,
                             title=a.title)
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
