#!/usr/bin/env python3
"""Throughput of the coarse Dirac operator S_bb = D_bb - D_br D_rr^{-1} D_rb on one GPU.

Workload (one "step" = one S_bb apply of the whole batch, every stage of the
method on the GPU: scatter to the lattice, D_rb, the D_rr solve, the final
D_bb/D_br combine and the gather):

  32^4 lattice, periodic in x, y, z and antiperiodic in t; synthetic SU(3)
  links U = reunitarised exp(i 0.5 sum_k a_k lambda_k), a_k ~ N(0,1), seed 3;
  Wilson mass m0 = -0.3; Type I permutation (coarse = all-even sites,
  N_b = 65536); 12 right-hand sides = unit point sources on coarse site 0, one
  per spin-colour; D_rr solved to a 1e-10 relative FP64 residual.

The product path (--inner, default bf16) stores the inner Krylov vectors and
links in bfloat16 with FP32 arithmetic inside an FP64 defect correction; the
plain-FP64 GCR path on the same workload is timed beside it.  value is
S_bb applies/s (right-hand sides x steps / seconds) with all inputs resident
in HBM.  The CPU oracle is timed on a bounded sample on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "S_bb applies/s + dslash HBM GB/s at 32^4; mixed+learned vs FP64 at 1e-10"
PEAK_HBM_GBS = 8000.0
REAL_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2}
def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def dslash_bytes_per_launch(prec: str, volume: int, nrhs: int) -> int:
    """Compulsory bytes of one stencil launch: every site reads 12 complex of
    input and writes 12 complex of output per RHS, and reads its 4 links
    (4 x 9 complex) once; neighbour spinors and backward links are re-reads."""
    b = REAL_BYTES[prec]
    return volume * (nrhs * 2 * 24 * b + 72 * b)


PREC_ID = {"fp64": 0, "fp32": 1, "bf16": 2}


def eo_bytes_per_launch(prec: str, volume: int, nrhs: int, iters: int, outer: int) -> float:
    """Compulsory bytes of the reduced operator's half-lattice stencils (the
    timed launches: every iteration runs one first and one second half),
    averaged: the first half reads one parity and writes the other (V sites'
    fields in all), the second also reads a field of the output parity
    (1.5 V); each half reads all V sites' links (the forward links of one
    parity, the backward ones of the other).  The once-per-outer-step
    full-layout halves are not among the timed launches."""
    b = REAL_BYTES[prec]
    spinor, links = nrhs * 24 * b, 72 * b
    k1 = volume * spinor + volume * links
    k2 = 1.5 * volume * spinor + volume * links
    return (k1 + k2) / 2


def launch_descriptor(info: dict, prec: str, launches: int, eo: bool = False) -> dict:
    """The stencil kernel a tuned launch runs, as a profiler names it, and its
    work-items per dispatch."""
    p = PREC_ID[prec]
    if eo and info["split"] == 7:
        # the plane form of the reduced operator's half-stencil (compact
        # fields: IO 0), one workgroup of SB lanes per x-y plane, RG planes
        # per workgroup; the first half of each operator application has no
        # alpha term (epilogue 0), the second the alpha term and the fused
        # sums (epilogue 2)
        npl = info["RG"]
        sym = f"eo_plane_kernel<0, 0, {npl}> + eo_plane_kernel<0, 2, {npl}>"
        gs = info["grid"] * info["SB"]
    elif eo:
        # the compact half-stencils of the reduced operator in the tuned form
        # (hop schedule info["split"], compact fields: IO 0)
        sym, gs = f"eo_hop_kernel<{p}, {info['split']}, 0>", info["grid"] * info["SB"]
    elif info["march"] > 0:
        # t-marching form: one wavefront per RHS of a group of RG
        sym, gs = f"march_kernel<grg::StoreEpi<{p}> >", info["grid"] * 64 * info["RG"]
    else:
        sym, gs = f"dslash_kernel<{p}, {info['split']}>", info["grid"] * info["SB"]
    shape = {k: info[k] for k in ("SB", "RG", "split", "grid", "chunk", "march")}
    return {"symbol": sym, "grid_size": gs, "launches": launches, "shape": shape}


def copy_calibration(torch, mib: int) -> int:
    """A plain streaming kernel of known size for the counter runs: torch's
    negation reads and writes n bytes once each."""
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return n


def time_applies(grg, s, xb, yb, nrhs, steps, warmup, profile):
    """Time `steps` applies after `warmup` untimed ones.  With profile set,
    HIP events bracket every stencil launch of the timed applies (the
    library's launch-only profiling: no per-phase events, and the events are
    read once, after the timed region)."""
    import torch

    for _ in range(warmup):
        grg.grg_schur_apply(s, xb, yb, nrhs)
    grg.grg_profile_enable(s, profile, launches_only=True)
    grg.grg_profile_reset(s)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(grg.grg_schur_apply(s, xb, yb, nrhs))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {p: grg.grg_profile_read(s, p) for p in ("fp64", "fp32", "bf16")}
    prof.update({p + "_eo": grg.grg_profile_read(s, p, eo=True) for p in ("fp64", "fp32", "bf16")})
    grg.grg_profile_enable(s, False)
    return t1 - t0, stats, prof


def learned_leg(grg, torch, args, lat, s, xb, yb, y_plain, nrhs, plain_value, plain_stats):
    """Train the network on a 16^4 field (m0 -0.3, seed 5) from pairs of the
    even-odd reduced inner solve, then use it as the right preconditioner of
    that reduced solve inside the same 32^4 S_bb apply."""
    from grg_inputs import su3_links

    dims16 = (16, 16, 16, 16)
    lat16 = grg.grg_lattice_create(dims16)
    grg.grg_gauge_set(lat16, su3_links(dims16, 0.5, 5))
    q16, nb16 = grg.grg_permutation_block(dims16, grg.GRG_PERM_I)
    s16 = grg.grg_schur_create(lat16, -0.3, q16, nb16,
                               grg.grg_solver_params_default(inner="bf16", inner_tol=1e-2, max_rhs=12))
    p16 = grg.grg_precond_create(s16)
    log(f"training the preconditioner: {args.train_steps} steps x 12 pairs on 16^4")
    tr = grg.grg_precond_train(p16, steps=args.train_steps, batch=12, max_mr_steps=30, lr=2e-3, seed=5,
                               log_every=50, reduced=True)
    w = grg.grg_precond_get_weights(p16)
    grg.grg_precond_destroy(p16)
    grg.grg_schur_destroy(s16)
    grg.grg_lattice_destroy(lat16)
    p = grg.grg_precond_create(s)
    grg.grg_precond_set_weights(p, w)
    grg.grg_schur_attach_precond(s, p)
    k = max(1, args.steps // 2)
    dt, stats, _ = time_applies(grg, s, xb, yb, nrhs, k, 1, False)
    st = stats[-1]
    y = yb.cpu().numpy()
    grg.grg_schur_attach_precond(s, None)
    grg.grg_precond_destroy(p)
    val = nrhs * k / dt
    diff = float(np.max(np.linalg.norm(y - y_plain, axis=1) / np.linalg.norm(y_plain, axis=1)))
    log(f"learned: {dt / k * 1e3:.1f} ms/step, {val:.1f} applies/s, iters {st['iters']} "
        f"(plain {plain_stats['iters']}), fallbacks {st['fallbacks']}")
    args._trained_weights = w
    return {"train": {"pairs": tr["pairs"], "steps": tr["steps"], "loss_first": tr["loss_first"],
                      "loss_last": tr["loss_last"], "seconds": tr["t_ms"] / 1e3, "lattice": "16^4"},
            "value": val, "ms_per_step": dt / k * 1e3, "inner_iters": st["iters"],
            "inner_iters_plain": plain_stats["iters"], "outer": st["outer"], "fallbacks": st["fallbacks"],
            "true_rel_resid": st["true_rel_resid"], "max_rel_diff_vs_plain": diff,
            "speedup_vs_plain_mixed": val / plain_value}


def vcycle_leg(grg, torch):
    """Section 4's experiment on synthetic fields: D x = f to 1e-8 at
    kappa = 1/6 (m0 = -1) by BiCGstab, plain and right-preconditioned by the
    3-level cyclic-reduction V-cycle (Type I at every level) and by the
    two-level cycles on the orderings of Table 1 (Type I^-1 and II^-1, with
    section 3's S~_bb on top); A_rr solves by BiCGstab to 1e-2, top level to
    1e-12; average convergence rate R per solve."""
    from grg_inputs import gaussian_vectors, su3_links

    out = {}
    cycles = (("vcycle_bicgstab", dict(levels=3)),
              ("two_level_I_inv_bicgstab", dict(levels=2, perm=1, inverse=1)),
              ("two_level_II_inv_bicgstab", dict(levels=2, perm=2, inverse=1)))
    for dims in ((8, 8, 8, 8), (16, 16, 16, 16)):
        lat = grg.grg_lattice_create(dims)
        grg.grg_gauge_set(lat, su3_links(dims, 0.5, 7))
        V = int(np.prod(dims))
        f = torch.from_numpy(gaussian_vectors(12 * V, 4, 7)).to("cuda")
        x = torch.empty_like(f)
        row = {}
        for name, kw in cycles:
            v = grg.grg_vcycle_create(lat, -1.0, grg.grg_vcycle_params_default(max_rhs=4, **kw))
            runs = (("bicgstab", False), (name, True)) if name == "vcycle_bicgstab" else ((name, True),)
            for key, pre in runs:
                st = grg.grg_vcycle_solve(v, f, x, 4, tol=1e-8, precondition=pre)
                row[key] = {"iters": st["iters"], "rate": st["rate"], "ms": st["t_ms"],
                            "true_rel_resid": st["true_rel_resid"], "cycles": st["cycles"]}
            grg.grg_vcycle_destroy(v)
        key = "x".join(map(str, dims))
        out[key] = row
        log(f"V-cycle {key}, m0 -1: " + "; ".join(
            f"{k} {r['iters']} iters, R {r['rate']:.3f}, {r['ms']:.1f} ms" for k, r in row.items()))
        grg.grg_lattice_destroy(lat)
    out["workload"] = ("synthetic links eps 0.5 seed 7, m0 = -1 (kappa = 1/6), 4 Gaussian RHS, tol 1e-8; "
                       "3-level Type I cycle, and two-level cycles on Type I^-1 and II^-1")
    return out


def stream_ceiling(torch, mib: int = 1024, reps: int = 10) -> dict:
    """A plain streaming kernel's bandwidth on this GPU (torch's negation of
    a 1 GiB FP32 array: reads and writes it once), the practical ceiling the
    stencils are compared with beside the 8 TB/s peak."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * (mib << 20) / (ms * 1e-3) / 1e9
    del src, dst
    return {"kernel": "torch.neg on 1 GiB fp32 (reads + writes 1 GiB)", "GBps": gbs,
            "frac_of_peak": gbs / PEAK_HBM_GBS}


def host_rates(torch, matfree, links, dims, m0, volume):
    """The oracle's FP64 stencil on one field (median of three; 960 B per site
    algorithmic: in, out and links), a multi-threaded copy of 1 GiB on the
    host (read plus written bytes), and the host's CPU model."""
    from grg_inputs import gaussian_vectors

    x = gaussian_vectors(12 * volume, 1, 9)
    ts = []
    for _ in range(3):
        t = time.perf_counter()
        matfree.dirac_apply(links, dims, m0, x)
        ts.append(time.perf_counter() - t)
    ds = sorted(ts)[1]
    src = torch.ones(1 << 27, dtype=torch.float64)
    dst = torch.empty_like(src)
    dst.copy_(src)
    cs = []
    for _ in range(3):
        t = time.perf_counter()
        dst.copy_(src)
        cs.append(time.perf_counter() - t)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"dslash_ms": ds * 1e3, "dslash_gbs": 960.0 * volume / ds / 1e9,
            "host_copy_gbs": 2.0 * src.numel() * 8 / sorted(cs)[1] / 1e9,
            "host_copy_threads": torch.get_num_threads(), "cpu_model": model}


def parse_stencil_launches(spec: str) -> dict:
    """'fp64_nrhs1=SB,RG,SPLIT,GRID,CHUNK,MARCH;...' -> {row: [6 ints]}."""
    out = {}
    for item in filter(None, (x.strip() for x in spec.split(";"))):
        name, vals = item.split("=")
        out[name.strip()] = [int(v) for v in vals.split(",")]
    return out


def stencil_table(grg, torch, lat, m0, q, nb, volume, dims, reps: int = 10, pin: dict | None = None):
    """The full masked D_rr stencil at this lattice in FP64, FP32 and BF16
    with 1 and 12 right-hand sides, each in the launch the autotuner picks
    for it: average time per launch (HIP events on the library's stream
    around every stencil launch) and algorithmic GB/s.  Every launch is tuned
    first, then the copy ceiling runs, then the timed launches in table
    order, so that a counter run finds each row's launches in sequence after
    the copy's.  Returns (table, ceiling)."""
    from grg_inputs import gaussian_vectors
    from paper_0704_2341_amd.profiling import measured_traffic, traffic_key

    out = {}
    x12 = torch.from_numpy(gaussian_vectors(12 * volume, 12, 91)).to("cuda")
    y12 = torch.empty_like(x12)
    handles = {}
    for prec in ("fp64", "fp32", "bf16"):
        prm = grg.grg_solver_params_default(tol=1e-10, inner=prec, max_rhs=12)
        handles[prec] = grg.grg_schur_create(lat, m0, q, nb, prm)
        for nrhs in (1, 12):
            grg.grg_schur_tune(handles[prec], nrhs)
            row = f"{prec}_nrhs{nrhs}"
            if pin and row in pin:
                grg.grg_schur_set_launch(handles[prec], prec, nrhs, pin[row])
    torch.cuda.synchronize()
    ceiling = stream_ceiling(torch)
    log(f"copy ceiling: {ceiling['GBps']:.0f} GB/s")
    for prec, s in handles.items():
        for nrhs in (1, 12):
            x, y = x12[:nrhs], y12[:nrhs]
            grg.grg_block_apply(s, prec, 0, 0, x, y, nrhs)
            grg.grg_profile_enable(s, True)
            grg.grg_profile_reset(s)
            for _ in range(reps):
                grg.grg_block_apply(s, prec, 0, 0, x, y, nrhs)
            torch.cuda.synchronize()
            cnt, ms = grg.grg_profile_read(s, prec)
            grg.grg_profile_enable(s, False)
            avg = ms / cnt
            alg = dslash_bytes_per_launch(prec, volume, nrhs)
            info = grg.grg_schur_tune_info(s, prec, nrhs)
            launch = launch_descriptor(info, prec, cnt)
            out[f"{prec}_nrhs{nrhs}"] = {"avg_ms": avg, "alg_bytes_per_launch": alg,
                                        "alg_GBps": alg / (avg * 1e-3) / 1e9,
                                        "frac_of_peak": alg / (avg * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                        "launch": launch,
                                        # counter-measured bytes of this launch shape, or None
                                        "traffic": measured_traffic(traffic_key(prec, nrhs, dims,
                                                                                launch["shape"]))}
            log(f"stencil {prec} nrhs {nrhs}: {avg * 1e3:.1f} us per launch, "
                f"{out[f'{prec}_nrhs{nrhs}']['alg_GBps']:.0f} GB/s algorithmic")
    for s in handles.values():
        grg.grg_schur_destroy(s)
    del x12, y12
    return out, ceiling


def solver_legs(grg, torch, args, lat, m0, q, nb, xb, yb, y_ref, nrhs, tol, k):
    """The same S_bb apply with the inner solve in FP32 (FP64 refinement to
    tol), and in FP64 on the even-odd reduced system of D_rr: with the plain
    FP64 leg (no reduction) they split the mixed path's gain into the
    reduction's and the precision's."""
    out = {}
    for name, kw in (("fp32_mixed_reduced", dict(inner="fp32", inner_tol=1e-5, eo=1)),
                     ("fp64_reduced", dict(inner="fp64", eo=1))):
        prm = grg.grg_solver_params_default(tol=tol, max_rhs=nrhs, max_iter=4000, check_every=args.check_every,
                                            **kw)
        s2 = grg.grg_schur_create(lat, m0, q, nb, prm)
        if not args.no_tune:
            grg.grg_schur_tune(s2, nrhs)
        dt2, st2, _ = time_applies(grg, s2, xb, yb, nrhs, k, 1, False)
        y2 = yb.cpu().numpy()
        d2 = np.linalg.norm(y2 - y_ref, axis=1) / np.linalg.norm(y_ref, axis=1)
        out[name] = {"value": nrhs * k / dt2, "ms_per_step": dt2 / k * 1e3, "iters": st2[-1]["iters"],
                     "outer": st2[-1]["outer"], "true_rel_resid": st2[-1]["true_rel_resid"],
                     "max_rel_diff_vs_product": float(d2.max())}
        log(f"{name}: {dt2 / k * 1e3:.2f} ms/step, {nrhs * k / dt2:.1f} applies/s, iters {st2[-1]['iters']} "
            f"outer {st2[-1]['outer']}, diff {d2.max():.2e}")
        grg.grg_schur_destroy(s2)
    return out


def learned_leg_24(grg, torch, args, w, nrhs=12, steps=3):
    """The trained network at 24^4 (m0 -0.3, links seed 3, 12 point sources,
    1e-10): the mixed solve with and without it as the right preconditioner
    of the reduced inner solve; iterations and wall time."""
    from grg_inputs import point_sources, su3_links

    dims = (24, 24, 24, 24)
    lat = grg.grg_lattice_create(dims, (1, 1, 1, -1))
    grg.grg_gauge_set(lat, su3_links(dims, 0.5, 3))
    q, nb = grg.grg_permutation_block(dims, grg.GRG_PERM_I, False)
    xb = torch.from_numpy(point_sources(nb, nrhs)).to("cuda")
    yb = torch.empty_like(xb)
    prm = grg.grg_solver_params_default(tol=1e-10, inner="bf16", inner_tol=1e-2, max_rhs=nrhs, max_iter=4000)
    s = grg.grg_schur_create(lat, -0.3, q, nb, prm)
    if not args.no_tune:
        grg.grg_schur_tune(s, nrhs)
    out = {"lattice": "24^4"}
    dt0, st0, _ = time_applies(grg, s, xb, yb, nrhs, steps, 1, False)
    y0 = yb.cpu().numpy()
    p = grg.grg_precond_create(s)
    grg.grg_precond_set_weights(p, w)
    grg.grg_schur_attach_precond(s, p)
    dt1, st1, _ = time_applies(grg, s, xb, yb, nrhs, steps, 1, False)
    y1 = yb.cpu().numpy()
    grg.grg_schur_attach_precond(s, None)
    grg.grg_precond_destroy(p)
    out["plain"] = {"ms_per_step": dt0 / steps * 1e3, "value": nrhs * steps / dt0, "inner_iters": st0[-1]["iters"],
                    "outer": st0[-1]["outer"], "true_rel_resid": st0[-1]["true_rel_resid"]}
    out["learned"] = {"ms_per_step": dt1 / steps * 1e3, "value": nrhs * steps / dt1,
                      "inner_iters": st1[-1]["iters"], "outer": st1[-1]["outer"],
                      "fallbacks": st1[-1]["fallbacks"], "true_rel_resid": st1[-1]["true_rel_resid"],
                      "max_rel_diff_vs_plain": float(np.max(np.linalg.norm(y1 - y0, axis=1)
                                                            / np.linalg.norm(y0, axis=1)))}
    log(f"24^4: plain {out['plain']['ms_per_step']:.1f} ms, {st0[-1]['iters']} inner iters; learned "
        f"{out['learned']['ms_per_step']:.1f} ms, {st1[-1]['iters']} inner iters")
    grg.grg_schur_destroy(s)
    grg.grg_lattice_destroy(lat)
    return out


def batch_leg(grg, torch, args):
    """48 lattices, sizes uniform over {8^4, 12^4, 16^4, 8^3x16}, own seeds,
    m0 in [-0.3, 0.1], 4 RHS each, FP32 inner / FP64 outer, one batch; the
    inner solve on each lattice's even-odd reduced D_rr (every extent is
    even), and once more on D_rr itself for comparison."""
    from grg_inputs import batch_instances, gaussian_vectors, su3_links

    descs = batch_instances(48)
    ms = []
    for d in descs:
        q, nb = grg.grg_permutation_block(d["dims"], grg.GRG_PERM_I)
        ms.append(dict(dims=d["dims"], m0=d["m0"], links=su3_links(d["dims"], 0.5, d["seed"]), q=q,
                       n_coarse=nb))
    nrhs = 4
    prm = grg.grg_solver_params_default(tol=1e-10, inner="fp32", inner_tol=1e-5, check_every=4)
    b = grg.grg_batch_create(ms, nrhs, prm)
    grg.grg_batch_tune(b)
    total, _ = grg.grg_batch_layout(b, 48)
    x = np.zeros(total, np.complex128)
    for i in range(48):
        off, nb = grg.grg_batch_layout(b, i)
        x[off:off + 12 * nb * nrhs] = gaussian_vectors(12 * nb, nrhs, 4000 + i).reshape(-1)
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.empty_like(xd)
    out = {"lattices": 48, "rhs_per_lattice": nrhs, "systems": 48 * nrhs,
           "sites": int(sum(int(np.prod(m["dims"])) for m in ms))}
    for mode, graph in (("graph", True), ("eager", False)):
        # graph: the first apply runs eagerly and records the outer and inner
        # counts, the second captures the whole apply; the timed ones replay it
        for _ in range(2):
            grg.grg_batch_apply(b, xd, yd, use_graph=graph)
        torch.cuda.synchronize()
        k = max(1, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(k):
            st = grg.grg_batch_apply(b, xd, yd, use_graph=graph)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k
        out[mode] = {"ms_per_batch": dt * 1e3, "applies_per_s": 48 * nrhs / dt, "inner_iters": st["iters"],
                     "outer": st["outer"], "true_rel_resid": st["true_rel_resid"]}
        if graph:
            out[mode]["captured_outer_inner"] = list(grg.grg_batch_graph_info(b))
        log(f"batch ({mode}): {dt * 1e3:.2f} ms per 48 x {nrhs} applies, {48 * nrhs / dt:.1f} applies/s")
    # roofline of the batch's per-iteration kernels at the tuned launch, every
    # system active (HIP events on the batch's stream, timed by the tuner):
    # one half-step of the reduced operator on the compact fields (the two
    # halves averaged: the output side's half-sites written, the other
    # side's read, the second half also reading in2, every site's links), and
    # the MR update on the compact fields (reads x, r, q and writes x, r)
    ti = grg.grg_batch_tune_info(b, "fp32")
    vt = out["sites"]
    kb = {"stencil": eo_bytes_per_launch("fp32", vt, nrhs, 0, 0),
          "mr_update": vt // 2 * nrhs * 5 * 24 * REAL_BYTES["fp32"]}
    kms = {"stencil": ti["stencil_ms"], "mr_update": ti["update_ms"]}
    dom = max(kms, key=kms.get)
    ach = kb[dom] / (kms[dom] * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": f"batch {'reduced half-step' if dom == 'stencil' else dom} "
                                                 f"(fp32, compact fields, all 192 systems)", "achieved": ach,
                       "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                       "alg_bytes_per_launch": kb[dom], "avg_launch_ms": kms[dom],
                       "other": {k: {"ms": kms[k], "alg_GBps": kb[k] / (kms[k] * 1e-3) / 1e9} for k in kms},
                       "launch": {k: ti[k] for k in ("SB", "RG", "grid")}}
    log(f"batch roofline: {dom} {kms[dom]:.3f} ms, {ach:.0f} GB/s ({ach / PEAK_HBM_GBS:.2f} of peak); "
        + ", ".join(f"{k} {kms[k]:.3f} ms" for k in kms))
    grg.grg_batch_destroy(b)
    # the same batch with the inner solve on D_rr (no even-odd reduction)
    b = grg.grg_batch_create(ms, nrhs, grg.grg_solver_params_default(tol=1e-10, inner="fp32", inner_tol=1e-5,
                                                                       check_every=4, eo=0))
    grg.grg_batch_tune(b)
    for _ in range(2):
        grg.grg_batch_apply(b, xd, yd, use_graph=True)
    torch.cuda.synchronize()
    k = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(k):
        st = grg.grg_batch_apply(b, xd, yd, use_graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / k
    out["graph_unreduced"] = {"ms_per_batch": dt * 1e3, "applies_per_s": 48 * nrhs / dt,
                              "inner_iters": st["iters"], "outer": st["outer"],
                              "true_rel_resid": st["true_rel_resid"]}
    log(f"batch (graph, inner solve on D_rr): {dt * 1e3:.2f} ms, {48 * nrhs / dt:.1f} applies/s, "
        f"{st['iters']} inner iterations")
    grg.grg_batch_destroy(b)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--inner", default="bf16", choices=["bf16", "fp32", "fp64"])
    ap.add_argument("--inner-tol", type=float, default=None)
    ap.add_argument("--restart", type=int, default=1)
    ap.add_argument("--check-every", type=int, default=2, help="inner iterations between norm reads")
    ap.add_argument("--fp64-restart", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--dims", default="32,32,32,32")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the stencil autotuner")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 48-lattice batch leg")
    ap.add_argument("--no-reusken", action="store_true", help="skip the section 3 approximation leg")
    ap.add_argument("--no-vcycle", action="store_true", help="skip the section 4 V-cycle leg")
    ap.add_argument("--no-stencils", action="store_true",
                    help="skip the stencil table (FP64 / FP32 / BF16 x 1 / 12 RHS) and the copy ceiling")
    ap.add_argument("--stencil-launches", default="", metavar="ROW=SB,RG,SPLIT,GRID,CHUNK,MARCH;...",
                    help="pin launches of the stencil table after tuning (rows fp64_nrhs1 ... bf16_nrhs12)")
    ap.add_argument("--no-solver-legs", action="store_true",
                    help="skip the FP32-inner and FP64-reduced solver legs")
    ap.add_argument("--train-steps", type=int, default=1667, help="12-pair Adam steps (1667 = 20k pairs)")
    ap.add_argument("--eo-launch", default="", metavar="SB,RG,SPLIT,GRID,CHUNK,MARCH",
                    help="pin the half-lattice stencil's launch after tuning")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain copy kernel of MIB MiB (for counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the path across several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_0704_2341_amd as grg
    from grg_inputs import point_sources, su3_links
    from paper_0704_2341_amd.profiling import measured_traffic, traffic_key

    dims = tuple(int(d) for d in args.dims.split(","))
    volume = int(np.prod(dims))
    m0, eps, seed, nrhs, tol = -0.3, 0.5, 3, 12, 1e-10
    inner_tol = args.inner_tol or {"bf16": 1e-2, "fp32": 1e-5, "fp64": tol}[args.inner]

    log(f"links {dims} eps={eps} seed={seed}")
    t = time.perf_counter()
    links = su3_links(dims, eps, seed)
    log(f"links ready in {time.perf_counter() - t:.1f} s")
    torch.cuda.init()
    lat = grg.grg_lattice_create(dims, (1, 1, 1, -1))
    grg.grg_gauge_set(lat, links)
    q, nb = grg.grg_permutation_block(dims, grg.GRG_PERM_I, False)
    xb_host = point_sources(nb, nrhs)
    xb = torch.from_numpy(xb_host).to("cuda")
    yb = torch.empty_like(xb)

    prm = grg.grg_solver_params_default(tol=tol, inner=args.inner, inner_tol=inner_tol,
                                        check_every=args.check_every,
                                        restart=args.restart, max_rhs=nrhs, max_iter=4000)
    s = grg.grg_schur_create(lat, m0, q, nb, prm)
    if not args.no_tune:
        t = time.perf_counter()
        grg.grg_schur_tune(s, nrhs)
        log(f"tuned in {time.perf_counter() - t:.1f} s: "
            f"{args.inner} {grg.grg_schur_tune_info(s, args.inner, nrhs)}, "
            f"fp64 {grg.grg_schur_tune_info(s, 'fp64', nrhs)}, "
            f"even-odd {grg.grg_schur_tune_info(s, args.inner, nrhs, eo=True)}, "
            f"defect correction {grg.grg_schur_dc_launch_info(s, args.inner, nrhs)}")
    if args.eo_launch:
        # pin the half-lattice stencil (runs that must time the same launch,
        # such as the two counter passes of one traffic measurement)
        grg.grg_schur_set_launch(s, args.inner, nrhs, [int(v) for v in args.eo_launch.split(",")], eo=True)
        log(f"even-odd launch pinned: {grg.grg_schur_tune_info(s, args.inner, nrhs, eo=True)}")
    log(f"timing {args.inner} path: warmup {args.warmup}, steps {args.steps}")
    dt, stats, prof = time_applies(grg, s, xb, yb, nrhs, args.steps, args.warmup, True)
    y_mixed = yb.cpu().numpy()
    value = nrhs * args.steps / dt
    st = stats[-1]
    log(f"{args.inner}: {dt / args.steps * 1e3:.2f} ms/step, {value:.1f} applies/s, "
        f"iters {st['iters']} outer {st['outer']} resid {st['true_rel_resid']:.2e}")

    kernels = {}
    for p, (cnt, ms) in prof.items():
        if cnt:
            avg = ms / cnt
            eo = p.endswith("_eo")
            pr = p[:-3] if eo else p
            alg = (eo_bytes_per_launch(pr, volume, nrhs, st["iters"], st["outer"]) if eo
                   else dslash_bytes_per_launch(pr, volume, nrhs))
            kernels[f"dslash_{p}"] = {"launches": cnt, "avg_ms": avg, "total_ms": ms,
                                      "alg_GBps": alg / (avg * 1e-3) / 1e9, "alg_bytes_per_launch": alg}
    # the dominant stencil: the one with the most time in the timed region
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dk = kernels[dom]
    dom_eo = dom.endswith("_eo")
    dom_prec = dom[len("dslash_"):].replace("_eo", "")
    dlaunch = launch_descriptor(grg.grg_schur_tune_info(s, dom_prec, nrhs, eo=dom_eo), dom_prec,
                                dk["launches"], eo=dom_eo)
    # traffic of this very launch shape (counter runs are per shape)
    tkey = traffic_key(dom_prec + ("_eo" if dom_eo else ""), nrhs, dims, dlaunch["shape"])
    traffic = measured_traffic(tkey)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["alg_GBps"], "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": dk["alg_GBps"] / PEAK_HBM_GBS,
                "traffic": traffic, "alg_bytes_per_launch": dk["alg_bytes_per_launch"],
                "avg_launch_ms": dk["avg_ms"], "traffic_key": tkey, "launch": dlaunch}

    fp64 = None
    bicg = None
    if not args.no_fp64 and args.inner != "fp64":
        # the baseline: plain FP64 minimal residual / GCR on D_rr (no even-odd reduction)
        prm64 = grg.grg_solver_params_default(tol=tol, inner="fp64", restart=args.fp64_restart,
                                              max_rhs=nrhs, max_iter=4000, eo=0)
        s64 = grg.grg_schur_create(lat, m0, q, nb, prm64)
        if not args.no_tune:
            grg.grg_schur_tune(s64, nrhs)
        k64 = args.fp64_steps or max(1, args.steps // 2)
        log(f"timing fp64 path: steps {k64}")
        dt64, st64, prof64 = time_applies(grg, s64, xb, yb, nrhs, k64, 1, True)
        y64 = yb.cpu().numpy()
        diff = np.linalg.norm(y_mixed - y64, axis=1) / np.linalg.norm(y64, axis=1)
        cnt, ms = prof64["fp64"]
        fp64 = {"value": nrhs * k64 / dt64, "ms_per_step": dt64 / k64 * 1e3,
                "iters": st64[-1]["iters"], "restart": args.fp64_restart,
                "true_rel_resid": st64[-1]["true_rel_resid"],
                "dslash_fp64_avg_ms": ms / cnt,
                "dslash_fp64_alg_GBps": dslash_bytes_per_launch("fp64", volume, nrhs) / (ms / cnt * 1e-3) / 1e9,
                "max_rel_diff_mixed_vs_fp64": float(diff.max())}
        log(f"fp64: {fp64['ms_per_step']:.2f} ms/step, {fp64['value']:.1f} applies/s, "
            f"diff vs mixed {diff.max():.2e}")
        grg.grg_schur_destroy(s64)
        # the paper's solver for D_rr: FP64 BiCGstab on D_rr itself, and the
        # same inside the product's mixed-precision, even-odd reduced path
        bicg = {}
        for name, kw in (("fp64", dict(inner="fp64", eo=0)),
                         (args.inner + "_mixed_reduced", dict(inner=args.inner, inner_tol=inner_tol,
                                                              check_every=args.check_every, eo=1))):
            prm_b = grg.grg_solver_params_default(tol=tol, max_rhs=nrhs, max_iter=4000, method="bicgstab", **kw)
            sbg = grg.grg_schur_create(lat, m0, q, nb, prm_b)
            if not args.no_tune:
                grg.grg_schur_tune(sbg, nrhs)
            dtb, stb, _ = time_applies(grg, sbg, xb, yb, nrhs, k64, 1, False)
            yb_h = yb.cpu().numpy()
            db = np.linalg.norm(y_mixed - yb_h, axis=1) / np.linalg.norm(yb_h, axis=1)
            bicg[name] = {"value": nrhs * k64 / dtb, "ms_per_step": dtb / k64 * 1e3, "iters": stb[-1]["iters"],
                          "outer": stb[-1]["outer"], "true_rel_resid": stb[-1]["true_rel_resid"],
                          "max_rel_diff_vs_product": float(db.max())}
            log(f"bicgstab {name}: {dtb / k64 * 1e3:.2f} ms/step, {nrhs * k64 / dtb:.1f} applies/s, "
                f"iters {stb[-1]['iters']}, diff {db.max():.2e}")
            grg.grg_schur_destroy(sbg)

    solver = None
    if not args.no_solver_legs and args.inner != "fp64":
        solver = solver_legs(grg, torch, args, lat, m0, q, nb, xb, yb, y_mixed, nrhs, tol,
                             args.fp64_steps or max(1, args.steps // 2))

    reusken = None
    if not args.no_reusken:
        # the section 3 approximation on the same workload: no solve
        ya = torch.empty_like(xb)
        grg.grg_reusken_apply(s, xb, ya, nrhs)
        torch.cuda.synchronize()
        kr = max(1, args.steps)
        t0 = time.perf_counter()
        for _ in range(kr):
            grg.grg_reusken_apply(s, xb, ya, nrhs)
        torch.cuda.synchronize()
        dtr = (time.perf_counter() - t0) / kr
        ya_h = ya.cpu().numpy()
        rd = float(np.max(np.linalg.norm(ya_h - y_mixed, axis=1) / np.linalg.norm(y_mixed, axis=1)))
        reusken = {"value": nrhs / dtr, "unit": "S~_bb applies/s", "ms_per_step": dtr * 1e3,
                   "rel_diff_vs_exact": rd}
        log(f"reusken: {dtr * 1e3:.2f} ms/step, {nrhs / dtr:.1f} applies/s, |S~x - Sx|/|Sx| {rd:.3f}")
        # the older approximation that ignores the couplings inside D_rr
        grg.grg_diag_schur_apply(s, xb, ya, nrhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(kr):
            grg.grg_diag_schur_apply(s, xb, ya, nrhs)
        torch.cuda.synchronize()
        dt0 = (time.perf_counter() - t0) / kr
        ya_h = ya.cpu().numpy()
        rd0 = float(np.max(np.linalg.norm(ya_h - y_mixed, axis=1) / np.linalg.norm(y_mixed, axis=1)))
        reusken["ignoring_drr"] = {"value": nrhs / dt0, "unit": "S0_bb applies/s", "ms_per_step": dt0 * 1e3,
                                   "rel_diff_vs_exact": rd0}
        log(f"ignoring D_rr: {dt0 * 1e3:.2f} ms/step, {nrhs / dt0:.1f} applies/s, |S0x - Sx|/|Sx| {rd0:.3f}")

    learned = None
    if not args.no_learned:
        learned = learned_leg(grg, torch, args, lat, s, xb, yb, y_mixed, nrhs, value, st)
        learned["at_24"] = learned_leg_24(grg, torch, args, args._trained_weights)
    vc = None
    if not args.no_vcycle:
        vc = vcycle_leg(grg, torch)
    batch = None
    if not args.no_batch:
        batch = batch_leg(grg, torch, args)

    stencils = ceiling = None
    if not args.no_stencils:
        stencils, ceiling = stencil_table(grg, torch, lat, m0, q, nb, volume, dims,
                                          pin=parse_stencil_launches(args.stencil_launches))

    copy_bytes = copy_calibration(torch, args.calibrate_copy) if args.calibrate_copy else None

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import matfree

        log("timing the CPU oracle on one right-hand side")
        t = time.perf_counter()
        y_or, it_or, rr_or = matfree.schur_apply(links, dims, m0, q, nb, xb_host[:1], restart=8, tol=tol)
        dt_cpu = time.perf_counter() - t
        agree = float(np.linalg.norm(y_mixed[0] - y_or[0]) / np.linalg.norm(y_or[0]))
        cpu = {"value": 1.0 / dt_cpu, "unit": "S_bb applies/s", "cores": matfree.num_threads(),
               "kind": "oracle",
               "sample": f"one of the 12 point sources, full S_bb apply at {args.dims.replace(',', 'x')} "
                         f"(C oracle, GCR(8) to {tol:g}, {int(it_or[0])} iterations) in {dt_cpu:.1f} s",
               "gpu_vs_oracle_rel_diff": agree}
        cpu.update(host_rates(torch, matfree, links, dims, m0, volume))
        log(f"oracle: {dt_cpu:.1f} s per apply, GPU agreement {agree:.2e}; "
            f"its stencil {cpu['dslash_ms']:.1f} ms ({cpu['dslash_gbs']:.1f} GB/s algorithmic), "
            f"host copy {cpu['host_copy_gbs']:.1f} GB/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "S_bb applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16-store/f32-arith inner + f64 outer",
                  "fp32": "f32 inner + f64 outer", "fp64": "f64"}[args.inner],
        "data": "synthetic",
        "config": {"workload": f"S_bb apply, {args.dims.replace(',', 'x')} Wilson, Type I, m0={m0}, "
                               f"eps={eps}, {nrhs} point sources, tol={tol:g}",
                   "lattice": list(dims), "nrhs": nrhs, "inner": args.inner,
                   "inner_tol": inner_tol, "restart": args.restart, "tol": tol,
                   "dslash_launch": grg.grg_schur_tune_info(s, args.inner, nrhs),
                   "eo_launch": grg.grg_schur_tune_info(s, args.inner, nrhs, eo=True),
                   "dc_launch": grg.grg_schur_dc_launch_info(s, args.inner, nrhs),
                   "parallelism": "1 GPU"},
        "solver": {"iters": st["iters"], "outer": st["outer"],
                   "true_rel_resid": st["true_rel_resid"], "n_dslash": st["n_dslash"]},
        "kernels": kernels,
        "roofline": roofline,
        "fp64_gcr": fp64,
        "bicgstab": bicg,
        "speedup_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "solver_legs": solver,
        "stencils_32": stencils,
        "copy_ceiling": ceiling,
        "reusken_approximation": reusken,
        "learned_preconditioner": learned,
        "batch_48": batch,
        "vcycle_section4": vc,
        "cpu_baseline": cpu,
    }
    if copy_bytes:
        out["calibration_copy_bytes"] = copy_bytes
    print(json.dumps(out), flush=True)
    grg.grg_schur_destroy(s)
    grg.grg_lattice_destroy(lat)


if __name__ == "__main__":
    main()
