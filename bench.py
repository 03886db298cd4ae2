"""Benchmark of the monodomain step on one MI355X.

Workload: the 40 x 40 x 10 mm ventricular slab at h = 0.25 mm (5,120,000
tets), fibres rotating -60 -> +60 deg through the wall with 5 deg jitter,
TP06 endo/mid/epi layers, corner stimulus, dt = 0.02 ms (synthetic, seeded).
A step is the whole explicit step: node gather + fused flux / cell model /
update / detection kernel (+ the vbar trace every 50 steps).

Prints one JSON line: cell-steps/s of the FP32-mixed path (the `value`),
the FP64 path beside it, p50/p99 step latency, the roofline of the dominant
(cell) kernel and the CPU oracle timed on a bounded sample on the host.
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

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2112_12854_amd/csrc/kernels.hpp", "paper_2112_12854_amd/csrc/cellmodels.hpp",
                  "paper_2112_12854_amd/csrc/instance.hip", "paper_2112_12854_amd/build.py")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_cell_slab-40x40x10mm-h0.25.md")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(prec: str):
    """HBM bytes per cell-kernel launch from the rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"kernel_sources_sha256:\s*([0-9a-f]{64})", text)
    v = re.search(rf"{prec}_hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not v or m.group(1) != kernel_sources_sha256():
        return None
    return float(v.group(1))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(ep, w, prec, steps, warmup, chunk, profile_steps):
    import torch
    t0 = time.time()
    sim = ep.Sim(w, prec=prec, allocator="torch", trace_every=50)
    log(f"prec={prec}: init {time.time() - t0:.1f}s, footprint {sim.footprint() / 2**30:.2f} GiB")
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    lat = []
    done = 0
    t_start = time.perf_counter()
    while done < steps:
        k = min(chunk, steps - done)
        t1 = time.perf_counter()
        sim.step(k)
        sim.sync()
        lat.append((time.perf_counter() - t1) / k)
        done += k
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log(f"prec={prec}: {steps} steps in {elapsed:.3f}s")
    node_b, cell_b = sim.algorithmic_bytes()
    at = sim.activation()
    n_sub = sim.purkinje_n_sub() if sim.n_purkinje else 0
    sim.close()
    # kernel durations over the same window of the same job: a fresh
    # simulation, the same untimed warm-up, then event-timed direct launches
    sim = ep.Sim(w, prec=prec, allocator="torch", trace_every=50)
    sim.step(warmup)
    cell_ms, node_ms = sim.profile_steps(profile_steps)
    res = dict(ms_per_step=1e3 * elapsed / steps,
               graph_node_steps_per_s=sim.n_purkinje * n_sub * steps / elapsed,
               graph_substeps=n_sub,
               cell_steps_per_s=w.n_tets * steps / elapsed,
               p50_ms=1e3 * float(np.percentile(lat, 50)),
               p99_ms=1e3 * float(np.percentile(lat, 99)),
               cell_kernel_ms=cell_ms, node_kernel_ms=node_ms,
               cell_bytes=cell_b, node_bytes=node_b,
               activated=int(np.isfinite(at).sum()))
    sim.close()
    return res


def measure_hbm(mib: int = 2048, reps: int = 20):
    """Achievable HBM bandwidth on this device for reference: a device copy
    (read + write) and a read-only reduction of a 2 GiB buffer."""
    import torch
    x = torch.ones(mib * 2**20 // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, nbytes in (("copy", lambda: y.copy_(x), 2 * x.nbytes),
                             ("read", lambda: x.sum(), x.nbytes)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    return out


def cpu_baseline(steps: int, nx: int, ny: int, nz: int):
    """The oracle (as it stands) on a sub-slab of the same recipe, on all host
    threads, then on one thread (beside the paper's single-core figure)."""
    import oracle
    from paper_2112_12854_amd import meshgen
    w = meshgen.scaled_config2(nx, ny, nz, n_steps=steps)
    ref = oracle.Sim(w)
    ref.step(2)
    t0 = time.perf_counter()
    ref.step(steps)
    el = time.perf_counter() - t0
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    s1 = max(2, steps // 30)
    t0 = time.perf_counter()
    ref.step(s1)
    el1 = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=w.n_tets * steps / el, unit="cell-steps/s",
                cores=threads, kind="oracle",
                sample=f"{w.n_tets} tets ({nx}x{ny}x{nz} hexes of the same slab recipe, "
                       f"h=0.25 mm), {steps} FP64 steps after 2 untimed, {el:.1f} s",
                single_thread={"value": w.n_tets * s1 / el1, "steps": s1},
                host_cpu=cpu, host_cpus_visible=os.cpu_count())


def run_serving(ep, n_req, n_steps, rate, seed=4, prec=None, one_at_a_time=False, trial=20):
    """Serving stream: slab requests log-uniform in [1e4, 1e6] tets with
    Poisson arrivals at a fixed `rate` (requests/s); continuous batching with
    the autotuned schedule (re-tuned as the batch grows or shrinks), or one
    request at a time."""
    from paper_2112_12854_amd import meshgen
    specs = meshgen.serving_requests(n=n_req, seed=seed)
    ws = [meshgen.serving_workload(sp, n_steps) for sp in specs]
    work = np.array([w.n_tets * n_steps for w in ws], dtype=np.float64)
    lam = rate
    rng = np.random.default_rng(seed + 1000)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
    sv = ep.Server(prec=prec, max_slots=1 if one_at_a_time else 256)
    if not one_at_a_time:
        sv.autotune(trial, retune=True)
    t0 = time.perf_counter()
    ids = []
    for i, w in enumerate(ws):
        wait = arrivals[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        ids.append(sv.submit(w, n_steps))
    res = [sv.wait(r) for r in ids]
    st = sv.stats()
    sv.close()
    bad = [r for r in res if r["status"] != ep.EP_OK]
    if bad:
        raise RuntimeError(f"{len(bad)} serving requests failed")
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), cell_steps_per_s=float(work.sum() / span),
                span_s=span, arrival_rate_per_s=lam, n_requests=n_req, steps=n_steps,
                mean_tets=float(np.mean([w.n_tets for w in ws])),
                steps_per_graph=st["steps_per_graph"], xcd_remap=st["xcd_remap"],
                autotune_runs=st["autotune_runs"])


def run_uq(ep, n_inst, n_steps, prec, trial=25, seed=5):
    """Config-5 batch: uneven slabs (8k-64k tets) with per-instance ionic
    conductance scales, all resident together, autotuned once on the full
    batch, then timed from the live progress counter."""
    from paper_2112_12854_amd import meshgen
    specs = meshgen.uq_instances(n=n_inst, seed=seed)
    ws = [meshgen.uq_workload(sp, n_steps) for sp in specs]
    total = sum(w.n_tets for w in ws)
    sv = ep.Server(prec=prec, max_slots=n_inst)
    sv.hold(True)
    t0 = time.perf_counter()
    ids = [sv.submit(w, n_steps) for w in ws]
    while sv.stats()["running"] < n_inst:
        if time.perf_counter() - t0 > 300:
            raise RuntimeError("UQ batch did not become resident")
        time.sleep(0.01)
    t_res = time.perf_counter() - t0
    sv.autotune(trial)
    sv.hold(False)
    while sv.stats()["autotune_runs"] < 1:
        time.sleep(0.005)
    # steady state: from the end of the tuning to 90 % of the batch's steps
    # issued (the counter advances as launches are queued, at most two
    # launches ahead of the device, alike at both ends of the window)
    st1, t1 = sv.stats(), time.perf_counter()
    goal = 0.9 * total * n_steps
    while True:
        st2, t2 = sv.stats(), time.perf_counter()
        if st2["cell_steps"] >= goal or st2["completed"] == n_inst:
            break
        time.sleep(0.002)
    res = [sv.wait(r) for r in ids]
    t3 = time.perf_counter()
    sv.close()
    if any(r["status"] != ep.EP_OK for r in res):
        raise RuntimeError("UQ instances failed")
    return dict(n_instances=n_inst, total_tets=total, steps=n_steps,
                cell_steps_per_s=(st2["cell_steps"] - st1["cell_steps"]) / (t2 - t1),
                end_to_end_cell_steps_per_s=total * n_steps / (t3 - t0),
                end_to_end_s=t3 - t0,
                tuned_ms_per_step=st1["tuned_ms_per_step"],
                tuned_cell_steps_per_s=total / (st1["tuned_ms_per_step"] * 1e-3),
                steps_per_graph=st1["steps_per_graph"], xcd_remap=st1["xcd_remap"],
                resident_after_s=t_res)


def _err_stats(a, b):
    d = np.abs(a - b)
    d = d[np.isfinite(d)]
    if d.size == 0:
        return None
    return {"max": float(d.max()), "p99": float(np.percentile(d, 99)), "mean": float(d.mean()),
            "n": int(d.size)}


def fp32_accuracy(ep, meshgen, n_uq=16, uq_steps=25000):
    """FP32-mixed error per result: activation time and APD90 of every cell
    against the GPU FP64 path (held to the FP64 oracle by the parity tests)
    on a layered rotating-fibre slab and on a seeded subset of the UQ batch,
    both over 500 ms."""
    out = {}
    w = meshgen.config2(n_steps=25000, nx=24, ny=20, nz=8, h=0.25)
    r = {}
    for name, prec in (("fp32", ep.EP_FP32_MIXED), ("fp64", ep.EP_FP64)):
        g = ep.Sim(w, prec=prec)
        g.step(w.n_steps)
        r[name] = (g.activation(), g.apd90())
        g.close()
    out["slab_vs_gpu_fp64"] = {"workload": f"{w.name} {w.n_tets} tets, 500 ms",
                               "at_ms": _err_stats(r["fp32"][0], r["fp64"][0]),
                               "apd90_ms": _err_stats(r["fp32"][1], r["fp64"][1]),
                               "at_nan_pattern_equal": bool(np.array_equal(np.isnan(r["fp32"][0]),
                                                                           np.isnan(r["fp64"][0])))}
    specs = meshgen.uq_instances(n=1024, seed=5)[:n_uq]
    ws = [meshgen.uq_workload(sp, uq_steps) for sp in specs]
    res = {}
    for name, prec in (("fp32", ep.EP_FP32_MIXED), ("fp64", ep.EP_FP64)):
        sv = ep.Server(prec=prec, max_slots=n_uq)
        ids = [sv.submit(x, uq_steps) for x in ws]
        for i in ids:
            sv.wait(i)
        res[name] = ([sv.activation(i) for i in ids], [sv.apd90(i) for i in ids])
        sv.close()
    at32, at64 = np.concatenate(res["fp32"][0]), np.concatenate(res["fp64"][0])
    ap32, ap64 = np.concatenate(res["fp32"][1]), np.concatenate(res["fp64"][1])
    out["uq_vs_gpu_fp64"] = {"workload": f"first {n_uq} UQ instances ({at32.size} tets), 500 ms",
                             "at_ms": _err_stats(at32, at64), "apd90_ms": _err_stats(ap32, ap64)}
    return out


def run_bidomain(ep, meshgen, args):
    """The paper's benchmark box (20 x 7 x 3 mm, fibres along x, TP06, 1.5 mm
    corner stimulus) at dx = 0.5, 0.2, 0.1 mm: wall time of one bidomain step
    (FP64, GMRES(30) to a relative residual of 1e-6 from the previous
    extracellular potential) and of one monodomain step, during the
    upstroke, on the library stream."""
    import torch
    out = []
    for h in (0.5, 0.2, 0.1):
        w = meshgen.niederer_box(h=h, dt=0.005, n_steps=args.steps)
        w.bidomain = meshgen.Bidomain(tol=1e-6, restart=30)
        b = ep.Sim(w, prec=ep.EP_FP64)
        b.step(args.warmup)
        b.sync()
        t0 = time.perf_counter()
        b.step(args.steps)
        b.sync()
        tb = (time.perf_counter() - t0) / args.steps
        last, total, rr = b.bidomain_stats()
        b.close()
        w.bidomain = None
        m = ep.Sim(w, prec=ep.EP_FP64)
        m.step(args.warmup)
        m.sync()
        t0 = time.perf_counter()
        m.step(args.steps)
        m.sync()
        tm = (time.perf_counter() - t0) / args.steps
        m.close()
        r = {"dx_mm": h, "tets": w.n_tets, "bidomain_s_per_step": tb, "monodomain_s_per_step": tm,
             "gmres_steps_per_time_step": total / (args.warmup + args.steps)}
        log(f"box dx={h}: {w.n_tets} tets, bidomain {tb * 1e3:.2f} ms/step "
            f"({r['gmres_steps_per_time_step']:.0f} GMRES steps), monodomain {tm * 1e3:.3f} ms/step")
        out.append(r)
    print(json.dumps({"metric": "wall time per time step (s), bidomain vs monodomain, FP64",
                      "workload": "box-20x7x3mm, dt 0.005 ms, GMRES(30) rtol 1e-6",
                      "steps": args.steps, "warmup": args.warmup, "grids": out}), flush=True)


def run_heart(ep, meshgen, args):
    """Three coupled media: the synthetic biventricle + atrial cap + Purkinje
    tree (~11.6M tets, 60k graph nodes, dt 0.01 ms), FP32-mixed and FP64."""
    t0 = time.time()
    w = meshgen.heart(h=0.375, scale=1.0, purkinje_nodes=60000, n_pmj=2000)
    log(f"workload {w.name}: {w.n_tets} tets, {w.purkinje.xyz.shape[0]} graph nodes, "
        f"{len(w.purkinje.pmj_nodes)} junctions ({time.time() - t0:.1f}s)")
    f32 = run_precision(ep, w, ep.EP_FP32_MIXED, args.steps, args.warmup, args.chunk, args.steps)
    f64 = run_precision(ep, w, ep.EP_FP64, args.steps, args.warmup, args.chunk, args.steps)
    achieved = f32["cell_bytes"] / (f32["cell_kernel_ms"] * 1e-3) / 1e9
    out = {
        "metric": "cell-steps/s (ionic+FV step) FP32 vs FP64; p50/p99 solve latency",
        "value": f32["cell_steps_per_s"], "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64conc", "data": "synthetic",
        "config": {"workload": w.name, "n_tets": w.n_tets, "n_nodes": w.n_nodes,
                   "graph_nodes": int(w.purkinje.xyz.shape[0]),
                   "junctions": int(len(w.purkinje.pmj_nodes)), "dt_ms": w.dt,
                   "cells": {"tp06": int((w.model <= 2).sum()), "crn": int((w.model == 3).sum())}},
        "latency_ms": {"p50": f32["p50_ms"], "p99": f32["p99_ms"],
                       "per": f"step (timed in chunks of {args.chunk} steps)"},
        "graph": {"substeps": f32["graph_substeps"],
                  "node_steps_per_s_fp32": f32["graph_node_steps_per_s"],
                  "node_steps_per_s_fp64": f64["graph_node_steps_per_s"]},
        "fp64": {"value": f64["cell_steps_per_s"], "ms_per_step": f64["ms_per_step"],
                 "cell_kernel_ms": f64["cell_kernel_ms"], "node_kernel_ms": f64["node_kernel_ms"]},
        "kernels_fp32": {"cell_kernel_ms": f32["cell_kernel_ms"],
                         "node_kernel_ms": f32["node_kernel_ms"]},
        "roofline": {"bound": "hbm", "kernel": "k_cell<float> (fused flux+ionic+update)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_ab2(ep, meshgen, args):
    """The default slab with the non-gating states stepped by Adams-Bashforth
    2 (Sec. 4) instead of forward Euler: cost of the extra rate history."""
    t0 = time.time()
    w = meshgen.config2(n_steps=args.steps, nx=args.nx, ny=args.ny, nz=args.nz)
    w.time_scheme = args.ab2
    tag = "ab2" if args.ab2 == 1 else "rl2-ab2"
    log(f"workload {w.name} ({tag}): {w.n_tets} tets ({time.time() - t0:.1f}s)")
    res = {}
    for name, prec in (("fp32", ep.EP_FP32_MIXED), ("fp64", ep.EP_FP64)):
        r = run_precision(ep, w, prec, args.steps, args.warmup, args.chunk, args.steps)
        r["cell_GBps"] = r["cell_bytes"] / (r["cell_kernel_ms"] * 1e-3) / 1e9
        res[name] = r
    f32 = res["fp32"]
    out = {
        "metric": "cell-steps/s (ionic+FV step, " + ("Adams-Bashforth 2 non-gating states)"
                   if args.ab2 == 1 else "second-order Rush-Larsen + Adams-Bashforth 2)"),
        "value": f32["cell_steps_per_s"], "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64conc", "data": "synthetic",
        "config": {"workload": w.name + "-" + tag, "n_tets": w.n_tets, "dt_ms": w.dt},
        "fp64": {"value": res["fp64"]["cell_steps_per_s"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "cell_kernel_ms": res["fp64"]["cell_kernel_ms"],
                 "cell_GBps": res["fp64"]["cell_GBps"], "cell_bytes": res["fp64"]["cell_bytes"]},
        "roofline": {"bound": "hbm", "kernel": f"k_cell<float, scheme {args.ab2}>", "achieved": f32["cell_GBps"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": f32["cell_GBps"] / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes": f32["cell_bytes"]},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_sheet(ep, meshgen, args):
    """A 2D medium of 5.12M triangles (the paper's Purkinje-shell
    discretisation, Sec. 3.2): a 400 x 400 mm TP06 sheet at h = 0.25 mm."""
    t0 = time.time()
    w = meshgen.sheet_workload(1600, 1600, 0.25, n_steps=args.steps)
    log(f"workload {w.name}: {w.n_tets} triangles, {w.n_nodes} nodes ({time.time() - t0:.1f}s)")
    res = {}
    for name, prec in (("fp32", ep.EP_FP32_MIXED), ("fp64", ep.EP_FP64)):
        r = run_precision(ep, w, prec, args.steps, args.warmup, args.chunk, args.steps)
        r["cell_GBps"] = r["cell_bytes"] / (r["cell_kernel_ms"] * 1e-3) / 1e9
        res[name] = r
    f32 = res["fp32"]
    out = {
        "metric": "cell-steps/s (ionic+FV step on triangles)",
        "value": f32["cell_steps_per_s"], "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64conc", "data": "synthetic",
        "config": {"workload": w.name, "n_cells": w.n_tets, "n_nodes": w.n_nodes, "dt_ms": w.dt},
        "fp64": {"value": res["fp64"]["cell_steps_per_s"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "cell_kernel_ms": res["fp64"]["cell_kernel_ms"],
                 "node_kernel_ms": res["fp64"]["node_kernel_ms"]},
        "kernels_fp32": {"cell_kernel_ms": f32["cell_kernel_ms"],
                         "node_kernel_ms": f32["node_kernel_ms"]},
        "roofline": {"bound": "hbm", "kernel": "k_cell<float> on triangles",
                     "achieved": f32["cell_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": f32["cell_GBps"] / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes": f32["cell_bytes"]},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000,
                    help="timed steps (default: the slab's whole 400 ms job)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--chunk", type=int, default=50,
                    help="steps per timed launch (one HIP graph of 50 steps)")
    ap.add_argument("--nx", type=int, default=160)
    ap.add_argument("--ny", type=int, default=160)
    ap.add_argument("--nz", type=int, default=40)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--only-fp32", action="store_true",
                    help="FP32-mixed only (short profiling runs)")
    ap.add_argument("--only-fp64", action="store_true",
                    help="FP64 only (short profiling runs)")
    ap.add_argument("--serving", type=str, default="32x2500", metavar="NxSTEPS",
                    help="serving stream sample (requests x steps each; '0' skips; "
                         "the full stream is 256x15000)")
    ap.add_argument("--serve-rate", type=float, default=17.0, metavar="PER_S",
                    help="Poisson arrival rate of the serving stream (requests/s)")
    ap.add_argument("--uq", type=str, default="1024x2000", metavar="NxSTEPS",
                    help="UQ batch sample (instances x steps; '0' skips; the full "
                         "batch is 1024x25000)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32-vs-FP64 error distributions")
    ap.add_argument("--bidomain", action="store_true",
                    help="bidomain vs monodomain step time on the paper's benchmark box")
    ap.add_argument("--sheet", action="store_true",
                    help="a 2D medium of 5.12M triangles instead of the slab")
    ap.add_argument("--ab2", type=int, nargs="?", const=1, default=0, metavar="SCHEME",
                    help="the slab with Adams-Bashforth 2 for the non-gating states "
                         "(1), also with second-order Rush-Larsen gates (2)")
    ap.add_argument("--heart", action="store_true",
                    help="the three-media heart instead of the slab (timed steps only)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB ten times "
                         "(calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        x = torch.ones(args.copy_calib * 2**20 // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calib} MiB x 10")
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: spreading instances or mesh partitions "
              "over several GPUs is designed, not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_12854_amd import ep, meshgen
    ep.lib()
    torch.cuda.init()
    if args.heart:
        return run_heart(ep, meshgen, args)
    if args.bidomain:
        return run_bidomain(ep, meshgen, args)
    if args.ab2:
        return run_ab2(ep, meshgen, args)
    if args.sheet:
        return run_sheet(ep, meshgen, args)
    t0 = time.time()
    w = meshgen.config2(n_steps=args.steps, nx=args.nx, ny=args.ny, nz=args.nz)
    log(f"workload {w.name}: {w.n_tets} tets, {w.n_nodes} nodes ({time.time() - t0:.1f}s)")

    if args.only_fp64:
        run_precision(ep, w, ep.EP_FP64, args.steps, args.warmup, args.chunk, args.steps)
        return
    # the serving and UQ legs first: each starts from the state a serving
    # process starts in (device memory and streams of the slab runs, still
    # held by this process, made the stream's latency less repeatable)
    serving = uq = None
    if not (args.only_fp32 or args.serving == "0"):
        nreq, nst = (int(x) for x in args.serving.split("x"))
        log(f"serving stream: {nreq} requests x {nst} steps (batched FP32-mixed) ...")
        bat = run_serving(ep, nreq, nst, args.serve_rate, prec=ep.EP_FP32_MIXED)
        log(f"  p50 {bat['p50_s']:.3f}s p99 {bat['p99_s']:.3f}s, {bat['cell_steps_per_s']:.3e} cell-steps/s")
        log("serving stream: one at a time, FP64 ...")
        one = run_serving(ep, nreq, nst, args.serve_rate, prec=ep.EP_FP64, one_at_a_time=True)
        log(f"  p50 {one['p50_s']:.3f}s p99 {one['p99_s']:.3f}s, {one['cell_steps_per_s']:.3e} cell-steps/s")
        serving = {"workload": f"{nreq} slab requests, 1e4-1e6 tets log-uniform, sigma scale "
                               f"U[0.5,2], random stimulus face, {nst} steps each, Poisson "
                               f"arrivals at a fixed {args.serve_rate:g} requests/s",
                   "batched_fp32": bat, "one_at_a_time_fp64": one}
    if not (args.only_fp32 or args.uq == "0"):
        ni, nst = (int(x) for x in args.uq.split("x"))
        uq = {}
        for name, prec in (("fp32", ep.EP_FP32_MIXED), ("fp64", ep.EP_FP64)):
            log(f"UQ batch {name}: {ni} instances x {nst} steps ...")
            uq[name] = run_uq(ep, ni, nst, prec)
            log(f"  {uq[name]['cell_steps_per_s']:.3e} cell-steps/s "
                f"(k={uq[name]['steps_per_graph']}, remap={uq[name]['xcd_remap']})")
    f32 = run_precision(ep, w, ep.EP_FP32_MIXED, args.steps, args.warmup, args.chunk, args.steps)
    f64 = None if (args.no_fp64 or args.only_fp32) else run_precision(ep, w, ep.EP_FP64, args.steps,
                                                  args.warmup, args.chunk, args.steps)
    hbm = None if args.only_fp32 else measure_hbm()
    acc = None
    if not (args.only_fp32 or args.no_accuracy):
        log("FP32 accuracy (500 ms runs) ...")
        acc = fp32_accuracy(ep, meshgen)
        log(f"  slab: AT max {acc['slab_vs_gpu_fp64']['at_ms']['max']:.4f} ms, "
            f"APD90 max {acc['slab_vs_gpu_fp64']['apd90_ms']['max']:.4f} ms")
    cpu = None
    if not (args.no_cpu or args.only_fp32):
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_steps, 80, 80, 40)
        log(f"cpu baseline {cpu['value']:.3e} cell-steps/s on {cpu['cores']} threads")

    achieved = f32["cell_bytes"] / (f32["cell_kernel_ms"] * 1e-3) / 1e9
    out = {
        "metric": "cell-steps/s (ionic+FV step) FP32 vs FP64; p50/p99 solve latency",
        "value": f32["cell_steps_per_s"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64conc",
        "data": "synthetic",
        "config": {"workload": w.name, "n_tets": w.n_tets, "n_nodes": w.n_nodes,
                   "dt_ms": w.dt, "cells": "TP06 endo/mid/epi 30/40/30%",
                   "fibres": "-60..+60 deg transmural + 5 deg jitter"},
        "latency_ms": {"p50": f32["p50_ms"], "p99": f32["p99_ms"],
                       "per": f"step (timed in chunks of {args.chunk} steps)"},
        "fp64": None if f64 is None else {
            "value": f64["cell_steps_per_s"], "ms_per_step": f64["ms_per_step"],
            "p50_ms": f64["p50_ms"], "p99_ms": f64["p99_ms"],
            "cell_kernel_ms": f64["cell_kernel_ms"], "node_kernel_ms": f64["node_kernel_ms"],
            "cell_kernel_GBps": f64["cell_bytes"] / (f64["cell_kernel_ms"] * 1e-3) / 1e9,
            "cell_bytes": f64["cell_bytes"], "node_bytes": f64["node_bytes"],
            "traffic": measured_traffic("fp64")},
        "kernels_fp32": {"cell_kernel_ms": f32["cell_kernel_ms"],
                         "node_kernel_ms": f32["node_kernel_ms"],
                         "node_kernel_GBps": f32["node_bytes"] / (f32["node_kernel_ms"] * 1e-3) / 1e9,
                         "cell_bytes": f32["cell_bytes"], "node_bytes": f32["node_bytes"]},
        "roofline": {"bound": "hbm", "kernel": "k_cell<float> (fused flux+ionic+update)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("fp32"),
                     "algorithmic_bytes": f32["cell_bytes"]},
        "cpu_baseline": cpu,
        "hbm_measured_GBps": hbm,
        "serving": serving,
        "uq_batch": uq,
        "fp32_error": acc,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
