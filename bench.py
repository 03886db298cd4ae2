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
# the files that define the cell kernel's code (its source and compiler
# flags); the counters in the traffic profile hold while their hash matches
KERNEL_SOURCES = ("paper_2112_12854_amd/csrc/kernels.hpp", "paper_2112_12854_amd/csrc/cellmodels.hpp",
                  "paper_2112_12854_amd/build.py")
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


FIXED_LAUNCH = None   # (tile cells, steps per graph, XCD remap) from --launch, else autotuned
PROFILE_EVERY = 8     # timed region: the kernels of every PROFILE_EVERY-th step carry events


def run_precision(ep, w, prec, steps, warmup, chunk, lat_steps=200, diffusion_reps=0):
    """One precision on workload w.  The timed region is `steps` steps by
    direct launches on the simulation's stream; the kernels of every
    PROFILE_EVERY-th step of it are timed by the start and end timestamps of
    their own dispatch (HIP events set by the launch; the others launch
    plainly, which keeps the events' own cost out of the throughput); the
    queue stays at least 64 timed steps deep, so the kernels run back to
    back.  The throughput and the kernel durations of the roofline come from
    the same window.  Then
    `lat_steps` more event-timed steps give the per-step latency
    distribution and `diffusion_reps` applications of the diffusion operator
    alone are timed with events on the same stream.  Last, a fresh
    simulation runs the same steps in the production schedule the autotuner
    chose (HIP graphs or direct launches, cell tile size), wall-clock timed
    between device synchronisations, so both windows cover the same part of
    the job."""
    import torch
    t0 = time.time()
    sim = ep.Sim(w, prec=prec, allocator="torch", trace_every=50)
    log(f"prec={prec}: init {time.time() - t0:.1f}s, footprint {sim.footprint() / 2**30:.2f} GiB")
    sim.set_launch(256, chunk, 1)
    sim.step(warmup)
    # schedule and cell tile shape from the autotuner (its trials are
    # ordinary steps of the same job, before the timed region)
    if FIXED_LAUNCH is None:
        tuned = sim.autotune(20)
    else:
        sim.set_launch(*FIXED_LAUNCH)
        tuned = {"ms_per_step": None}
    sim.sync()
    start_step, _ = sim.time()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    cell_ms, node_ms, per = sim.profile_steps(steps, per_step=True, every=PROFILE_EVERY)
    sim.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log(f"prec={prec}: {steps} steps in {elapsed:.3f}s (event-timed launches)")
    _, _, lat = sim.profile_steps(lat_steps, per_step=True)
    launch = sim.launch()
    node_b, cell_b, diff_b = sim.algorithmic_bytes(with_diffusion=True)
    at = sim.activation()
    n_sub = sim.purkinje_n_sub() if sim.n_purkinje else 0
    diff = None
    if diffusion_reps:
        diff = time_diffusion(ep, sim, w, diffusion_reps)
        diff["bytes"] = diff_b
        diff["GBps"] = diff_b / (diff["ms"] * 1e-3) / 1e9
    sim.close()
    # the production schedule over the same steps of the job
    prod = ep.Sim(w, prec=prec, allocator="torch", trace_every=50)
    prod.set_launch(256, launch["steps_per_graph"], launch["xcd_remap"])
    prod.set_tile_size(launch["tile_cells"])
    prod.step(start_step)
    prod.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prod.step(steps)
    prod.sync()
    torch.cuda.synchronize()
    graph_elapsed = time.perf_counter() - t1
    prod.close()
    return dict(ms_per_step=1e3 * elapsed / steps,
                graph_ms_per_step=1e3 * graph_elapsed / steps,
                graph_node_steps_per_s=sim.n_purkinje * n_sub * steps / elapsed,
                graph_substeps=n_sub,
                cell_steps_per_s=w.n_tets * steps / elapsed,
                p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)),
                n_latency=int(lat.size),
                timed_p50_ms=float(np.percentile(per, 50)), timed_kernel_steps=int(per.size),
                cell_kernel_ms=cell_ms, node_kernel_ms=node_ms,
                cell_bytes=cell_b, node_bytes=node_b,
                activated=int(np.isfinite(at).sum()), diffusion_op=diff,
                launch=launch, tuned_ms_per_step=tuned["ms_per_step"], timed_from_step=start_step)


def time_diffusion(ep, sim, w, reps):
    """The diffusion operator alone (ep_apply_diffusion_noalloc: three
    kernels, no allocation, no wait) applied `reps` times to a device field,
    bracketed by events on the simulation's stream."""
    import ctypes as C
    import torch
    st = sim._stream
    v = torch.linspace(-85.0, 30.0, w.n_tets, dtype=torch.float64, device="cuda")
    L = torch.empty_like(v)
    torch.cuda.synchronize()
    fn = ep.lib().ep_apply_diffusion_noalloc
    args = (sim.h, C.c_void_p(v.data_ptr()), C.c_void_p(L.data_ptr()), w.n_tets)
    assert fn(*args) == ep.EP_OK
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn(*args)
    e1.record(st)
    torch.cuda.synchronize()
    return {"ms": e0.elapsed_time(e1) / reps, "reps": reps,
            "kernels": "k_diff_in + k_diff_nodes + k_diff_out"}


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


def host_cpu_model() -> str:
    """The host CPU's model name, family/model/stepping and core count as the
    kernel reports them."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                info[k] = v.strip()
            if len(info) == 4:
                break
    except OSError:
        pass
    return (f"{info.get('model name', 'unknown')} (family {info.get('cpu family', '?')}, "
            f"model {info.get('model', '?')}, stepping {info.get('stepping', '?')})")


def cpu_baseline(steps: int, nx: int, ny: int, nz: int):
    """The oracle (as it stands, built -O3 -march=native for this host, no
    fast-math, no FMA contraction) on a sub-slab of the same recipe, on all
    host threads, then on one thread (beside the paper's single-core
    figure)."""
    import oracle
    from paper_2112_12854_amd import meshgen
    oracle.use_native()
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
    return dict(value=w.n_tets * steps / el, unit="cell-steps/s",
                cores=threads, kind="oracle",
                sample=f"{w.n_tets} tets ({nx}x{ny}x{nz} hexes of the same slab recipe, "
                       f"h=0.25 mm), {steps} FP64 steps after 2 untimed, {el:.1f} s",
                single_thread={"value": w.n_tets * s1 / el1, "steps": s1},
                build=" ".join(oracle.build_flags()),
                host_cpu=host_cpu_model(), host_cpus_visible=os.cpu_count())


def _pct(x):
    x = np.asarray(x, dtype=np.float64)
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)),
            "mean": float(x.mean()), "max": float(x.max())}


def saturated_rate(ep, ws, n_steps, prec, trial=20):
    """Cell-steps/s of the server with the workloads ws all resident (held
    until admitted, autotuned, then measured from the live progress counter
    up to 90 % of the work issued)."""
    sv = ep.Server(prec=prec, max_slots=len(ws))
    sv.hold(True)
    ids = [sv.submit(w, n_steps) for w in ws]
    t0 = time.perf_counter()
    while sv.stats()["running"] < len(ws):
        if time.perf_counter() - t0 > 300:
            raise RuntimeError("calibration batch did not become resident")
        time.sleep(0.01)
    sv.autotune(trial)
    sv.hold(False)
    while sv.stats()["autotune_runs"] < 1:
        time.sleep(0.005)
    st1, t1 = sv.stats(), time.perf_counter()
    goal = 0.9 * sum(w.n_tets for w in ws) * n_steps
    while True:
        st2, t2 = sv.stats(), time.perf_counter()
        if st2["cell_steps"] >= goal or st2["completed"] == len(ws):
            break
        time.sleep(0.002)
    for r in ids:
        sv.wait(r)
    sv.close()
    if st2["cell_steps"] <= st1["cell_steps"] or t2 <= t1:
        raise RuntimeError("calibration window empty: the autotuner's trials took every step")
    return (st2["cell_steps"] - st1["cell_steps"]) / (t2 - t1)


def run_serving(ep, ws, arrivals, n_steps, prec=None, one_at_a_time=False, trial=20):
    """Serving stream: the workloads ws submitted at the given arrival times
    (s); continuous batching with the autotuned schedule (re-tuned as the
    batch grows or shrinks), or one request at a time.  Latency = completion
    - submission, split into host precompute, wait for memory or a slot, and
    the device run."""
    n_req = len(ws)
    work = np.array([w.n_tets * n_steps for w in ws], dtype=np.float64)
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
                mean_s=float(lat.mean()), n_requests=n_req, steps=n_steps,
                cell_steps_per_s=float(work.sum() / span), span_s=span,
                breakdown_s={"precompute": _pct([r["t_ready"] - r["t_submit"] for r in res]),
                             "wait": _pct([r["t_admit"] - r["t_ready"] for r in res]),
                             "device": _pct([r["t_done"] - r["t_admit"] for r in res])},
                mean_tets=float(np.mean([w.n_tets for w in ws])),
                steps_per_graph=st["steps_per_graph"], xcd_remap=st["xcd_remap"],
                tile_cells=st["tile_cells"],
                autotune_runs=st["autotune_runs"])


def serving_leg(ep, meshgen, n_req, n_steps, load, n_fp64, seed=4):
    """Config-4 stream: n_req slab requests (1e4-1e6 tets log-uniform), each
    n_steps, Poisson arrivals at `load` x the measured capacity (the
    saturated FP32-mixed rate of the server on the stream's first 16
    requests over the stream's mean work per request); batched FP32-mixed
    on the whole stream, FP64 one request at a time on its first n_fp64
    requests at the same arrival times."""
    specs = meshgen.serving_requests(n=n_req, seed=seed)
    ws = [meshgen.serving_workload(sp, n_steps) for sp in specs]
    mean_work = float(np.mean([w.n_tets for w in ws])) * n_steps
    cal_steps = 4000      # the autotuner's trials take up to ~1,400 of them
    rate = saturated_rate(ep, ws[:16], cal_steps, ep.EP_FP32_MIXED)
    capacity = rate / mean_work
    lam = load * capacity
    log(f"serving: capacity {capacity:.2f} requests/s ({rate:.3e} cell-steps/s saturated), "
        f"arrivals at {lam:.2f}/s")
    rng = np.random.default_rng(seed + 1000)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
    log(f"serving stream: {n_req} requests x {n_steps} steps (batched FP32-mixed) ...")
    bat = run_serving(ep, ws, arrivals, n_steps, prec=ep.EP_FP32_MIXED)
    log(f"  p50 {bat['p50_s']:.3f}s p99 {bat['p99_s']:.3f}s, {bat['cell_steps_per_s']:.3e} cell-steps/s")
    one = None
    if n_fp64:
        log(f"serving stream: first {n_fp64} requests one at a time, FP64 ...")
        one = run_serving(ep, ws[:n_fp64], arrivals[:n_fp64], n_steps, prec=ep.EP_FP64,
                          one_at_a_time=True)
        log(f"  p50 {one['p50_s']:.3f}s p99 {one['p99_s']:.3f}s, "
            f"{one['cell_steps_per_s']:.3e} cell-steps/s")
    return {"workload": f"{n_req} slab requests, 1e4-1e6 tets log-uniform, sigma scale "
                        f"U[0.5,2], random stimulus face, {n_steps} steps each, Poisson "
                        f"arrivals at {load:g} x measured capacity",
            "capacity": {"requests_per_s": capacity, "saturated_cell_steps_per_s": rate,
                         "calibration": f"first 16 requests of the stream, {cal_steps} steps, "
                                        "all resident, FP32-mixed"},
            "arrival_rate_per_s": lam,
            "batched_fp32": bat,
            "one_at_a_time_fp64": one,
            "one_at_a_time_fp64_subset": f"first {n_fp64} requests of the same stream, "
                                         "same arrival times" if n_fp64 else None}


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
                tile_cells=st1["tile_cells"],
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


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    d["info"] = json.loads(str(d["info"]))
    return d


def _vs(a, b):
    return {"at_ms": _err_stats(a[0], b[0]), "apd90_ms": _err_stats(a[1], b[1]),
            "v_end_mV": _err_stats(a[2], b[2]),
            "nan_pattern_equal": bool(np.array_equal(np.isnan(a[0]), np.isnan(b[0])) and
                                      np.array_equal(np.isnan(a[1]), np.isnan(b[1])))}


def accuracy_vs_oracle(ep, meshgen):
    """FP32-mixed and FP64 error per result against the FP64 oracle's stored
    run of the same seeded inputs (tests/golden, keyed by input hash): the
    benchmark slab's whole 400 ms job (a seeded sample of 100,000 cells) and
    64 instances of the UQ batch over 500 ms (1,500 sampled cells each)."""
    out = {}
    g = _golden("slab_400ms_oracle.npz")
    if g is not None:
        w = meshgen.config2(n_steps=g["info"]["steps"])
        if meshgen.workload_sha256(w) != g["info"]["sha256"]:
            raise RuntimeError("slab oracle fixture is of other inputs")
        c = g["cells"]
        ref = (g["t_act"], g["apd90"], g["v_end"])
        r = {"workload": f"{w.name}: {w.n_tets} tets, {w.n_steps} steps, "
                         f"{c.size} sampled cells", "oracle_seconds": g["info"]["seconds"]}
        for name, prec in (("fp32", ep.EP_FP32_MIXED), ("fp64", ep.EP_FP64)):
            sim = ep.Sim(w, prec=prec)
            sim.step(w.n_steps)
            r[name] = _vs((sim.activation()[c], sim.apd90()[c], sim.vm()[c]), ref)
            sim.close()
        out["slab_vs_oracle"] = r
    g = _golden("uq64_500ms_oracle.npz")
    if g is not None:
        specs = meshgen.uq_instances(n=1024, seed=5)
        idx, offs = g["instance"], g["offsets"]
        ws = [meshgen.uq_workload(specs[int(i)], g["info"]["steps"]) for i in idx]
        if [meshgen.workload_sha256(x) for x in ws] != g["info"]["sha256"]:
            raise RuntimeError("UQ oracle fixture is of other inputs")
        ref = (g["t_act"], g["apd90"], g["v_end"])
        r = {"workload": f"{len(ws)} UQ instances ({sum(x.n_tets for x in ws)} tets), "
                         f"{g['info']['steps']} steps, {g['cells'].size} sampled cells"}
        for name, prec in (("fp32", ep.EP_FP32_MIXED), ("fp64", ep.EP_FP64)):
            sv = ep.Server(prec=prec, max_slots=len(ws))
            ids = [sv.submit(x, g["info"]["steps"]) for x in ws]
            at, apd, ve = [], [], []
            for k, i in enumerate(ids):
                sv.wait(i)
                cc = g["cells"][offs[k]:offs[k + 1]]
                at.append(sv.activation(i)[cc])
                apd.append(sv.apd90(i)[cc])
                ve.append(sv.vm(i)[cc])
            sv.close()
            r[name] = _vs((np.concatenate(at), np.concatenate(apd), np.concatenate(ve)), ref)
        out["uq_vs_oracle"] = r
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
        _, total0, _ = b.bidomain_stats()
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
             "gmres_steps_per_time_step": (total - total0) / args.steps}
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
    w = meshgen.config3()
    log(f"workload {w.name}: {w.n_tets} tets, {w.purkinje.xyz.shape[0]} graph nodes, "
        f"{len(w.purkinje.pmj_nodes)} junctions ({time.time() - t0:.1f}s)")
    f32 = run_precision(ep, w, ep.EP_FP32_MIXED, args.steps, args.warmup, args.chunk)
    f64 = run_precision(ep, w, ep.EP_FP64, args.steps, args.warmup, args.chunk)
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
        r = run_precision(ep, w, prec, args.steps, args.warmup, args.chunk)
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
        r = run_precision(ep, w, prec, args.steps, args.warmup, args.chunk)
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
    global FIXED_LAUNCH, PROFILE_EVERY
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000,
                    help="timed steps (default: the slab's whole 400 ms job)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--launch", default=None, metavar="TILE,K,REMAP",
                    help="fix the slab legs' launch (cell tile size, steps per HIP graph, "
                         "XCD remap 0/1/2) instead of autotuning it")
    ap.add_argument("--profile-every", type=int, default=PROFILE_EVERY, metavar="N",
                    help="time the kernels of every N-th step of the timed region with "
                         "dispatch events (1: every step)")
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
    ap.add_argument("--serving", type=str, default="256x15000", metavar="NxSTEPS",
                    help="serving stream (requests x steps each; '0' skips)")
    ap.add_argument("--serve-load", type=float, default=0.7, metavar="FRAC",
                    help="Poisson arrival rate as a fraction of the measured capacity")
    ap.add_argument("--serve-fp64", type=int, default=32, metavar="N",
                    help="requests of the stream served one at a time in FP64 (0 skips)")
    ap.add_argument("--uq", type=str, default="1024x25000", metavar="NxSTEPS",
                    help="UQ batch, FP32-mixed (instances x steps; '0' skips)")
    ap.add_argument("--uq-fp64-steps", type=int, default=2500,
                    help="steps of the FP64 UQ batch (0 skips)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the error distributions against the oracle")
    ap.add_argument("--diffusion-reps", type=int, default=50,
                    help="applications of the diffusion operator alone to time (0 skips)")
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
    if args.launch:
        FIXED_LAUNCH = tuple(int(x) for x in args.launch.split(","))
    if args.profile_every < 1:
        sys.exit("--profile-every must be at least 1")
    PROFILE_EVERY = args.profile_every
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
        r = run_precision(ep, w, ep.EP_FP64, args.steps, args.warmup, args.chunk)
        print(json.dumps({"metric": "cell-steps/s (ionic+FV step), FP64 only", "value": r["cell_steps_per_s"],
                          "unit": "cell-steps/s", "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": r["ms_per_step"], "ms_per_step_production": r["graph_ms_per_step"],
                          "launch": r["launch"], "cell_kernel_ms": r["cell_kernel_ms"],
                          "node_kernel_ms": r["node_kernel_ms"], "cell_bytes": r["cell_bytes"],
                          "node_bytes": r["node_bytes"], "config": {"workload": w.name}}), flush=True)
        return
    # the serving and UQ legs first: each starts from the state a serving
    # process starts in (device memory and streams of the slab runs, still
    # held by this process, made the stream's latency less repeatable)
    serving = uq = None
    if not (args.only_fp32 or args.serving == "0"):
        nreq, nst = (int(x) for x in args.serving.split("x"))
        serving = serving_leg(ep, meshgen, nreq, nst, args.serve_load, args.serve_fp64)
    if not (args.only_fp32 or args.uq == "0"):
        ni, nst = (int(x) for x in args.uq.split("x"))
        uq = {}
        for name, prec, k in (("fp32", ep.EP_FP32_MIXED, nst), ("fp64", ep.EP_FP64, args.uq_fp64_steps)):
            if k <= 0:
                continue
            log(f"UQ batch {name}: {ni} instances x {k} steps ...")
            uq[name] = run_uq(ep, ni, k, prec)
            log(f"  {uq[name]['cell_steps_per_s']:.3e} cell-steps/s "
                f"(k={uq[name]['steps_per_graph']}, remap={uq[name]['xcd_remap']})")
    f32 = run_precision(ep, w, ep.EP_FP32_MIXED, args.steps, args.warmup, args.chunk,
                        diffusion_reps=args.diffusion_reps)
    f64 = None if (args.no_fp64 or args.only_fp32) else run_precision(
        ep, w, ep.EP_FP64, args.steps, args.warmup, args.chunk, diffusion_reps=args.diffusion_reps)
    hbm = None if args.only_fp32 else measure_hbm()
    acc = None
    if not (args.only_fp32 or args.no_accuracy):
        log("accuracy against the oracle's stored runs ...")
        acc = accuracy_vs_oracle(ep, meshgen)
        if not acc:
            log("  no oracle fixtures: FP32 against the GPU FP64 path (500 ms runs) ...")
            acc = fp32_accuracy(ep, meshgen)
        for k, v in acc.items():
            if isinstance(v, dict) and "fp32" in v:
                log(f"  {k}: FP32 AT max {v['fp32']['at_ms']['max']:.4f} ms, "
                    f"APD90 max {v['fp32']['apd90_ms']['max']:.4f} ms; FP64 V max "
                    f"{v['fp64']['v_end_mV']['max']:.2e} mV")
            elif isinstance(v, dict) and "at_ms" in v:
                log(f"  {k}: AT max {v['at_ms']['max']:.4f} ms, APD90 max {v['apd90_ms']['max']:.4f} ms")
    cpu = None
    if not (args.no_cpu or args.only_fp32):
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_steps, 80, 80, 40)
        log(f"cpu baseline {cpu['value']:.3e} cell-steps/s on {cpu['cores']} threads")

    achieved = f32["cell_bytes"] / (f32["cell_kernel_ms"] * 1e-3) / 1e9

    def gbps(b, ms):
        return b / (ms * 1e-3) / 1e9

    def sweep(r):
        """The diffusion sweep: the node gather of the step (its only kernel
        that does nothing else) and the operator alone (three kernels)."""
        d = {"node_gather": {"achieved": gbps(r["node_bytes"], r["node_kernel_ms"]),
                             "frac": gbps(r["node_bytes"], r["node_kernel_ms"]) / HBM_PEAK_GBS,
                             "ms": r["node_kernel_ms"], "algorithmic_bytes": r["node_bytes"]},
             "step": {"achieved": gbps(r["node_bytes"] + r["cell_bytes"],
                                       r["node_kernel_ms"] + r["cell_kernel_ms"]),
                      "frac": gbps(r["node_bytes"] + r["cell_bytes"],
                                   r["node_kernel_ms"] + r["cell_kernel_ms"]) / HBM_PEAK_GBS}}
        if r["diffusion_op"]:
            op = r["diffusion_op"]
            d["operator_alone"] = dict(op, frac=op["GBps"] / HBM_PEAK_GBS)
        d["peak"], d["unit"] = HBM_PEAK_GBS, "GB/s"
        return d

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
        "timed_region": f"direct launches in the autotuned tile size and XCD remap; the kernels "
                        f"of every {PROFILE_EVERY}th step ({f32['timed_kernel_steps']} steps) "
                        f"carry HIP events set from their own dispatch's start and end (the "
                        f"roofline's kernel durations), the others launch plainly; wall clock "
                        f"between device synchronisations",
        "timed_from_step": f32["timed_from_step"],
        "launch": f32["launch"],
        "ms_per_step_production": f32["graph_ms_per_step"],
        "production": "the autotuned launch (tile size, HIP graph length or direct, XCD remap) "
                      "on a fresh simulation over the same steps, wall clock between syncs",
        "latency_ms": {"p50": f32["p50_ms"], "p99": f32["p99_ms"], "n": f32["n_latency"],
                       "per": "step: device time from its first kernel's start to its last "
                              "kernel's end, consecutive event-timed steps after the timed region"},
        "fp64": None if f64 is None else {
            "value": f64["cell_steps_per_s"], "ms_per_step": f64["ms_per_step"],
            "ms_per_step_production": f64["graph_ms_per_step"], "launch": f64["launch"],
            "p50_ms": f64["p50_ms"], "p99_ms": f64["p99_ms"], "n_latency": f64["n_latency"],
            "cell_kernel_ms": f64["cell_kernel_ms"], "node_kernel_ms": f64["node_kernel_ms"],
            "cell_kernel_GBps": gbps(f64["cell_bytes"], f64["cell_kernel_ms"]),
            "cell_bytes": f64["cell_bytes"], "node_bytes": f64["node_bytes"],
            "traffic": measured_traffic("fp64"), "diffusion_sweep": sweep(f64)},
        "kernels_fp32": {"cell_kernel_ms": f32["cell_kernel_ms"],
                         "node_kernel_ms": f32["node_kernel_ms"],
                         "node_kernel_GBps": gbps(f32["node_bytes"], f32["node_kernel_ms"]),
                         "cell_bytes": f32["cell_bytes"], "node_bytes": f32["node_bytes"]},
        "roofline": {"bound": "hbm", "kernel": "k_cell<float> (fused flux+ionic+update)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("fp32"),
                     "algorithmic_bytes": f32["cell_bytes"]},
        "diffusion_sweep": sweep(f32),
        "cpu_baseline": cpu,
        "hbm_measured_GBps": hbm,
        "serving": serving,
        "uq_batch": uq,
        "accuracy": acc,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
