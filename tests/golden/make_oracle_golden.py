"""Write the FP64 oracle's results on the full-size workloads as test fixtures.

Only the CPU oracle (oracle/) computes anything here; the inputs come from
the seeded generators of meshgen.  Each fixture is keyed by the sha256 of its
workload's inputs (meshgen.workload_sha256), so a change of the generator
makes the GPU tests that read it fail instead of comparing other inputs.

  slab   The 40 x 40 x 10 mm rotating-fibre slab at h = 0.25 mm (5,120,000
         tets), 20,000 steps of 0.02 ms (400 ms).  At a seeded sample of
         100,000 cells: activation time, APD90, V at 50 ms and at 400 ms;
         over all cells: counts and moments of activation time and APD90.
  uq     64 instances of the UQ batch (seed 5), every 16th of the 1,024
         sorted by size (8k-64k tets across the range), each with its own
         conductance scales, 25,000 steps (500 ms).  At a seeded sample of
         1,500 cells per instance: activation time, APD90, V at 500 ms.

The oracle's results do not depend on its thread count.  A full slab run is
about 1e11 cell-steps (hours on a few cores).

Usage: python tests/golden/make_oracle_golden.py {slab|uq|merge-uq} [--threads N]
           [--native] [--ckpt DIR] [--shard i/n]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SLAB_FILE = os.path.join(HERE, "slab_400ms_oracle.npz")
UQ_FILE = os.path.join(HERE, "uq64_500ms_oracle.npz")
SLAB_SAMPLE, SLAB_SEED = 100_000, 12
UQ_COUNT, UQ_STRIDE, UQ_SAMPLE, UQ_SEED = 64, 16, 1_500, 13


def slab_workload():
    from paper_2112_12854_amd import meshgen
    return meshgen.config2(n_steps=20000)


def slab_sample(n_cells: int) -> np.ndarray:
    rng = np.random.default_rng(SLAB_SEED)
    return np.sort(rng.choice(n_cells, SLAB_SAMPLE, replace=False)).astype(np.int64)


def uq_subset():
    """(index in the 1,024-instance batch, spec) of the 64 instances."""
    from paper_2112_12854_amd import meshgen
    specs = meshgen.uq_instances(n=1024, seed=5)
    size = np.array([s["nx"] * s["ny"] for s in specs])
    order = np.argsort(size, kind="stable")
    pick = order[UQ_STRIDE // 2::UQ_STRIDE][:UQ_COUNT]
    return [(int(i), specs[i]) for i in pick]


def uq_sample(k: int, n_cells: int) -> np.ndarray:
    rng = np.random.default_rng([UQ_SEED, k])
    m = min(UQ_SAMPLE, n_cells)
    return np.sort(rng.choice(n_cells, m, replace=False)).astype(np.int64)


def _moments(x):
    f = x[np.isfinite(x)]
    return dict(n=int(f.size), mean=float(f.mean()) if f.size else None,
                min=float(f.min()) if f.size else None,
                max=float(f.max()) if f.size else None)


def _save_ckpt(path, s, **extra):
    tmp = path + ".tmp.npz"
    np.savez(tmp, states=s.states(), detection=s.detection(), step=s.step_index, **extra)
    os.replace(tmp, path)


def make_slab(log, ckpt_dir=None):
    import oracle
    from paper_2112_12854_amd import meshgen
    w = slab_workload()
    key = meshgen.workload_sha256(w)
    cells = slab_sample(w.n_tets)
    log(f"slab: {w.n_tets} tets, {w.n_steps} steps, key {key[:16]}")
    s = oracle.Sim(w)
    ck = os.path.join(ckpt_dir, f"slab_{key[:16]}.npz") if ckpt_dir else None
    v50, spent = None, 0.0
    if ck and os.path.exists(ck):
        with np.load(ck, allow_pickle=False) as z:
            s.set_states(z["states"])
            s.set_detection(z["detection"])
            s.set_step(int(z["step"]))
            spent = float(z["seconds"])
            if z["v_50ms"].size:
                v50 = z["v_50ms"]
        log(f"slab: resumed at step {s.step_index} ({spent:.0f} s spent before)")
    t0 = time.time() - spent
    while s.step_index < w.n_steps:
        k = min(2500 - s.step_index % 2500, w.n_steps - s.step_index)
        s.step(k)
        if s.step_index == 2500:
            v50 = s.vm()[cells]
        log(f"slab: step {s.step_index} after {time.time() - t0:.0f} s")
        if ck and s.step_index < w.n_steps:
            os.makedirs(ckpt_dir, exist_ok=True)
            _save_ckpt(ck, s, seconds=time.time() - t0,
                       v_50ms=v50 if v50 is not None else np.empty(0))
    at, apd, v400 = s.activation(), s.apd90(), s.vm()
    info = dict(workload=w.name, sha256=key, n_tets=w.n_tets, steps=w.n_steps, dt=w.dt,
                threads=oracle.num_threads(), seconds=time.time() - t0,
                oracle_flags=" ".join(oracle.build_flags()),
                activation_all=_moments(at), apd90_all=_moments(apd),
                v_end_all=_moments(v400), vbar_end=float(s.mean_vm()))
    np.savez_compressed(SLAB_FILE, cells=cells, t_act=at[cells], apd90=apd[cells],
                        v_50ms=v50, v_end=v400[cells], info=json.dumps(info))
    log(f"slab: wrote {SLAB_FILE} ({info['seconds']:.0f} s)")
    if ck and os.path.exists(ck):
        os.remove(ck)


def make_uq(log, shard=(0, 1)):
    """The UQ subset, or with shard (i, n) the instances k = i, i + n, ...
    of it into a part file (merged by `merge_uq`)."""
    import oracle
    from paper_2112_12854_amd import meshgen
    i_sh, n_sh = shard
    sub = uq_subset()
    keys, idx, offs, cells, at, apd, vend = [], [], [0], [], [], [], []
    t0 = time.time()
    for n, (i, sp) in enumerate(sub):
        if n % n_sh != i_sh:
            continue
        w = meshgen.uq_workload(sp, 25000)
        keys.append(meshgen.workload_sha256(w))
        s = oracle.Sim(w)
        s.step(w.n_steps)
        c = uq_sample(i, w.n_tets)
        idx.append(i)
        cells.append(c)
        offs.append(offs[-1] + c.size)
        at.append(s.activation()[c])
        apd.append(s.apd90()[c])
        vend.append(s.vm()[c])
        log(f"uq: instance {i} ({w.n_tets} tets) {n + 1}/{len(sub)} after {time.time() - t0:.0f} s")
        del s
    info = dict(batch="uq_instances(n=1024, seed=5)", steps=25000, dt=0.02,
                threads=oracle.num_threads(), seconds=time.time() - t0,
                oracle_flags=" ".join(oracle.build_flags()), sha256=keys)
    out = UQ_FILE if n_sh == 1 else UQ_FILE.replace(".npz", f".part{i_sh}of{n_sh}.npz")
    np.savez_compressed(out, instance=np.array(idx, np.int64),
                        offsets=np.array(offs, np.int64), cells=np.concatenate(cells),
                        t_act=np.concatenate(at), apd90=np.concatenate(apd),
                        v_end=np.concatenate(vend), info=json.dumps(info))
    log(f"uq: wrote {out} ({info['seconds']:.0f} s)")


def merge_uq(n_sh, log):
    """The part files of n_sh shards merged into one fixture, instances in
    the subset's order."""
    parts = [load(UQ_FILE.replace(".npz", f".part{i}of{n_sh}.npz")) for i in range(n_sh)]
    rows = []
    for p in parts:
        for k, inst in enumerate(p["instance"]):
            a, b = p["offsets"][k], p["offsets"][k + 1]
            rows.append((int(inst), p["info"]["sha256"][k], p["cells"][a:b], p["t_act"][a:b],
                         p["apd90"][a:b], p["v_end"][a:b]))
    order = {i: n for n, (i, _) in enumerate(uq_subset())}
    rows.sort(key=lambda r: order[r[0]])
    offs = np.cumsum([0] + [r[2].size for r in rows])
    info = dict(batch="uq_instances(n=1024, seed=5)", steps=25000, dt=0.02,
                threads=sum(p["info"]["threads"] for p in parts),
                seconds=max(p["info"]["seconds"] for p in parts),
                oracle_flags=parts[0]["info"]["oracle_flags"], sha256=[r[1] for r in rows],
                shards=n_sh)
    np.savez_compressed(UQ_FILE, instance=np.array([r[0] for r in rows], np.int64),
                        offsets=offs.astype(np.int64), cells=np.concatenate([r[2] for r in rows]),
                        t_act=np.concatenate([r[3] for r in rows]),
                        apd90=np.concatenate([r[4] for r in rows]),
                        v_end=np.concatenate([r[5] for r in rows]), info=json.dumps(info))
    log(f"uq: merged {n_sh} parts into {UQ_FILE} ({len(rows)} instances)")


def load(path):
    """The stored arrays and the info record of a fixture."""
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    d["info"] = json.loads(str(d["info"]))
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=("slab", "uq", "merge-uq"))
    ap.add_argument("--shard", default="0/1", help="i/n: the UQ instances k with k % n == i")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--ckpt", default=None,
                    help="directory for a resumable checkpoint of the slab run")
    ap.add_argument("--native", action="store_true",
                    help="use the -march=native copy of the oracle (same results)")
    a = ap.parse_args()
    import oracle
    if a.native:
        oracle.use_native()
    if a.threads:
        oracle.set_num_threads(a.threads)

    def log(m):
        print(f"[golden] {m}", flush=True)

    i_sh, n_sh = (int(x) for x in a.shard.split("/"))
    if a.which == "slab":
        make_slab(log, a.ckpt)
    elif a.which == "uq":
        make_uq(log, (i_sh, n_sh))
    else:
        merge_uq(n_sh, log)


if __name__ == "__main__":
    main()
