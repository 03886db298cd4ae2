"""The stored FP64 oracle runs of the full-size workloads
(tests/golden/make_oracle_golden.py) checked on the CPU: they belong to the
inputs the generators make now (input hash), and they show what the
physiology fixes, independently of any GPU result: every sampled cell
activates, activation time grows with the distance from the stimulated
corner (conduction from the corner, Sec. 4), action potentials last as long
as a ventricular TP06 cell's (about 300 ms, with the mid-myocardial layer
longer than the others), and cells far from the corner are still at rest
50 ms in.  The GPU comparison against them is in test_gpu_golden.py.
"""
import json
import os

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fixture(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written yet (tests/golden/make_oracle_golden.py)")
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    d["info"] = json.loads(str(d["info"]))
    return d


def ranks(x):
    r = np.empty(x.size)
    r[np.argsort(x, kind="stable")] = np.arange(x.size)
    return r


def centroids(w, cells):
    return w.xyz[w.tets[cells]].mean(axis=1)


def test_slab_fixture_physiology():
    g = fixture("slab_400ms_oracle.npz")
    w = M.config2(n_steps=g["info"]["steps"])
    assert M.workload_sha256(w) == g["info"]["sha256"]
    c = g["cells"]
    assert c.size == 100_000 and np.all(np.diff(c) > 0) and c[-1] < w.n_tets
    at, apd, v50, vend = g["t_act"], g["apd90"], g["v_50ms"], g["v_end"]
    # everything activates within the 400 ms, from the corner outwards: the
    # stimulated cube first (during its pulse), the cells farthest from it
    # last.  The front is elongated along the fibres, which turn through
    # 120 degrees across the wall, so Euclidean distance orders activation
    # only roughly (rank correlation well above 0.8, not near 1).
    assert np.isfinite(at).all() and at.min() >= 0.0 and at.max() < 400.0
    xyz = centroids(w, c)
    d = np.linalg.norm(xyz, axis=1)
    cube = np.all(xyz <= 1.5, axis=1)
    assert cube.any() and at[cube].max() < 3.0
    rho = np.corrcoef(ranks(d), ranks(at))[0, 1]
    assert rho > 0.8, rho
    assert d[at >= np.percentile(at, 99)].min() > 0.7 * d.max()
    # apparent speed from the corner of every cell beyond 5 mm: between the
    # transverse and the longitudinal conduction speed of ventricular
    # tissue (0.2-0.8 m/s)
    far = d > 5.0
    speed = d[far] / at[far]                    # mm/ms = m/s
    assert speed.min() > 0.2 and speed.max() < 0.8, (speed.min(), speed.max())
    # APD90 of the cells that repolarise: ventricular TP06 lengths, mid-wall
    # cells longest
    ok = np.isfinite(apd)
    assert ok.mean() > 0.2
    assert 200.0 < np.median(apd[ok]) < 400.0
    model = w.model[c]
    mid, epi = (model == M.TP06_MID) & ok, (model == M.TP06_EPI) & ok
    if mid.any() and epi.any():
        assert np.median(apd[mid]) > np.median(apd[epi])
    # 50 ms in: the cells activated by then are depolarised, the far ones at rest
    assert np.all(v50[at < 40.0] > -40.0)
    late = at > 70.0
    assert late.any() and np.all(np.abs(v50[late] + 86.2) < 2.0)
    assert np.isfinite(vend).all()


def test_uq_fixture_physiology():
    g = fixture("uq64_500ms_oracle.npz")
    specs = M.uq_instances(n=1024, seed=5)
    idx, offs = g["instance"], g["offsets"]
    assert idx.size == 64 and offs[-1] == g["cells"].size
    med, score = [], []
    for k, i in enumerate(idx):
        w = M.uq_workload(specs[int(i)], g["info"]["steps"])
        assert M.workload_sha256(w) == g["info"]["sha256"][k]
        a, b = offs[k], offs[k + 1]
        c, at, apd = g["cells"][a:b], g["t_act"][a:b], g["apd90"][a:b]
        assert np.isfinite(at).all() and at.max() < 250.0
        d = centroids(w, c)[:, 0]               # stimulated on the x = 0 face
        assert np.corrcoef(ranks(d), ranks(at))[0, 1] > 0.9
        # all repolarised by 500 ms, at lengths that follow the conductance
        # scales (a larger G_Kr or G_Ks shortens the action potential)
        assert np.isfinite(apd).all() and 150.0 < np.median(apd) < 450.0
        assert np.isfinite(g["v_end"][a:b]).all()
        sp = specs[int(i)]
        med.append(np.median(apd))
        score.append(sp["GCaL"] - 0.5 * (sp["GKr"] + sp["GKs"]))
    # more inward calcium current lengthens the plateau, more repolarising
    # potassium current shortens it: across the instances the median APD90
    # follows G_CaL - (G_Kr + G_Ks) / 2 in rank
    assert np.corrcoef(ranks(np.array(score)), ranks(np.array(med)))[0, 1] > 0.7
