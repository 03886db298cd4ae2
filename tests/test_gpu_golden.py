"""The whole benchmark jobs against the FP64 oracle's stored runs of the same
seeded inputs (tests/golden/make_oracle_golden.py, keyed by the sha256 of
the inputs): the 5.12M-tet rotating-fibre slab over its full 400 ms (20,000
steps, a seeded sample of 100,000 cells) in the launch configuration the
benchmark times, and 64 instances of the UQ batch over 500 ms (25,000 steps,
1,500 sampled cells each) batched in one server as the benchmark runs them.

Bars: FP64 V within 1e-6 mV, activation time and APD90 within 1e-6 ms, the
same undefined (NaN) results; FP32-mixed activation time within 0.5 ms and
APD90 within 1 ms wherever both are defined, at most 1 in 10,000 sampled
cells defined on one side only (a cell repolarising within rounding of the
run's end).
"""
import json
import os

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LAUNCH = (256, 50, 1)


@pytest.fixture(scope="module")
def ep():
    from paper_2112_12854_amd import ep as _ep
    _ep.lib()
    return _ep


def say(msg):
    print(msg, flush=True)


def fixture(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written yet (tests/golden/make_oracle_golden.py)")
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    d["info"] = json.loads(str(d["info"]))
    return d


def check(prec_fp64, got, ref, what):
    at, apd, v = got
    rat, rapd, rv = ref
    if prec_fp64:
        assert np.array_equal(np.isnan(at), np.isnan(rat)), what
        assert np.array_equal(np.isnan(apd), np.isnan(rapd)), what
        f = np.isfinite(rat)
        assert np.max(np.abs(at[f] - rat[f])) <= 1e-6, what
        f = np.isfinite(rapd)
        if f.any():
            assert np.max(np.abs(apd[f] - rapd[f])) <= 1e-6, what
        dv = np.max(np.abs(v - rv))
        assert dv <= 1e-6, (what, dv)
        return dv
    for x, r, tol in ((at, rat, 0.5), (apd, rapd, 1.0)):
        one = np.isfinite(x) != np.isfinite(r)
        assert one.sum() <= max(0, x.size // 10000), (what, int(one.sum()))
        f = np.isfinite(x) & np.isfinite(r)
        if f.any():
            err = np.max(np.abs(x[f] - r[f]))
            assert err <= tol, (what, err)
    return float(np.max(np.abs(v - rv)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_slab_400ms_against_stored_oracle(ep, prec):
    g = fixture("slab_400ms_oracle.npz")
    w = M.config2(n_steps=g["info"]["steps"])
    assert M.workload_sha256(w) == g["info"]["sha256"], "the fixture is of other inputs"
    c = g["cells"]
    p = ep.EP_FP64 if prec == "fp64" else ep.EP_FP32_MIXED
    say(f"slab {w.n_tets} tets, {w.n_steps} steps, {prec}, {c.size} sampled cells")
    sim = ep.Sim(w, prec=p, allocator="torch", launch=LAUNCH)
    if prec == "fp32":
        sim.set_tile_size(128)    # a tile the benchmark's autotuner may pick
    sim.step(2500)
    v50 = sim.vm()[c]
    if prec == "fp64":
        assert np.max(np.abs(v50 - g["v_50ms"])) <= 1e-6
    sim.step(w.n_steps - 2500)
    dv = check(prec == "fp64", (sim.activation()[c], sim.apd90()[c], sim.vm()[c]),
               (g["t_act"], g["apd90"], g["v_end"]), "slab")
    sim.close()
    say(f"  max |dV| at 400 ms {dv:.2e} mV")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uq64_500ms_against_stored_oracle(ep, prec):
    g = fixture("uq64_500ms_oracle.npz")
    specs = M.uq_instances(n=1024, seed=5)
    idx, offs, steps = g["instance"], g["offsets"], g["info"]["steps"]
    ws = [M.uq_workload(specs[int(i)], steps) for i in idx]
    assert [M.workload_sha256(x) for x in ws] == g["info"]["sha256"], "other inputs"
    p = ep.EP_FP64 if prec == "fp64" else ep.EP_FP32_MIXED
    say(f"{len(ws)} UQ instances ({sum(x.n_tets for x in ws)} tets), {steps} steps, {prec}")
    sv = ep.Server(prec=p, max_slots=len(ws))
    try:
        ids = [sv.submit(x, steps) for x in ws]
        worst = 0.0
        for k, rid in enumerate(ids):
            assert sv.wait(rid)["status"] == ep.EP_OK
            cc = g["cells"][offs[k]:offs[k + 1]]
            a, b = offs[k], offs[k + 1]
            got = (sv.activation(rid)[cc], sv.apd90(rid)[cc], sv.vm(rid)[cc])
            ref = (g["t_act"][a:b], g["apd90"][a:b], g["v_end"][a:b])
            worst = max(worst, check(prec == "fp64", got, ref, f"instance {int(idx[k])}"))
    finally:
        sv.close()
    say(f"  max |dV| at 500 ms {worst:.2e} mV")
