"""Continuous batching on the GPU: requests of uneven size run together, join
while others run, are admitted by HBM footprint, and each result is the same
(bitwise) as the same request run alone.  A request that goes non-finite
fails alone."""
import time

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ep():
    from paper_2112_12854_amd import ep as _ep
    _ep.lib()
    return _ep


def say(msg):
    print(msg, flush=True)


def requests(n, seed=4, n_lo=2e3, n_hi=2e4, steps=600):
    specs = M.serving_requests(n=n, seed=seed, n_lo=n_lo, n_hi=n_hi)
    out = []
    rng = np.random.default_rng(seed)
    for sp in specs:
        w = M.serving_workload(sp, n_steps=steps)
        w.ionic_scale = {k: float(rng.uniform(0.7, 1.3)) for k in ("GKr", "GKs", "GCaL", "GNa")}
        out.append(w)
    return out


def alone(ep, w, prec, steps):
    s = ep.Sim(w, prec=prec)
    s.step(steps)
    return s.vm(), s.activation(), s.apd90()


@pytest.mark.parametrize("prec_name", ["EP_FP32_MIXED", "EP_FP64"])
def test_mix_equals_alone_bitwise(ep, prec_name):
    prec = getattr(ep, prec_name)
    steps = 600
    ws = requests(5, steps=steps)
    say(f"serving mix ({prec_name}): sizes {[w.n_tets for w in ws]}")
    sv = ep.Server(prec=prec, max_slots=8, steps_per_graph=50)
    ids = [sv.submit(ws[0], steps), sv.submit(ws[1], steps)]
    time.sleep(0.05)                       # the rest joins while these run
    ids += [sv.submit(w, steps) for w in ws[2:]]
    res = [sv.wait(i) for i in ids]
    assert all(r["status"] == ep.EP_OK for r in res)
    for w, i in zip(ws, ids):
        vm, at, apd = alone(ep, w, prec, steps)
        assert np.array_equal(sv.vm(i), vm)
        assert np.array_equal(sv.activation(i), at, equal_nan=True)
        assert np.array_equal(sv.apd90(i), apd, equal_nan=True)
    st = sv.stats()
    assert st["completed"] == len(ws) and st["running"] == 0
    assert st["cell_steps"] == sum(w.n_tets for w in ws) * steps
    sv.close()


def test_admission_by_footprint(ep):
    """A budget that holds only about two requests: all still finish, never
    more than the budget is resident, results unchanged."""
    steps = 300
    ws = requests(6, seed=7, steps=steps)
    probe = ep.Sim(ws[0], prec=ep.EP_FP32_MIXED)
    per_tet = probe.footprint() / ws[0].n_tets
    probe.close()
    budget = int(2.2 * per_tet * max(w.n_tets for w in ws))
    say(f"admission: budget {budget / 2**20:.1f} MiB for sizes {[w.n_tets for w in ws]}")
    sv = ep.Server(prec=ep.EP_FP32_MIXED, hbm_budget=budget, max_slots=16)
    ids = [sv.submit(w, steps) for w in ws]
    peak = 0
    while any(sv.poll(i) is None for i in ids):
        peak = max(peak, sv.stats()["bytes_in_use"])
        time.sleep(0.002)
    assert peak <= budget
    res = [sv.wait(i) for i in ids]
    assert all(r["status"] == ep.EP_OK for r in res)
    # with this budget some requests had to queue behind others
    assert max(r["t_admit"] for r in res) > min(r["t_done"] for r in res) - 1e-9
    for w, i in zip(ws[:2], ids[:2]):
        vm, at, _ = alone(ep, w, ep.EP_FP32_MIXED, steps)
        assert np.array_equal(sv.vm(i), vm)
    sv.close()


def test_nonfinite_request_fails_alone(ep):
    steps = 200
    ws = requests(3, seed=9, steps=steps)
    bad = requests(1, seed=10, steps=steps)[0]
    bad.stimuli[0].amp = -1e35             # drives v out of range -> non-finite
    sv = ep.Server(prec=ep.EP_FP32_MIXED, max_slots=8)
    ids = [sv.submit(w, steps) for w in ws]
    bid = sv.submit(bad, steps)
    res = {i: sv.wait(i) for i in ids + [bid]}
    assert res[bid]["status"] == ep.EP_ENUMERIC
    for w, i in zip(ws, ids):
        assert res[i]["status"] == ep.EP_OK
        vm, _, _ = alone(ep, w, ep.EP_FP32_MIXED, steps)
        assert np.array_equal(sv.vm(i), vm)
    sv.close()


def test_malformed_and_oversized_requests(ep):
    sv = ep.Server(prec=ep.EP_FP32_MIXED, hbm_budget=1 << 20, max_slots=2)
    w = requests(1, seed=3, n_lo=2e4, n_hi=3e4)[0]
    with pytest.raises(ep.EPError):
        sv.submit(w, 0)                    # no steps
    try:                                   # cannot fit 1 MiB
        rid = sv.submit(w, 10)
    except ep.EPError as e:
        assert e.status == ep.EP_ENOMEM
    else:
        assert sv.wait(rid)["status"] == ep.EP_ENOMEM
    sv.close()


def test_autotuned_schedule_keeps_results(ep):
    """The autotuner's trial steps are ordinary steps: a simulation tuned on
    the way, and a server batch tuned (and re-tuned as it grows) while it
    runs, give bitwise the results of a fixed schedule."""
    w = M.config1(nx=10, ny=8, nz=2)
    a = ep.Sim(w)
    choice = a.autotune(20)
    assert choice["steps_per_graph"] in (0, 10, 25, 50, 100)
    assert choice["xcd_remap"] in (0, 1, 2, 3) and choice["ms_per_step"] > 0
    assert choice["tile_cells"] in (256, 128, 64)
    # per remap: 20 direct steps, then each graph length k in whole graphs
    # (20, 25, 50, 100) after one untimed graph (1 + 10 + 25 + 50 + 100);
    # then three tile sizes at the chosen k, each an untimed graph (or one
    # direct step) and whole graphs covering 20 steps
    k = choice["steps_per_graph"]
    shape = (k if k > 0 else 1) + (-(-20 // k) * k if k > 0 else 20)
    used = 4 * (20 + 20 + 25 + 50 + 100) + 4 * (1 + 10 + 25 + 50 + 100) + 3 * shape
    assert a.time()[0] == used
    a.step(3000 - used)
    b = ep.Sim(w)
    b.step(3000)
    assert np.array_equal(a.vm(), b.vm())
    assert np.array_equal(a.apd90(), b.apd90(), equal_nan=True)

    steps = 900
    ws = requests(6, seed=9, steps=steps)
    sv = ep.Server(prec=ep.EP_FP32_MIXED, max_slots=8)
    sv.autotune(10, retune=True)
    ids = [sv.submit(x, steps) for x in ws]
    res = [sv.wait(i) for i in ids]
    assert all(r["status"] == ep.EP_OK for r in res)
    st = sv.stats()
    assert st["autotune_runs"] >= 1 and st["steps_per_graph"] in (10, 25, 50, 100)
    assert st["tile_cells"] in (256, 128, 64)
    for x, i in zip(ws, ids):
        vm, at, _ = alone(ep, x, ep.EP_FP32_MIXED, steps)
        assert np.array_equal(sv.vm(i), vm)
        assert np.array_equal(sv.activation(i), at, equal_nan=True)
    sv.close()


@pytest.mark.parametrize("which", ["slab", "mixed-substeps", "graph"])
def test_profiled_steps_keep_results(ep, which):
    """Steps timed by ep_profile_steps (kernels launched with events set
    from their own dispatch) are ordinary steps: bitwise the results of
    plain stepping, on a slab, a mixed tets + triangles mesh whose sheet
    takes substeps, and a slab with a Purkinje graph, with every step timed
    and with every third (100 timed steps, more than the ring of 64 events
    the host cycles through); every kernel time is positive and the two
    kernels fit inside their step."""
    if which == "slab":
        w = M.config1(nx=10, ny=8, nz=2)
    elif which == "mixed-substeps":
        w = M.mixed_workload(M.config1(n_steps=0, nx=8, ny=6, nz=2),
                             M.sheet_workload(12, 6, 0.5, model=M.CRN, n_steps=0))
        w.medium_substeps = 3
    else:
        w = M.purkinje_slab()
    n = 300
    for prec, every in ((ep.EP_FP32_MIXED, 1), (ep.EP_FP64, 1), (ep.EP_FP32_MIXED, 3),
                        (ep.EP_FP64, 3)):
        a = ep.Sim(w, prec=prec)
        a.step(5)
        cell_ms, node_ms, per = a.profile_steps(n, per_step=True, every=every)
        b = ep.Sim(w, prec=prec)
        b.step(5 + n)
        assert a.time()[0] == b.time()[0] == 5 + n
        assert np.array_equal(a.vm(), b.vm())
        assert np.array_equal(a.activation(), b.activation(), equal_nan=True)
        if which == "graph":
            assert np.array_equal(a.purkinje_vm(), b.purkinje_vm())
        assert per.shape == ((n + every - 1) // every,) and (per > 0).all()
        assert cell_ms > 0 and node_ms > 0
        assert cell_ms + node_ms <= float(np.median(per)) * 1.01
        say(f"{which} prec {prec} every {every}: cell {cell_ms * 1e3:.1f} us, "
            f"node {node_ms * 1e3:.1f} us, step p50 {np.median(per) * 1e3:.1f} us")
        with pytest.raises(ep.EPError):
            a.profile_steps(10, every=0)


@pytest.mark.parametrize("scheme", [1, 2])
def test_server_time_scheme_and_cell_junctions(ep, scheme):
    """A server whose requests step with Adams-Bashforth 2 (1) or the
    second-order Rush-Larsen variant (2): a plain slab, a slab with a graph
    and a shell-on-slab request with cell junctions, run together, each
    bitwise equal to the same workload run alone with that scheme; the
    scheme cannot change once requests have arrived."""
    plain = M.config1(n_steps=0)
    graph = M.purkinje_slab(drive="tissue", two_way=True)
    # (a 4x sheet: AB2's stable interval is half forward Euler's, and the
    # default 10x sheet exceeds it at dt = 0.02 ms)
    shell = M.shell_on_slab(drive="slab", two_way=True, sheet_scale=4.0)
    ws = [plain, graph, shell]
    for w in ws:
        w.time_scheme = scheme
    sv = ep.Server(prec=ep.EP_FP32_MIXED, dt=0.02, max_slots=4, time_scheme=scheme)
    try:
        ids = [sv.submit(w, 600) for w in ws]
        assert all(sv.wait(i)["status"] == ep.EP_OK for i in ids)
        for rid, w in zip(ids, ws):
            solo = ep.Sim(w, prec=ep.EP_FP32_MIXED)
            solo.step(600)
            assert np.array_equal(sv.vm(rid), solo.vm())
            assert np.array_equal(sv.activation(rid), solo.activation(), equal_nan=True)
        # the slab re-entered the shell through its two-way nodes
        assert np.isfinite(sv.activation(ids[2])[16 * 8 * 2 * 5:]).any()
        with pytest.raises(ep.EPError):
            sv._chk(ep.lib().ep_server_set_time_scheme(sv.h, 0))
    finally:
        sv.close()
