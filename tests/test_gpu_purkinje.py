"""GPU parity of the Purkinje graph and the Purkinje-muscle junctions
(Sec. 3.2 graph, Sec. 3.3 coupling) through the C ABI, against the FP64
oracle on the same seeded slab-plus-graph inputs.

Bars: FP64 max|dV| <= 1e-6 mV on the tissue and on the graph, activation
times within 1e-6 ms (same NaN pattern); FP32-mixed activation times within
0.5 ms of the FP64 oracle.
"""
import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

pytestmark = pytest.mark.gpu

TOL_MV = 1e-6


@pytest.fixture(scope="module")
def ep():
    from paper_2112_12854_amd import ep as _ep
    _ep.lib()
    return _ep


def say(msg):
    print(msg, flush=True)


def same_times(a, b, tol):
    assert np.array_equal(np.isnan(a), np.isnan(b))
    f = np.isfinite(a)
    return float(np.max(np.abs(a[f] - b[f]))) if f.any() else 0.0


@pytest.mark.parametrize("drive,two_way", [("graph", False), ("tissue", True)])
def test_purkinje_fp64_parity(ep, oracle_lib, drive, two_way):
    w = M.purkinje_slab(drive=drive, two_way=two_way)
    say(f"purkinje parity fp64 drive={drive} two_way={two_way}: {w.n_tets} tets, "
        f"{w.purkinje.xyz.shape[0]} graph nodes")
    g = ep.Sim(w, prec=ep.EP_FP64)
    o = oracle_lib.Sim(w)
    assert g.purkinje_n_sub() == o.purkinje_n_sub()
    worst = 0.0
    for chunk in range(5):
        g.step(150)
        o.step(150)
        dv = np.max(np.abs(g.vm() - o.vm()))
        dp = np.max(np.abs(g.purkinje_vm() - o.purkinje_vm()))
        worst = max(worst, dv, dp)
        assert dv <= TOL_MV and dp <= TOL_MV, (chunk, dv, dp)
    assert same_times(g.activation(), o.activation(), 0) <= 1e-6
    assert same_times(g.purkinje_activation(), o.purkinje_activation(), 0) <= 1e-6
    # the coupling really fired in the direction under test
    assert np.isfinite(o.purkinje_activation()).all()
    assert np.isfinite(o.activation()).sum() > 0
    say(f"  max|dV| {worst:.2e} mV")


def test_purkinje_fp32_activation(ep, oracle_lib):
    w = M.purkinje_slab()
    g = ep.Sim(w, prec=ep.EP_FP32_MIXED)
    o = oracle_lib.Sim(w)
    g.step(750)
    o.step(750)
    assert same_times(g.purkinje_activation(), o.purkinje_activation(), 0) <= 0.5
    assert same_times(g.activation(), o.activation(), 0) <= 0.5


def test_purkinje_graphs_match_direct_and_checkpoint(ep):
    """Replayed HIP graphs equal direct launches bitwise, and a checkpoint
    restores the graph state (junction schedule included) bitwise."""
    w = M.purkinje_slab(drive="tissue", two_way=True)
    for prec in (ep.EP_FP64, ep.EP_FP32_MIXED):
        a = ep.Sim(w, prec=prec, launch=(256, 50, 1))
        b = ep.Sim(w, prec=prec, launch=(256, 0, 1))
        a.step(230)
        b.step(230)
        assert np.array_equal(a.purkinje_vm(), b.purkinje_vm())
        assert np.array_equal(a.vm(), b.vm())
        blob = a.checkpoint()
        a.step(370)
        c = ep.Sim(w, prec=prec)
        c.restore(blob)
        c.step(370)
        assert np.array_equal(a.purkinje_vm(), c.purkinje_vm())
        assert np.array_equal(a.purkinje_activation(), c.purkinje_activation(), equal_nan=True)
        assert np.array_equal(a.vm(), c.vm())


def test_purkinje_abi_errors(ep):
    import ctypes as C
    L = ep.lib()
    w = M.purkinje_slab()
    o = ep.ep_options()
    L.ep_default_options(C.byref(o))
    h = C.c_void_p()
    assert L.ep_create(C.byref(o), C.byref(h)) == ep.EP_OK
    try:
        xyz = np.ascontiguousarray(w.xyz)
        tets = np.ascontiguousarray(w.tets, np.int32)
        assert L.ep_set_mesh(h, w.n_nodes, ep._d(xyz), w.n_tets, tets.ctypes.data_as(ep._ip)) == 0
        ids = np.array([0], np.int32)
        # graph stimulus before a graph exists
        assert L.ep_add_stimulus(h, 1, 1, ids.ctypes.data_as(ep._ip), 0.0, 1.0, -50.0, 0.0, 1) == ep.EP_ESTATE
        assert L.ep_add_pmj(h, 0, 0.5, 5.0, 3.0, 0, -200.0, 0.5) == ep.EP_ESTATE
        px = np.ascontiguousarray(w.purkinje.xyz)
        bad = np.array([[0, 1], [1, 10**6]], np.int32)
        assert L.ep_set_purkinje(h, px.shape[0], ep._d(px), 2, bad.ctypes.data_as(ep._ip),
                                 3.95, M.STEWART, 0) == ep.EP_EINVAL
        e = np.ascontiguousarray(w.purkinje.edges, np.int32)
        assert L.ep_set_purkinje(h, px.shape[0], ep._d(px), e.shape[0], e.ctypes.data_as(ep._ip),
                                 -1.0, M.STEWART, 0) == ep.EP_EINVAL
        assert L.ep_set_purkinje(h, px.shape[0], ep._d(px), e.shape[0], e.ctypes.data_as(ep._ip),
                                 3.95, 9, 0) == ep.EP_EINVAL
        assert L.ep_set_purkinje(h, px.shape[0], ep._d(px), e.shape[0], e.ctypes.data_as(ep._ip),
                                 3.95, M.STEWART, 0) == ep.EP_OK
        assert L.ep_add_pmj(h, px.shape[0], 0.5, 5.0, 3.0, 0, -200.0, 0.5) == ep.EP_EINVAL
        big = np.array([px.shape[0]], np.int32)
        assert L.ep_add_stimulus(h, 1, 1, big.ctypes.data_as(ep._ip), 0.0, 1.0, -50.0, 0.0, 1) == ep.EP_EINVAL
        n = C.c_int32()
        assert L.ep_get_purkinje_substeps(h, C.byref(n)) == ep.EP_ESTATE
    finally:
        L.ep_destroy(h)


def test_heart_three_media_fp64_parity(ep, oracle_lib):
    """The synthetic three-media heart at a small scale: TP06 layers, the
    CRN atrial cap, the Stewart tree and its junctions in one instance (His
    root driven at t = 0 here), 20 ms: FP64 parity on tissue and graph, and
    the FP32-mixed activation times within 0.5 ms."""
    w = M.heart(h=1.0, scale=0.3, purkinje_nodes=1500, n_pmj=60)
    w.stimuli[-1].t0 = 0.0
    say(f"heart: {w.n_tets} tets, {w.purkinje.xyz.shape[0]} graph nodes, "
        f"{len(w.purkinje.pmj_nodes)} junctions")
    g = ep.Sim(w, prec=ep.EP_FP64)
    f = ep.Sim(w, prec=ep.EP_FP32_MIXED)
    o = oracle_lib.Sim(w)
    for chunk in range(4):
        g.step(500)
        f.step(500)
        o.step(500)
        dv = np.max(np.abs(g.vm() - o.vm()))
        dp = np.max(np.abs(g.purkinje_vm() - o.purkinje_vm()))
        assert dv <= TOL_MV and dp <= TOL_MV, (chunk, dv, dp)
    ta_o, pa_o = o.activation(), o.purkinje_activation()
    assert same_times(g.activation(), ta_o, 0) <= 1e-6
    assert same_times(g.purkinje_activation(), pa_o, 0) <= 1e-6
    assert np.isfinite(pa_o).all()
    # junction-driven ventricular cells activated (not only the atrial ball)
    assert np.isfinite(ta_o[w.model <= 2]).sum() > 0
    assert same_times(f.purkinje_activation(), pa_o, 0) <= 0.5
    assert same_times(f.activation(), ta_o, 0) <= 0.5
