"""Pathology and pacing scenarios (Sec. 6) in the oracle: what the paper
states about each case, checked on seeded synthetic inputs.

- Bundle-branch block: a null conductivity of one bundle branch stops the
  wave in that branch of the Purkinje network, and the chamber it served
  activates later (only through the myocardium); a partial delay slows the
  branch more the more severe it is.
- AV block: with the atrio-ventricular conduction cut, nothing drives the
  Purkinje network or the ventricles.
- Pacing lead: a stimulus on the myocardium at the lead reaches the
  Purkinje network through its junctions (antidromic, two-way coupling)
  and then the rest of the network.

Windows stay below 18 ms: from the Stewart article's initial state an
unstimulated Purkinje cell fires by itself at 20.3 ms (checked below), which
would mask the scenarios.
"""
import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M
from paper_2112_12854_amd import scenarios as S


def test_stewart_automaticity_window(oracle_lib):
    """The Purkinje cell model is self-exciting: the first unstimulated
    upstroke comes at about 20 ms, after which the cycle is about 0.63 s."""
    t, v = oracle_lib.single_cell(M.STEWART, 700.0, 0.02, stim_amp=0.0)
    up = t[np.nonzero((v[:-1] <= 0) & (v[1:] > 0))[0]]
    assert 19.0 < up[0] < 22.0
    assert 550.0 < up[1] - up[0] < 700.0


def node_side(pk):
    side = np.full(pk.xyz.shape[0], -1)
    side[pk.edges[:, 1]] = pk.edge_side
    return side


@pytest.fixture(scope="module")
def small_heart():
    w = M.heart(h=1.0, scale=0.3, purkinje_nodes=1500, n_pmj=60)
    w.stimuli[-1].t0 = 0.0                  # His root driven at t = 0
    return w


def test_right_bundle_branch_block(oracle_lib, small_heart):
    w = small_heart
    pk = w.purkinje
    side = node_side(pk)
    root_ball = np.linalg.norm(pk.xyz - pk.xyz[0], axis=1) <= 0.5
    runs = {}
    for name, ww in (("healthy", w), ("rbbb", S.bundle_branch_block(w, "right"))):
        o = oracle_lib.Sim(ww)
        o.step(1800)
        runs[name] = (o.purkinje_activation(), o.activation())
    pa_h, ta_h = runs["healthy"]
    pa_b, ta_b = runs["rbbb"]
    # healthy: both branches conduct
    assert np.isfinite(pa_h[side == 0]).all() and np.isfinite(pa_h[side == 1]).all()
    # block: the right branch stays silent past the directly stimulated root
    assert not np.isfinite(pa_b[(side == 1) & ~root_ball]).any()
    assert np.isfinite(pa_b[side == 0]).all()
    # the myocardium served by the right junctions activates later: fewer
    # cells by 18 ms
    assert np.isfinite(ta_b).sum() < 0.9 * np.isfinite(ta_h).sum()


def test_bundle_delay_grows_with_severity(oracle_lib):
    """Graph-driven slab with a two-branch network: lowering branch 0's
    conductivity delays its leaf monotonically and leaves the other
    branch's leaf nearly unchanged."""
    w = M.purkinje_slab(drive="graph")
    leaf = w.purkinje.pmj_nodes
    t0, t1 = [], []
    for sev in (0.0, 0.5, 0.8):
        o = oracle_lib.Sim(S.bundle_branch_block(w, "left", sev))
        o.step(600)
        pa = o.purkinje_activation()
        t0.append(pa[leaf[0]])
        t1.append(pa[leaf[1]])
    assert np.isfinite(t0).all() and np.isfinite(t1).all()
    assert t0[0] < t0[1] < t0[2]
    # cable theory: the branch's conduction time grows like 1/sqrt(1 - sev)
    assert (t0[2] - t0[0]) > (t0[1] - t0[0]) * 1.5
    assert max(t1) - min(t1) < 0.1 * (t0[2] - t0[0])


def test_av_block_and_ventricular_lead(oracle_lib):
    """AV block alone: no activation anywhere.  With a lead on the muscle
    at the first junction and two-way junctions: the network is entered
    antidromically at that junction and conducts to the other one, whose
    muscle region then activates orthodromically."""
    w = M.purkinje_slab(drive="graph", pmj_amp=-1000.0)
    blocked = S.av_block(w)
    assert all(st.domain == 0 for st in blocked.stimuli)
    o = oracle_lib.Sim(blocked)
    o.step(700)
    assert not np.isfinite(o.activation()).any()
    assert not np.isfinite(o.purkinje_activation()).any()

    leaf = w.purkinje.pmj_nodes
    paced = S.two_way_junctions(S.pacing_lead(blocked, w.purkinje.xyz[leaf[0]], radius=1.0))
    o = oracle_lib.Sim(paced)
    o.step(700)
    pa, ta = o.purkinje_activation(), o.activation()
    assert np.isfinite(pa).all()
    assert pa[leaf[0]] < pa[leaf[1]]
    far = o.pmj_region(1)
    assert np.isfinite(ta[far]).all()
    # the far region was reached through the network: its cells activate
    # after its junction node does
    assert np.nanmin(ta[far]) > pa[leaf[1]]


def test_tissue_block_isolates_its_core(oracle_lib):
    """A ball of null conductivity: cells whose four neighbours are all
    inside carry no flux at all, so its core stays at rest while the
    surrounding slab activates."""
    w = M.config1(n_steps=0)
    cen = w.xyz[w.tets].mean(axis=1)
    centre = np.array([0.75, 0.5, 0.5]) * cen.max(axis=0)
    r = 0.3 * cen.max(axis=0)[0]
    b = S.tissue_block(w, centre, r)
    o = oracle_lib.Sim(b)
    o.step(1500)
    ta = o.activation()
    d = np.linalg.norm(cen - centre, axis=1)
    h = w.dims[3]
    assert np.isfinite(ta[d > r + h]).mean() > 0.99
    assert not np.isfinite(ta[d < r - 2 * h]).any()


def test_communication_node_spacing():
    """Sec. 3.3: nodes varsigma tau = 1 mm apart along the bundles; on a
    chain of 0.1 mm segments that is every tenth node, plus the far end;
    on the two-branch network each branch gets its own sequence."""
    from test_oracle_purkinje import chain_workload
    w = chain_workload(96, 0.1)
    cn = S.communication_nodes(w.purkinje)
    assert np.array_equal(cn, np.r_[np.arange(0, 96, 10), 95])
    y = M.purkinje_slab().purkinje
    cn = S.communication_nodes(y, spacing=1.0)
    assert set(y.pmj_nodes.tolist()) <= set(cn.tolist())
    # consecutive nodes along every path are at most spacing + one segment apart
    x = y.xyz
    d = np.linalg.norm(x[cn][:, None] - x[cn][None], axis=2)
    np.fill_diagonal(d, np.inf)
    assert d.min(axis=1).max() <= 1.0 + 0.1 + 1e-9


def test_bundle_coupling_speeds_the_atrium(oracle_lib):
    """A fast bundle (the graph) laid through a CRN atrial slab, both driven
    at x = 0 and coupled by communication nodes (R_S = 1 mm, no delay): the
    wave reaches the far half of the slab earlier than through the atrial
    tissue alone, and the nodes' regions activate in the order of their
    distance from the driven root."""
    w = M.purkinje_slab(drive="graph", nx=40, ny=8, nz=2, n_steps=0)
    w.model = np.full(w.n_tets, M.CRN, np.uint8)
    w.purkinje.pmj_nodes = np.array([], np.int32)
    x = w.xyz[w.tets].mean(axis=1)[:, 0]
    w.stimuli.append(M.Stimulus(ids=np.nonzero(x < 1.0)[0].astype(np.int32), t0=0.0, dur=2.0,
                                amp=-40.0))
    coupled = S.bundle_coupling(w, radius=1.0)
    ta = {}
    regions = None
    for name, ww in (("plain", w), ("coupled", coupled)):
        o = oracle_lib.Sim(ww)
        o.step(1000)
        ta[name] = o.activation()
        if name == "coupled":
            regions = [o.pmj_region(k) for k in range(len(ww.purkinje.pmj_nodes))]
    far = (x > 12.0) & (x < 14.0)
    assert np.isfinite(ta["coupled"][far]).all()
    plain = np.where(np.isfinite(ta["plain"][far]), ta["plain"][far], np.inf)
    assert np.mean(ta["coupled"][far]) < plain.min() - 2.0
    # along the trunk (nodes on the line y = const before the fork): regions
    # activate in the order of their distance from the root
    pk = coupled.purkinje
    trunk = [k for k, i in enumerate(pk.pmj_nodes) if pk.edge_side is not None
             and i < (pk.edge_side == -1).sum()]
    t_reg = [np.nanmin(ta["coupled"][regions[k]]) for k in trunk]
    assert len(t_reg) >= 3 and np.all(np.diff(t_reg) > 0)
