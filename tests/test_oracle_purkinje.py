"""Pins of the oracle's Purkinje graph and Purkinje-muscle junctions against
what the paper and the mathematics fix (Sec. 3.2 vertex-centred finite
volumes on 1D media, Sec. 3.3 junction coupling, Sec. 5 table: Stewart cells
with sigma = 3.95 mS/mm conduct at about 4 m/s).

Independent checks: a closed-form stability bound, charge balance of the
conservative graph flux, the textbook 1D Neumann finite-difference Laplacian
on a uniform chain (the vertex-centred scheme reduces to it), the measured
conduction velocity against the paper's table, brute-force junction regions,
and the integer-step timing of the junction pulses.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

HERE = os.path.dirname(os.path.abspath(__file__))
FACTS = json.load(open(os.path.join(HERE, "golden", "paper_facts.json")))
CHI_CM = M.CHI * M.CM


def chain_workload(n_nodes, L, model=M.STEWART, sigma=3.95, dt=0.02, stim_nodes=(),
                   stim_amp=-100.0, stim_dur=1.0, lengths=None, n_sub=0):
    """A straight graph along x next to a tiny passive slab (the tissue is
    only there because a simulation needs one; no junctions)."""
    w = M.config1(nx=2, ny=2, nz=1)
    w.model = np.full(w.n_tets, M.PASSIVE, np.uint8)
    w.stimuli = []
    w.dt = dt
    if lengths is None:
        lengths = np.full(n_nodes - 1, L)
    x = np.concatenate([[0.0], np.cumsum(lengths)])
    xyz = np.stack([x, np.full_like(x, 50.0), np.zeros_like(x)], axis=1)
    edges = np.stack([np.arange(n_nodes - 1), np.arange(1, n_nodes)], axis=1).astype(np.int32)
    w.purkinje = M.Purkinje(xyz=xyz, edges=edges, pmj_nodes=np.array([], np.int32),
                            sigma=sigma, model=model, n_sub=n_sub)
    if len(stim_nodes):
        w.stimuli.append(M.Stimulus(ids=np.array(stim_nodes, np.int32), t0=0.0, dur=stim_dur,
                                    amp=stim_amp, domain=1))
    return w


def test_substeps_closed_form(oracle_lib):
    """Uniform chain: every node has l_i sum_j 1/L_ij = 1 (interior: L * 2/L,
    ends: L/2 * 1/L), so the bound is chi Cm L^2 / (2 sigma)."""
    for L, dt in ((0.1, 0.02), (0.25, 0.02), (0.1, 0.01), (0.5, 0.05)):
        s = oracle_lib.Sim(chain_workload(20, L, dt=dt))
        bound = 0.9 * CHI_CM * L * L / (2 * 3.95)
        want = max(1, math.ceil(dt / bound - 1e-12))
        assert s.purkinje_n_sub() == want, (L, dt)


def test_substeps_nonuniform_chain(oracle_lib):
    """Segments 0.1 / 0.05 / 0.1 ...: the node between a long and a short
    segment has bound chi Cm L1 L2 / (2 sigma); the short end segment's node
    chi Cm L2^2 / (2 sigma) when it exists.  Minimum over nodes."""
    lengths = np.array([0.1, 0.05, 0.1, 0.1, 0.05, 0.1])
    s = oracle_lib.Sim(chain_workload(7, None, lengths=lengths))
    per_node = []
    ln = np.concatenate([[np.nan], lengths, [np.nan]])
    for i in range(7):
        a, b = ln[i], ln[i + 1]
        segs = [x for x in (a, b) if np.isfinite(x)]
        ell = 0.5 * sum(segs)
        inv = sum(1 / x for x in segs)
        per_node.append(CHI_CM * ell / (3.95 * inv))
    bound = 0.9 * min(per_node)
    assert s.purkinje_n_sub() == math.ceil(0.02 / bound - 1e-12)
    # explicit override is respected
    w = chain_workload(7, None, lengths=lengths, n_sub=40)
    assert oracle_lib.Sim(w).purkinje_n_sub() == 40


def test_graph_charge_balance_passive(oracle_lib):
    """Passive cells: sum_i l_i dv_i/dt = -sum_i l_i I_stim,i because the
    graph flux is conservative; after the pulse, sum_i l_i (v_i - v_0) =
    -amp * dur * sum_{stimulated} l_i (irregular segment lengths)."""
    rng = np.random.default_rng(4)
    lengths = rng.uniform(0.05, 0.2, 39)
    stim = [3, 4, 5, 17]
    w = chain_workload(40, None, model=M.PASSIVE, lengths=lengths, stim_nodes=stim,
                       stim_amp=-30.0, stim_dur=0.5)
    s = oracle_lib.Sim(w)
    v0 = s.purkinje_vm()
    s.step(100)
    v = s.purkinje_vm()
    ln = np.concatenate([[0.0], lengths, [0.0]])
    ell = 0.5 * (ln[:-1] + ln[1:])
    lhs = float(np.sum(ell * (v - v0)))
    rhs = 30.0 * 0.5 * float(np.sum(ell[stim]))
    assert lhs == pytest.approx(rhs, rel=1e-10)
    assert np.ptp(v) > 0.0          # the charge has spread unevenly


def test_graph_matches_textbook_fd_laplacian(oracle_lib):
    """On a uniform chain the vertex-centred scheme is the textbook
    finite-difference Laplacian with Neumann ends (ghost-node form:
    2 (v_1 - v_0) / L^2 at the ends).  Passive cells, a pulse on one node,
    explicit substeps: the oracle's graph potential equals the same
    recursion written with that matrix."""
    n, L, dt = 25, 0.1, 0.02
    w = chain_workload(n, L, model=M.PASSIVE, stim_nodes=[7], stim_amp=-40.0, stim_dur=0.1,
                       dt=dt)
    s = oracle_lib.Sim(w)
    nsub = s.purkinje_n_sub()
    dtp = dt / nsub
    A = np.zeros((n, n))
    for i in range(n):
        if 0 < i < n - 1:
            A[i, i - 1], A[i, i], A[i, i + 1] = 1.0, -2.0, 1.0
    A[0, 0], A[0, 1] = -2.0, 2.0
    A[-1, -1], A[-1, -2] = -2.0, 2.0
    A *= 3.95 / (CHI_CM * L * L)
    v = s.purkinje_vm().copy()
    n_steps = 40
    nstim = int(round(0.1 / dt))
    for step in range(n_steps):
        for _ in range(nsub):
            ist = np.zeros(n)
            if step < nstim:
                ist[7] = -40.0
            v = v + dtp * (A @ v - ist)
    s.step(n_steps)
    np.testing.assert_allclose(s.purkinje_vm(), v, rtol=0, atol=1e-10)


@pytest.mark.slow
def test_stewart_graph_conduction_velocity(oracle_lib):
    """Sec. 5 table: Purkinje (Stewart) with sigma = 3.95 mS/mm conducts at
    about 4 m/s.  A 24 mm chain of 0.1 mm segments, driven at one end; CV
    from the activation times 8 mm apart in the middle (15 % band)."""
    fact = FACTS["stewart_sigma_mS_per_mm"]
    w = chain_workload(241, 0.1, sigma=fact["value"], stim_nodes=list(range(5)),
                       stim_amp=-100.0, stim_dur=1.0)
    s = oracle_lib.Sim(w)
    s.step(500)
    ta = s.purkinje_activation()
    x = w.purkinje.xyz[:, 0]
    i0, i1 = np.argmin(abs(x - 8.0)), np.argmin(abs(x - 16.0))
    assert np.isfinite(ta[[i0, i1]]).all()
    cv = (x[i1] - x[i0]) / (ta[i1] - ta[i0])      # mm/ms = m/s
    assert cv == pytest.approx(fact["cv_m_per_s"], rel=0.15)


# ------------------------------------------------------------- junctions
def centroids(w):
    return w.xyz[w.tets].mean(axis=1)


def test_junction_region_radius(oracle_lib):
    """Region = the cells whose centroid lies within the radius (brute
    force over every cell)."""
    w = M.purkinje_slab()
    s = oracle_lib.Sim(w)
    cen = centroids(w)
    for k, node in enumerate(w.purkinje.pmj_nodes):
        d = np.linalg.norm(cen - w.purkinje.xyz[node], axis=1)
        want = np.nonzero(d <= w.purkinje.pmj_radius)[0]
        assert want.size > 0
        np.testing.assert_array_equal(np.sort(s.pmj_region(k)), want)


def test_junction_region_fallback(oracle_lib):
    """No centroid within the radius: the cells sharing a mesh node with the
    cell of nearest centroid."""
    w = M.purkinje_slab()
    w.purkinje.pmj_radius = 1e-3
    s = oracle_lib.Sim(w)
    cen = centroids(w)
    for k, node in enumerate(w.purkinje.pmj_nodes):
        d = np.linalg.norm(cen - w.purkinje.xyz[node], axis=1)
        near = int(np.argmin(d))
        shared = np.nonzero(np.isin(w.tets, w.tets[near]).any(axis=1))[0]
        np.testing.assert_array_equal(np.sort(s.pmj_region(k)), shared)


def test_orthodromic_pulse_timing(oracle_lib):
    """A junction whose node crosses the threshold during step n pulses its
    region from step n + 1 + round(delay/dt) for round(dur/dt) steps (Sec. 3.3
    delay of 5 ms): the region is at rest until that step, then each pulsed
    step raises it by about -amp dt."""
    w = M.purkinje_slab()
    pk = w.purkinje
    assert pk.delay_ortho == FACTS["pmj_orthodromic_delay_ms"]["value"]
    s = oracle_lib.Sim(w)
    dt = w.dt
    s.step(200)
    tn = s.purkinje_activation()[pk.pmj_nodes[0]]
    assert np.isfinite(tn)
    n_cross = int(math.floor(tn / dt))
    fire = n_cross + 1 + int(round(pk.delay_ortho / dt))
    region = s.pmj_region(0)
    v_rest = s.vm()[region]
    s.step(fire - 200)                  # steps 0 .. fire-1 done
    v_before = s.vm()[region]
    assert np.all(abs(v_before - v_rest) < 0.05)
    s.step(1)                           # step `fire`: first pulsed step
    rise = s.vm()[region] - v_before
    assert np.all(rise > 0.5 * (-pk.pmj_amp) * dt)


def test_antidromic_pulse_and_one_way(oracle_lib):
    """Two-way junction: the region's mean potential crossing the threshold
    during step n pulses the junction node from step n + 1 +
    round(delay_anti/dt); the graph then activates from that node.  One-way
    coupling leaves the graph at rest."""
    w = M.purkinje_slab(drive="tissue", two_way=True)
    pk = w.purkinje
    s = oracle_lib.Sim(w)
    region = s.pmj_region(0)
    dt = w.dt
    m_prev = s.vm()[region].mean()
    n_cross = None
    for n in range(200):
        s.step(1)
        m = s.vm()[region].mean()
        if m_prev <= 0.0 < m:
            n_cross = n
            break
        m_prev = m
    assert n_cross is not None
    fire = n_cross + 1 + int(round(pk.delay_anti / dt))
    s.step(fire - s.step_index)
    assert np.isnan(s.purkinje_activation()).all()     # nothing before the pulse
    s.step(400)
    ta = s.purkinje_activation()
    node = pk.pmj_nodes[0]
    assert fire * dt <= ta[node] < fire * dt + 1.0
    assert np.isfinite(ta).all()
    # one-way coupling: the graph never activates
    w1 = M.purkinje_slab(drive="tissue", two_way=False)
    s1 = oracle_lib.Sim(w1)
    s1.step(600)
    assert np.isnan(s1.purkinje_activation()).all()


# ------------------------------------------- segment conductivity (Sec. 6)
def test_segment_scale_matches_variable_coefficient_fd(oracle_lib):
    """Per-segment multipliers s_e (a bundle-branch delay lowers them, a
    block sets them to 0): on a uniform chain the scheme is the textbook
    conservative finite difference of (k v')' with k = sigma s at the
    half-points, (k+ (v_{i+1} - v_i) - k- (v_i - v_{i-1})) / L^2, Neumann
    ends by the ghost-node form (factor 2 at the ends); the substep count
    is the Gershgorin bound of that matrix."""
    n, L, dt = 30, 0.1, 0.02
    rng = np.random.default_rng(11)
    s_e = rng.uniform(0.2, 2.0, n - 1)
    s_e[[4, 20]] = 0.0
    w = chain_workload(n, L, model=M.PASSIVE, stim_nodes=[2, 10], stim_amp=-40.0,
                       stim_dur=0.2, dt=dt)
    w.purkinje.edge_scale = s_e
    s = oracle_lib.Sim(w)
    k = 3.95 * s_e / CHI_CM
    A = np.zeros((n, n))
    for i in range(n - 1):
        A[i, i + 1] += k[i]
        A[i + 1, i] += k[i]
        A[i, i] -= k[i]
        A[i + 1, i + 1] -= k[i]
    A /= L * L
    A[0] *= 2.0
    A[-1] *= 2.0
    lam = np.max(-np.diag(A) + np.abs(A - np.diag(np.diag(A))).sum(axis=1))
    nsub = s.purkinje_n_sub()
    assert nsub == max(1, math.ceil(dt * lam / (2 * 0.9) - 1e-12))
    dtp = dt / nsub
    v = s.purkinje_vm().copy()
    nstim = int(round(0.2 / dt))
    for step in range(40):
        for _ in range(nsub):
            ist = np.zeros(n)
            if step < nstim:
                ist[[2, 10]] = -40.0
            v = v + dtp * (A @ v - ist)
    s.step(40)
    got = s.purkinje_vm()
    np.testing.assert_allclose(got, v, rtol=0, atol=1e-10)
    # nothing crosses a blocked segment: the nodes past node 20 never move
    assert np.all(got[21:] == got[-1]) and got[-1] == w_rest(oracle_lib)


def w_rest(oracle_lib):
    return oracle_lib.model_init(M.PASSIVE)[0]


def test_blocked_leaf_evolves_as_an_isolated_cell(oracle_lib):
    """A complete block (s = 0) removes the segment's flux exactly: the
    leaf behind it follows the single-cell Stewart model integrated with the
    graph substep, while the driven chain in front of it activates."""
    n, L, dt = 40, 0.1, 0.02
    s_e = np.ones(n - 1)
    s_e[-1] = 0.0
    w = chain_workload(n, L, stim_nodes=list(range(5)), dt=dt)
    w.purkinje.edge_scale = s_e
    s = oracle_lib.Sim(w)
    nsub = s.purkinje_n_sub()
    steps = 400
    s.step(steps)
    _, trace = oracle_lib.single_cell(M.STEWART, steps * dt, dt / nsub, stim_amp=0.0)
    assert s.purkinje_vm()[-1] == pytest.approx(trace[-1], abs=1e-12)
    ta = s.purkinje_activation()
    assert np.isfinite(ta[:-1]).all() and np.isnan(ta[-1])


@pytest.mark.slow
def test_bundle_delay_velocity_scales_with_sqrt_conductivity(oracle_lib):
    """Cable theory: conduction velocity grows as the square root of the
    axial conductivity, so a bundle at a quarter of its conductivity (the
    paper's proportional bundle-branch delay) conducts at half the speed
    (10 % band for the discrete chain)."""
    cvs = []
    for scale in (1.0, 0.25):
        w = chain_workload(241, 0.1, stim_nodes=list(range(5)), stim_amp=-100.0, stim_dur=1.0)
        w.purkinje.edge_scale = np.full(240, scale)
        s = oracle_lib.Sim(w)
        s.step(900)
        ta = s.purkinje_activation()
        x = w.purkinje.xyz[:, 0]
        i0, i1 = np.argmin(abs(x - 8.0)), np.argmin(abs(x - 16.0))
        assert np.isfinite(ta[[i0, i1]]).all()
        cvs.append((x[i1] - x[i0]) / (ta[i1] - ta[i0]))
    assert cvs[1] / cvs[0] == pytest.approx(0.5, rel=0.10)
