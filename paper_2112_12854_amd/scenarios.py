"""Pathology and pacing presets (Sec. 6) as edits of a workload.

The paper models
- a bundle-branch delay by lowering the conductivity of the fast-conduction
  bundles in proportion to its severity, and a complete bundle-branch block
  by a null conductivity;
- an atrioventricular block by a null conductivity of the AV node, so that
  the sinus beat never reaches the His bundle;
- an implanted pacing lead as an extra stimulus current on the myocardium
  around the lead's tip, with leads at the ventricular apex, the septum, the
  left-ventricular wall, the atrial septum and wall, and the right atrial
  appendage.

Each function returns a modified copy and leaves its argument alone.  Like
the generators in `meshgen`, these only define inputs (conductivity
multipliers, stimulus cell sets); the simulation itself runs through the
library (`ep.Sim`, or `ep.Server` for sweeps: `sweep_requests`).
"""
from __future__ import annotations

import copy

import numpy as np

from . import meshgen as M

SIDES = {"left": 0, "right": 1}


def _copy(w: M.Workload) -> M.Workload:
    c = copy.copy(w)
    c.stimuli = list(w.stimuli)
    c.landmarks = dict(w.landmarks)
    if w.purkinje is not None:
        c.purkinje = copy.copy(w.purkinje)
    return c


def bundle_branch_block(w: M.Workload, side: str, severity: float = 1.0,
                        generations: int = 1) -> M.Workload:
    """Bundle-branch delay (0 < severity < 1) or block (severity 1) of the
    left or right branch of a heart's Purkinje tree: the segments of that
    side in the first `generations` branching generations (1 = the bundle
    branch itself) conduct with (1 - severity) times their conductivity."""
    if side not in SIDES:
        raise ValueError("side must be 'left' or 'right'")
    if not 0.0 <= severity <= 1.0:
        raise ValueError("severity must lie in [0, 1]")
    pk = w.purkinje
    if pk is None or pk.edge_side is None or pk.edge_depth is None:
        raise ValueError("needs a Purkinje tree with branch labels (meshgen.heart)")
    c = _copy(w)
    s = np.ones(pk.edges.shape[0]) if pk.edge_scale is None else np.array(pk.edge_scale, float)
    hit = (pk.edge_side == SIDES[side]) & (pk.edge_depth < generations)
    s[hit] *= 1.0 - severity
    c.purkinje.edge_scale = s
    c.name = f"{w.name}-{side[0]}bbb{severity:g}"
    return c


def av_block(w: M.Workload) -> M.Workload:
    """Complete AV block: the His bundle receives no beat from the atria.
    In the synthetic heart the atrio-ventricular conduction is the timed
    drive of the His root (a graph stimulus), so the block removes every
    stimulus on the graph."""
    c = _copy(w)
    c.stimuli = [st for st in w.stimuli if st.domain != 1]
    c.name = f"{w.name}-avb"
    return c


def lead_cells(w: M.Workload, point, radius: float = 1.5) -> np.ndarray:
    """Tissue cells of a lead tip at `point`: the tets whose centroid lies
    within `radius` mm, else the 20 nearest."""
    cen = w.xyz[w.tets].mean(axis=1)
    d = np.linalg.norm(cen - np.asarray(point, float), axis=1)
    ids = np.nonzero(d <= radius)[0]
    if ids.size == 0:
        ids = np.sort(np.argsort(d, kind="stable")[:20])
    return ids.astype(np.int32)


def pacing_lead(w: M.Workload, site, t0: float = 0.0, period: float = 0.0, count: int = 1,
                amp: float = -52.0, dur: float = 2.0, radius: float = 1.5) -> M.Workload:
    """Implanted lead: a stimulus on the myocardium around the tip, at a
    named landmark of the workload (e.g. "rv_apex", "septum", "lv_lateral",
    "ra_appendage") or at a point; period > 0 paces `count` beats."""
    point = w.landmarks[site] if isinstance(site, str) else np.asarray(site, float)
    c = _copy(w)
    c.stimuli.append(M.Stimulus(ids=lead_cells(w, point, radius), t0=t0, dur=dur, amp=amp,
                                period=period, count=count))
    c.name = f"{w.name}-lead-{site if isinstance(site, str) else 'pt'}"
    return c


def tissue_block(w: M.Workload, center, radius: float, severity: float = 1.0) -> M.Workload:
    """Conduction slowing or block in the myocardium (a scar-like ball): the
    cells whose centroid lies within `radius` of `center` conduct with
    (1 - severity) times their conductivity."""
    if not 0.0 <= severity <= 1.0:
        raise ValueError("severity must lie in [0, 1]")
    c = _copy(w)
    sc = np.ones(w.n_tets) if w.scale is None else np.array(w.scale, float)
    cen = w.xyz[w.tets].mean(axis=1)
    sc[np.linalg.norm(cen - np.asarray(center, float), axis=1) <= radius] *= 1.0 - severity
    c.scale = sc
    return c


def two_way_junctions(w: M.Workload, on: bool = True) -> M.Workload:
    """Enable the antidromic (muscle to Purkinje) coupling of the junctions,
    which a ventricular lead needs to reach the conduction system."""
    c = _copy(w)
    c.purkinje.two_way = bool(on)
    return c


def ventricular_pacing_with_av_block(w: M.Workload, site: str = "rv_apex", t0: float = 160.0,
                                     period: float = 0.0, count: int = 1) -> M.Workload:
    """The paper's pacing case: AV block, a right-ventricular apex lead
    firing 160 ms after the sinus beat, and two-way junctions so the wave
    enters the Purkinje network antidromically and re-excites the muscle
    through the other junctions."""
    return two_way_junctions(pacing_lead(av_block(w), site, t0=t0, period=period, count=count))


def atrial_appendage_pacing(w: M.Workload, t0: float = 0.0) -> M.Workload:
    """The paper's atrial lead: the right atrial appendage paced instead of
    the sinus node (the sinus stimulus on the atrial tissue is removed)."""
    if "ra_appendage" not in w.landmarks:
        raise ValueError("needs a heart with atria")
    cen = w.xyz[w.tets].mean(axis=1)
    sa = int(np.argmin(np.linalg.norm(cen - w.landmarks["sa_node"], axis=1)))
    c = _copy(w)
    c.stimuli = [st for st in w.stimuli if not (st.domain == 0 and np.any(st.ids == sa))]
    c = pacing_lead(c, "ra_appendage", t0=t0)
    c.name = f"{w.name}-ra-lead"
    return c


def sweep_requests(w: M.Workload, side: str, severities) -> list[M.Workload]:
    """One workload per bundle-branch severity, for submission to the
    server (`ep.Server.submit`) as a batch."""
    return [bundle_branch_block(w, side, float(s)) for s in severities]


# --------------------------------------------- communication nodes (Sec. 3.3)
# The paper spaces the nodes along its 1D bundles varsigma * tau apart:
# internodal conduction speed 2 m/s times 0.5 ms, the largest activation
# delay allowed between consecutive nodes (about 1 mm).
BUNDLE_SPEED_MM_PER_MS = 2.0
NODE_DELAY_MS = 0.5


def communication_nodes(pk: M.Purkinje, spacing: float = BUNDLE_SPEED_MM_PER_MS * NODE_DELAY_MS,
                        root: int = 0) -> np.ndarray:
    """Graph nodes chosen as communication nodes: walking the graph from
    `root`, a node is taken when its path distance from the last taken node
    on its path reaches `spacing`; leaves are always taken."""
    n = pk.xyz.shape[0]
    adj = [[] for _ in range(n)]
    for a, b in pk.edges:
        L = float(np.linalg.norm(pk.xyz[a] - pk.xyz[b]))
        adj[a].append((int(b), L))
        adj[b].append((int(a), L))
    chosen, seen = [], np.zeros(n, bool)
    stack = [(root, 0.0)]
    seen[root] = True
    chosen.append(root)
    while stack:
        i, since = stack.pop()
        kids = [(j, L) for j, L in adj[i] if not seen[j]]
        for j, L in kids:
            seen[j] = True
            d = since + L
            if d >= spacing - 1e-9 or len(adj[j]) == 1:
                chosen.append(j)
                d = 0.0
            stack.append((j, d))
    return np.array(sorted(chosen), np.int32)


def bundle_coupling(w: M.Workload, spacing: float = BUNDLE_SPEED_MM_PER_MS * NODE_DELAY_MS,
                    radius: float = 1.0, delay: float = 0.0, amp: float = -200.0,
                    two_way: bool = False) -> M.Workload:
    """Couple a workload's graph to the tissue through communication nodes
    every `spacing` mm (Sec. 3.3: range R_S = 1 mm onto the atria, 0.1 mm
    onto the Purkinje shell; the bundles fire the atria without delay)."""
    if w.purkinje is None:
        raise ValueError("needs a Purkinje / bundle graph")
    c = _copy(w)
    pk = c.purkinje
    pk.pmj_nodes = communication_nodes(pk, spacing)
    pk.pmj_radius = radius
    pk.delay_ortho = delay
    pk.pmj_amp = amp
    pk.two_way = two_way
    c.name = f"{w.name}-cn{spacing:g}"
    return c
