"""Seeded synthetic workloads for the monodomain step.

This module only *defines inputs*: node coordinates, tetrahedra, fibre
directions, per-cell model labels, stimulus cell sets and sweep parameters.
It holds none of the method's arithmetic (no volumes, normals, weights,
fluxes or ionic currents) so that the CPU oracle and the HIP library can both
be fed from it without sharing any part of the computation.

Units: mm, ms, mV, mS/mm, 1/mm, uF/mm^2, pA/pF (the cell models' current unit).

Geometry recipe (the paper's Cartesian test boxes, Sec. 4, and its
tetrahedral cell-centred FV setting, Sec. 3.2): a box of nx*ny*nz hexahedra of
side h; nodes numbered i-major, id = (i*(ny+1) + j)*(nz+1) + k.  Each hex is
split into five tetrahedra: a central tetrahedron on the four hex corners of
even global parity (i+j+k even) and four corner tetrahedra, each cutting off
one odd-parity corner together with its three edge neighbours.  Because the
central tetrahedron always uses the globally even corners, every square face
is cut along the same diagonal from both sides, so the mesh is conforming.
Tetrahedra are emitted hex by hex (hexes i-major), central one first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Cell-model labels (same values as the ep_model enum of the C-ABI).
TP06_ENDO, TP06_MID, TP06_EPI, CRN, STEWART, PASSIVE = 0, 1, 2, 3, 4, 5

# Parameter set of the paper (Sec. 3.1 and the conductivity table of Sec. 5).
CHI = 140.0          # 1/mm
CM = 0.01            # uF/mm^2
SIGMA_L = 0.17       # mS/mm, along the fibre
SIGMA_T = 0.019      # mS/mm, across the fibre


@dataclass
class Stimulus:
    """A stimulus on a set of cells: amplitude amp (pA/pF, negative depolarises)
    applied from t0 for dur ms, optionally repeated every `period` ms `count`
    times (period 0 = once)."""
    ids: np.ndarray
    t0: float
    dur: float
    amp: float
    period: float = 0.0
    count: int = 1
    domain: int = 0          # 0 tissue, 1 Purkinje graph


@dataclass
class CellJunction:
    """A communication node whose source is a cell (Sec. 3.3: the 2D
    Purkinje shell excites the 3D myocardium through them): the cells of the
    other kind within `radius` of the source's centroid get `amp` for `dur`
    ms, `delay_ortho` ms after the source's upward crossing; with two_way the
    region's mean crossing pulses the source after `delay_anti`."""
    cell: int
    radius: float = 0.1
    delay_ortho: float = 5.0
    delay_anti: float = 3.0
    two_way: bool = False
    amp: float = -200.0
    dur: float = 0.5


@dataclass
class Workload:
    name: str
    xyz: np.ndarray                  # [n_nodes, 3] float64
    tets: np.ndarray                 # [n_tets, 4] int32
    fibre: np.ndarray                # [n_tets, 3] float64, unit vectors
    model: np.ndarray                # [n_tets] uint8
    sigma_l: float = SIGMA_L
    sigma_t: float = SIGMA_T
    scale: np.ndarray | None = None  # [n_tets] conductivity scale or None
    stimuli: list = field(default_factory=list)
    dt: float = 0.02
    n_steps: int = 2500
    chi: float = CHI
    cm: float = CM
    ionic_scale: dict = field(default_factory=dict)  # "GKr","GKs","GCaL","GNa"
    hex_ijk: np.ndarray | None = None  # [n_tets, 3] hex index of each tet
    dims: tuple = ()                   # (nx, ny, nz, h)
    purkinje: object = None            # Purkinje graph (heart workloads)
    bidomain: object = None            # Bidomain parameters, or monodomain
    landmarks: dict = field(default_factory=dict)   # name -> [3] point (mm)
    time_scheme: int = 0               # 0 forward Euler, 1 AB2, 2 AB2 + second-order RL
    cell_junctions: list = field(default_factory=list)   # CellJunction, after the graph's
    medium_substeps: int | None = None  # 2D medium: substeps per step (0: from its bound)

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])


@dataclass
class Bidomain:
    """Bidomain: the workload's sigma_l / sigma_t are the intracellular
    conductivities, these the extracellular ones (Sec. 5 table, from the
    benchmark of Niederer et al.), with the elliptic solver's settings."""
    sigma_el: float = 0.62         # mS/mm along the fibre
    sigma_et: float = 0.24         # mS/mm across
    restart: int = 30
    tol: float = 1e-8              # relative residual of the elliptic solve
    max_iter: int = 2000           # Arnoldi steps per time step at most


def workload_sha256(w: Workload) -> str:
    """Hash of every input of a tissue workload (mesh, fibres, labels,
    conductivities, ionic scales, stimuli, time step and length), so that
    results stored for one input are never compared with another."""
    import hashlib
    hs = hashlib.sha256()

    def arr(a, dt):
        hs.update(np.ascontiguousarray(a, dtype=dt).tobytes())

    arr(w.xyz, np.float64)
    arr(w.tets, np.int32)
    arr(w.fibre, np.float64)
    arr(w.model, np.uint8)
    if w.scale is not None:
        arr(w.scale, np.float64)
    for st in w.stimuli:
        arr(st.ids, np.int32)
        arr([st.t0, st.dur, st.amp, st.period, st.count, st.domain], np.float64)
    arr([w.sigma_l, w.sigma_t, w.dt, w.n_steps, w.chi, w.cm, w.time_scheme], np.float64)
    if getattr(w, "medium_substeps", None) is not None:
        arr([w.medium_substeps], np.float64)
    arr([w.ionic_scale.get(k, 1.0) for k in ("GKr", "GKs", "GCaL", "GNa")], np.float64)
    return hs.hexdigest()


def slab(nx: int, ny: int, nz: int, h: float):
    """Box [0, nx h] x [0, ny h] x [0, nz h] of 5-tet-split hexes.

    Returns (xyz [N_n,3] f64, tets [N_c,4] i32, hex_ijk [N_c,3] i32)."""
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1),
                             np.arange(nz + 1), indexing="ij")
    xyz = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h],
                   axis=1).astype(np.float64)

    def nid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    hi, hj, hk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    hi, hj, hk = hi.ravel(), hj.ravel(), hk.ravel()
    nhex = hi.size
    # corner ids of every hex, indexed by local (a, b, c)
    corner = {}
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                corner[(a, b, c)] = nid(hi + a, hj + b, hk + c)
    hexpar = (hi + hj + hk) & 1
    tets = np.empty((nhex, 5, 4), dtype=np.int64)
    # local even corners are globally even when the hex parity is even;
    # otherwise the local odd corners are the globally even ones.
    even_local = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    odd_local = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]
    for hp in (0, 1):
        sel = hexpar == hp
        cen = even_local if hp == 0 else odd_local
        cut = odd_local if hp == 0 else even_local
        tets[sel, 0, :] = np.stack([corner[q][sel] for q in cen], axis=1)
        for t, (a, b, c) in enumerate(cut):
            nb = [(1 - a, b, c), (a, 1 - b, c), (a, b, 1 - c)]
            tets[sel, 1 + t, 0] = corner[(a, b, c)][sel]
            for m, q in enumerate(nb):
                tets[sel, 1 + t, 1 + m] = corner[q][sel]
    tets = tets.reshape(-1, 4).astype(np.int32)
    hex_ijk = np.repeat(np.stack([hi, hj, hk], axis=1), 5, axis=0).astype(np.int32)
    return xyz, tets, hex_ijk


def sheet(nx: int, ny: int, h: float, curvature_radius: float = 0.0):
    """Triangulated sheet (a 2D medium, Sec. 3.2): the rectangle [0, nx h] x
    [0, ny h] of squares of side h, each split into two triangles along the
    diagonal that alternates with the parity of i + j (nodes numbered
    i-major, id = i (ny+1) + j).  With curvature_radius R > 0 the sheet is
    bent around the x axis onto a cylinder of radius R (y becomes arc
    length).  Cells are returned as [n, 4] rows whose fourth entry is -1, the
    library's mark of a triangle; also returns the square (i, j) of each."""
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    x = (ii * h).ravel().astype(np.float64)
    y = (jj * h).ravel().astype(np.float64)
    if curvature_radius > 0:
        R = curvature_radius
        xyz = np.stack([x, R * np.sin(y / R), R - R * np.cos(y / R)], axis=1)
    else:
        xyz = np.stack([x, y, np.zeros_like(x)], axis=1)

    def nid(i, j):
        return i * (ny + 1) + j

    si, sj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    si, sj = si.ravel(), sj.ravel()
    a, b, c, d = nid(si, sj), nid(si + 1, sj), nid(si + 1, sj + 1), nid(si, sj + 1)
    even = ((si + sj) % 2) == 0
    t1 = np.where(even[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t2 = np.where(even[:, None], np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tri = np.stack([t1, t2], axis=1).reshape(-1, 3)
    cells = np.concatenate([tri, -np.ones((tri.shape[0], 1), np.int64)], axis=1).astype(np.int32)
    sq = np.repeat(np.stack([si, sj], axis=1), 2, axis=0)
    return xyz, cells, sq


def sheet_workload(nx: int = 40, ny: int = 20, h: float = 0.25, model: int = TP06_ENDO,
                   sigma_l: float = SIGMA_L, sigma_t: float = SIGMA_T,
                   curvature_radius: float = 0.0, dt: float = 0.02, n_steps: int = 1000,
                   fibre_angle_deg: float = 0.0) -> Workload:
    """A 2D sheet of one cell model, fibres at fibre_angle_deg from the x
    axis (in the sheet), stimulated for 1 ms at -52 pA/pF on the squares
    with x < 1 mm."""
    xyz, cells, sq = sheet(nx, ny, h, curvature_radius)
    n = cells.shape[0]
    a = np.deg2rad(fibre_angle_deg)
    if curvature_radius > 0:
        # in-sheet direction at arc length y: cos a x + sin a (tangent of the circle)
        yc = (sq[:, 1] + 0.5) * h / curvature_radius
        fib = np.stack([np.full(n, np.cos(a)), np.sin(a) * np.cos(yc), np.sin(a) * np.sin(yc)], 1)
    else:
        fib = np.tile([np.cos(a), np.sin(a), 0.0], (n, 1))
    nstim = max(1, int(round(1.0 / h)))
    ids = np.nonzero(sq[:, 0] < nstim)[0].astype(np.int32)
    return Workload(f"sheet-{nx}x{ny}-h{h}" + (f"-R{curvature_radius}" if curvature_radius else ""),
                    xyz, cells, fib, np.full(n, model, np.uint8), sigma_l=sigma_l,
                    sigma_t=sigma_t, stimuli=[Stimulus(ids=ids, t0=0.0, dur=1.0, amp=-52.0)],
                    dt=dt, n_steps=n_steps, hex_ijk=None, dims=(nx, ny, 0, h))


def mixed_workload(w3: Workload, w2: Workload) -> Workload:
    """One workload holding a tetrahedral medium and a separate triangulated
    one (disjoint node sets; the sheet's nodes and cells follow the tets')."""
    nn = w3.n_nodes
    cells2 = w2.tets.copy()
    cells2[:, :3] += nn
    stims = list(w3.stimuli) + [Stimulus(ids=st.ids + w3.n_tets, t0=st.t0, dur=st.dur, amp=st.amp,
                                         period=st.period, count=st.count)
                                for st in w2.stimuli]
    sc = None
    if w3.scale is not None or w2.scale is not None:
        sc = np.concatenate([np.ones(w3.n_tets) if w3.scale is None else w3.scale,
                             np.ones(w2.n_tets) if w2.scale is None else w2.scale])
    return Workload(f"{w3.name}+{w2.name}", np.concatenate([w3.xyz, w2.xyz]),
                    np.concatenate([w3.tets, cells2]).astype(np.int32),
                    np.concatenate([w3.fibre, w2.fibre]), np.concatenate([w3.model, w2.model]),
                    sigma_l=w3.sigma_l, sigma_t=w3.sigma_t, scale=sc, stimuli=stims, dt=w3.dt,
                    n_steps=w3.n_steps)


def shell_on_slab(nx: int = 16, ny: int = 8, nz: int = 2, h: float = 0.5, gap: float = 0.05,
                  cn_spacing: float = 1.0, radius: float = 0.6, drive: str = "sheet",
                  two_way: bool = False, amp: float = -200.0, sheet_scale: float = 10.0,
                  dt: float = 0.02, n_steps: int = 750) -> Workload:
    """A 2D Stewart sheet (the Purkinje shell, Sec. 2) lying `gap` mm above
    a TP06 slab, coupled to it by communication nodes: the sheet triangles
    nearest to a square grid of spacing cn_spacing (the paper spaces its
    nodes about 1 mm apart) are sources of junctions onto the tets within
    `radius`.  The sheet conducts with sheet_scale times the tissue's
    conductivities.  drive="sheet": -100 pA/pF for 1 ms on the sheet's
    triangles with x < 1 mm; drive="slab": -52 pA/pF for 1 ms on the slab's
    cells with x < 1 mm (with two_way the slab then excites the sheet)."""
    xyz3, tets, hijk = slab(nx, ny, nz, h)
    n3 = tets.shape[0]
    w3 = Workload("slab", xyz3, tets, _uniform_fibre(n3), np.full(n3, TP06_ENDO, np.uint8),
                  dt=dt, n_steps=n_steps, hex_ijk=hijk, dims=(nx, ny, nz, h))
    w2 = sheet_workload(nx, ny, h, model=STEWART, dt=dt, n_steps=n_steps)
    w2.xyz = w2.xyz + np.array([0.0, 0.0, nz * h + gap])
    w2.scale = np.full(w2.n_tets, sheet_scale)
    sheet_stim = w2.stimuli[0]
    w2.stimuli = []
    w = mixed_workload(w3, w2)
    w.name = f"shell-on-slab-{nx}x{ny}x{nz}-h{h}"
    w.hex_ijk, w.dims = None, (nx, ny, nz, h)
    cen2 = w2.xyz[w2.tets[:, :3]].mean(axis=1)
    gx = np.arange(0.5 * cn_spacing, nx * h, cn_spacing)
    gy = np.arange(0.5 * cn_spacing, ny * h, cn_spacing)
    src = []
    for x in gx:
        for y in gy:
            src.append(int(np.argmin((cen2[:, 0] - x) ** 2 + (cen2[:, 1] - y) ** 2)))
    w.cell_junctions = [CellJunction(cell=n3 + c, radius=radius, two_way=two_way, amp=amp)
                        for c in sorted(set(src))]
    if drive == "sheet":
        w.stimuli.append(Stimulus(ids=(sheet_stim.ids + n3).astype(np.int32), t0=0.0, dur=1.0,
                                  amp=-100.0))
    else:
        w.stimuli.append(Stimulus(ids=hex_box_ids(hijk, (0, None, None), (int(round(1.0 / h)), None, None)),
                                  t0=0.0, dur=1.0, amp=-52.0))
    return w


def slab6(nx: int, ny: int, nz: int, h: float):
    """Box of hexes split into six tets each around the main diagonal
    (0,0,0)-(1,1,1) (Kuhn's split: the tets along the six monotone corner
    paths; every hex is split alike, so the mesh is conforming and
    translation invariant).  Returns like slab()."""
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1),
                             np.arange(nz + 1), indexing="ij")
    xyz = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h],
                   axis=1).astype(np.float64)

    def nid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k

    hi, hj, hk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    hi, hj, hk = hi.ravel(), hj.ravel(), hk.ravel()
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = np.empty((hi.size, 6, 4), np.int64)
    for t, p in enumerate(perms):
        step = np.zeros(3, int)
        tets[:, t, 0] = nid(hi, hj, hk)
        for m in range(3):
            step[p[m]] += 1
            tets[:, t, m + 1] = nid(hi + step[0], hj + step[1], hk + step[2])
    tets = tets.reshape(-1, 4).astype(np.int32)
    hex_ijk = np.repeat(np.stack([hi, hj, hk], axis=1), 6, axis=0).astype(np.int32)
    return xyz, tets, hex_ijk


def hex_box_ids(hex_ijk: np.ndarray, lo, hi) -> np.ndarray:
    """Ids of the tets whose hex index lies in [lo, hi) per axis (None = open)."""
    sel = np.ones(hex_ijk.shape[0], dtype=bool)
    for ax in range(3):
        if lo[ax] is not None:
            sel &= hex_ijk[:, ax] >= lo[ax]
        if hi[ax] is not None:
            sel &= hex_ijk[:, ax] < hi[ax]
    return np.nonzero(sel)[0].astype(np.int32)


def _uniform_fibre(n: int) -> np.ndarray:
    f = np.zeros((n, 3), dtype=np.float64)
    f[:, 0] = 1.0
    return f


def config1(n_steps: int = 2500, nx: int = 20, ny: int = 20, nz: int = 4,
            h: float = 0.5) -> Workload:
    """10 x 10 x 2 mm ventricular slab at h = 0.5 mm (8,000 tets), all
    TP06-endocardial cells in the standard initial state, fibres along x,
    no-flux boundaries, -52 pA/pF for 1 ms on the cells of the hexes with
    x < 1 mm (800 tets), dt = 0.02 ms, 2,500 steps (50 ms)."""
    xyz, tets, hijk = slab(nx, ny, nz, h)
    n = tets.shape[0]
    nstim = int(round(1.0 / h))
    stim = Stimulus(ids=hex_box_ids(hijk, (0, None, None), (nstim, None, None)),
                    t0=0.0, dur=1.0, amp=-52.0)
    return Workload("slab-10x10x2mm-h0.5-tp06endo", xyz, tets, _uniform_fibre(n),
                    np.full(n, TP06_ENDO, np.uint8), stimuli=[stim], dt=0.02,
                    n_steps=n_steps, hex_ijk=hijk, dims=(nx, ny, nz, h))


def transmural_fibres_layers(hex_ijk: np.ndarray, nz: int, seed: int,
                             jitter_deg: float = 5.0):
    """Fibre field and TP06 layer labels of the rotating-fibre slab.

    Depth d of a tet = (k + 0.5) / nz from the z = 0 (endocardial) face, with
    k its hex layer.  Fibre angle alpha(d) = -60 deg + 120 deg * d plus a
    per-cell Gaussian jitter (sigma = jitter_deg, numpy PCG64 stream of
    `seed`, one draw per cell in cell order); f = (cos a, sin a, 0).
    Layers: d < 0.3 endo, 0.3 <= d < 0.7 mid, d >= 0.7 epi."""
    n = hex_ijk.shape[0]
    d = (hex_ijk[:, 2].astype(np.float64) + 0.5) / nz
    rng = np.random.default_rng(seed)
    jit = rng.normal(0.0, jitter_deg, n)
    a = np.deg2rad(-60.0 + 120.0 * d + jit)
    fibre = np.stack([np.cos(a), np.sin(a), np.zeros(n)], axis=1)
    model = np.where(d < 0.3, TP06_ENDO, np.where(d < 0.7, TP06_MID, TP06_EPI))
    return fibre, model.astype(np.uint8)


def config2(n_steps: int = 20000, nx: int = 160, ny: int = 160, nz: int = 40,
            h: float = 0.25, seed: int = 2) -> Workload:
    """40 x 40 x 10 mm slab at h = 0.25 mm (5.12M tets), fibres rotating
    transmurally -60 -> +60 deg with 5 deg Gaussian jitter, TP06 endo/mid/epi
    layers at 30/40/30 % depth, corner stimulus (hexes inside [0, 1.5]^3 mm,
    1,080 tets) of -52 pA/pF for 1 ms, dt = 0.02 ms, 20,000 steps (400 ms)."""
    xyz, tets, hijk = slab(nx, ny, nz, h)
    fibre, model = transmural_fibres_layers(hijk, nz, seed)
    m = int(round(1.5 / h))
    stim = Stimulus(ids=hex_box_ids(hijk, (0, 0, 0), (m, m, m)), t0=0.0,
                    dur=1.0, amp=-52.0)
    return Workload(f"slab-40x40x10mm-h{h}-tp06-layers-rotfibre", xyz, tets,
                    fibre, model, stimuli=[stim], dt=0.02, n_steps=n_steps,
                    hex_ijk=hijk, dims=(nx, ny, nz, h))


def scaled_config2(nx: int, ny: int, nz: int, h: float = 0.25, seed: int = 2,
                   n_steps: int = 100) -> Workload:
    """A config-2-style slab of another size (same fibre, layer and corner
    stimulus recipe), for parity runs the oracle finishes in seconds."""
    return config2(n_steps=n_steps, nx=nx, ny=ny, nz=nz, h=h, seed=seed)


def niederer_box(h: float, dt: float, n_steps: int, lx=20.0, ly=7.0, lz=3.0,
                 stim_side: float = 1.5, split: int = 5) -> Workload:
    """The paper's convergence box (Sec. 4): 20 x 7 x 3 mm, fibres along the
    long (x) axis, TP06 (endocardial parameters), stimulus on a corner cube of
    side 1.5 mm at the origin (-52 pA/pF for 2 ms); hexes split into 5 or 6
    tets."""
    nx, ny, nz = int(round(lx / h)), int(round(ly / h)), int(round(lz / h))
    xyz, tets, hijk = (slab if split == 5 else slab6)(nx, ny, nz, h)
    n = tets.shape[0]
    m = int(round(stim_side / h))
    stim = Stimulus(ids=hex_box_ids(hijk, (0, 0, 0), (m, m, m)), t0=0.0,
                    dur=2.0, amp=-52.0)
    return Workload(f"box-20x7x3mm-h{h}", xyz, tets, _uniform_fibre(n),
                    np.full(n, TP06_ENDO, np.uint8), stimuli=[stim], dt=dt,
                    n_steps=n_steps, hex_ijk=hijk, dims=(nx, ny, nz, h))


def cable(n_hex: int, h: float, model: int, sigma: float, dt: float,
          n_steps: int, width: int = 1) -> Workload:
    """A thin bar of n_hex x width x width hexes with isotropic conductivity
    sigma, stimulated on its first 1 mm, for conduction-velocity checks."""
    xyz, tets, hijk = slab(n_hex, width, width, h)
    n = tets.shape[0]
    m = max(1, int(round(1.0 / h)))
    stim = Stimulus(ids=hex_box_ids(hijk, (0, None, None), (m, None, None)),
                    t0=0.0, dur=2.0, amp=-52.0 if model != CRN else -40.0)
    return Workload(f"cable-{model}", xyz, tets, _uniform_fibre(n),
                    np.full(n, model, np.uint8), sigma_l=sigma, sigma_t=sigma,
                    stimuli=[stim], dt=dt, n_steps=n_steps, hex_ijk=hijk,
                    dims=(n_hex, width, width, h))


# ---------------------------------------------------------------- sweeps --

def uq_instances(n: int = 1024, seed: int = 5, h: float = 0.5,
                 nx_range=(20, 80), ny_range=(20, 40), nz: int = 4):
    """UQ batch recipe: n slabs with nx ~ U{20..80}, ny ~ U{20..40}, nz = 4 at
    h = 0.5 mm (8k-64k tets), per-instance G_Kr, G_Ks, G_CaL, G_Na scales
    drawn independently from U[0.7, 1.3].  Returns a list of dicts with
    nx, ny, nz, h and the four scales (the meshes are built on demand)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        sc = rng.uniform(0.7, 1.3, 4)
        out.append(dict(nx=nx, ny=ny, nz=nz, h=h, GKr=float(sc[0]),
                        GKs=float(sc[1]), GCaL=float(sc[2]), GNa=float(sc[3])))
    return out


def uq_workload(spec: dict, n_steps: int, dt: float = 0.02) -> Workload:
    w = config1(n_steps=n_steps, nx=spec["nx"], ny=spec["ny"], nz=spec["nz"],
                h=spec["h"])
    w.dt = dt
    w.name = f"uq-{spec['nx']}x{spec['ny']}x{spec['nz']}"
    w.ionic_scale = {k: spec[k] for k in ("GKr", "GKs", "GCaL", "GNa")}
    return w


def serving_requests(n: int = 256, seed: int = 4, h: float = 0.5,
                     n_lo: float = 1e4, n_hi: float = 1e6, nz: int = 4):
    """Serving recipe: n slab requests, target tet count log-uniform in
    [n_lo, n_hi], nx = ny = round(sqrt(N / 20)) at nz = 4, conductivity scale
    U[0.5, 2], stimulus on the cells within 1 mm of one of the six faces
    (uniform), -52 pA/pF for 1 ms."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nt = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
        side = max(2, int(round(math.sqrt(nt / (5 * nz)))))
        out.append(dict(nx=side, ny=side, nz=nz, h=h,
                        sigma_scale=float(rng.uniform(0.5, 2.0)),
                        face=int(rng.integers(0, 6))))
    return out


def serving_workload(spec: dict, n_steps: int, dt: float = 0.02) -> Workload:
    nx, ny, nz, h = spec["nx"], spec["ny"], spec["nz"], spec["h"]
    xyz, tets, hijk = slab(nx, ny, nz, h)
    n = tets.shape[0]
    m = max(1, int(round(1.0 / h)))
    dims = (nx, ny, nz)
    ax, side = divmod(spec["face"], 2)
    lo, hi = [None] * 3, [None] * 3
    if side == 0:
        hi[ax] = min(m, dims[ax])
    else:
        lo[ax] = max(0, dims[ax] - m)
    stim = Stimulus(ids=hex_box_ids(hijk, lo, hi), t0=0.0, dur=1.0, amp=-52.0)
    return Workload(f"req-{nx}x{ny}x{nz}", xyz, tets, _uniform_fibre(n),
                    np.full(n, TP06_ENDO, np.uint8),
                    scale=np.full(n, spec["sigma_scale"]), stimuli=[stim],
                    dt=dt, n_steps=n_steps, hex_ijk=hijk, dims=(nx, ny, nz, h))


# ------------------------------------------------------ three-media heart --

@dataclass
class Purkinje:
    """A 1D Purkinje graph: node coordinates [n,3], edges [m,2], terminal
    (junction) nodes, conductivity sigma (mS/mm), the cell model, and
    optionally a conductivity multiplier per edge (bundle-branch delay or
    block) and per-edge labels of the generator (branch side and depth)."""
    xyz: np.ndarray
    edges: np.ndarray
    pmj_nodes: np.ndarray
    sigma: float = 3.95            # mS/mm, Sec. 5 table (4 m/s)
    model: int = STEWART
    n_sub: int = 0                 # substeps per tissue step (0 = from stability)
    pmj_radius: float = 0.1        # mm, Sec. 3.3
    delay_ortho: float = 5.0       # ms, Sec. 3.3
    delay_anti: float = 3.0        # ms (antidromic, pathologic two-way coupling)
    two_way: bool = False
    pmj_amp: float = -200.0        # pA/pF
    pmj_dur: float = 0.5           # ms, Sec. 3.3 (S_d of communication nodes)
    edge_scale: np.ndarray | None = None   # [m] conductivity multipliers >= 0
    edge_side: np.ndarray | None = None    # [m] 0 left, 1 right bundle (heart tree)
    edge_depth: np.ndarray | None = None   # [m] branching generation (0 = bundle)


def _ellipsoid_depth(p, a_in, c_in, a_out, c_out, iters=30):
    """Normalised wall depth s in [0, 1] (0 inner surface, 1 outer) of points
    p [n,3] between two confocal-like prolate ellipsoids (axis z): the s with
    (x^2+y^2)/a(s)^2 + z^2/c(s)^2 = 1, a(s), c(s) linear in s (bisection)."""
    r2 = p[:, 0] ** 2 + p[:, 1] ** 2
    z2 = p[:, 2] ** 2
    lo = np.full(p.shape[0], -1.0)
    hi = np.full(p.shape[0], 2.0)
    for _ in range(iters):
        s = 0.5 * (lo + hi)
        a = a_in + s * (a_out - a_in)
        c = c_in + s * (c_out - c_in)
        f = r2 / a ** 2 + z2 / c ** 2 - 1.0
        lo = np.where(f > 0, s, lo)
        hi = np.where(f > 0, hi, s)
    return 0.5 * (lo + hi)


def heart(h: float = 0.5, seed: int = 3, scale: float = 1.0, purkinje_nodes: int = 60000,
          n_pmj: int = 2000, seg: float = 0.1, with_atria: bool = True,
          branch_mm: tuple = (1.0, 4.0)):
    """Synthetic three-media heart (stand-in for the paper's anatomical
    meshes, Sec. 2): a biventricle of two truncated prolate-ellipsoidal
    shells (LV, and an RV shell fused to it through the septum) with TP06
    layers and transmurally rotating fibres, an electrically insulated
    atrial cap shell above the base (Courtemanche, conductivity x 1.05, Sec. 5
    table), and a seeded fractal Purkinje tree grown on the endocardium with
    Stewart cells whose leaves outside the septum are the junctions.
    Voxelised on the 5-tet lattice at spacing h; `scale` shrinks every
    length (scale 1: ~10M ventricular + ~2M atrial tets at h = 0.5)."""
    L = scale
    # LV: inner (a, c) = (22, 70), outer (32, 80) mm; RV shifted +x, thinner
    lv = (22 * L, 70 * L, 32 * L, 80 * L)
    rv_off = np.array([26 * L, 0.0, -4 * L])
    rv = (28 * L, 62 * L, 33 * L, 66 * L)
    z_base = 0.0
    at_gap, at_thick = 4 * L, 3 * L
    at_a, at_c = 30 * L, 22 * L
    lo = np.array([-33 * L, -34 * L, -82 * L])
    hi = np.array([60 * L, 34 * L, (at_gap + at_c + at_thick + 1) * L if with_atria else 1.0])
    n = np.ceil((hi - lo) / h).astype(int)
    ii, jj, kk = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    cen = lo + (np.stack([ii, jj, kk], axis=-1).reshape(-1, 3) + 0.5) * h

    def shell(p, a_i, c_i, a_o, c_o):
        r2 = p[:, 0] ** 2 + p[:, 1] ** 2
        outer = r2 / a_o ** 2 + p[:, 2] ** 2 / c_o ** 2 <= 1.0
        inner = r2 / a_i ** 2 + p[:, 2] ** 2 / c_i ** 2 <= 1.0
        return outer & ~inner, inner

    below = cen[:, 2] < z_base
    lv_wall, lv_cav = shell(cen, *lv)
    rv_wall, rv_cav = shell(cen - rv_off, *rv)
    vent = below & ((lv_wall | rv_wall) & ~lv_cav & ~rv_cav)
    region = np.zeros(cen.shape[0], np.int8)
    region[vent] = 1
    if with_atria:
        pa = cen - np.array([8 * L, 0.0, at_gap])
        r2 = pa[:, 0] ** 2 + pa[:, 1] ** 2
        o = r2 / (at_a + at_thick) ** 2 + pa[:, 2] ** 2 / (at_c + at_thick) ** 2 <= 1
        i_ = r2 / at_a ** 2 + pa[:, 2] ** 2 / at_c ** 2 <= 1
        atria = o & ~i_ & (pa[:, 2] >= 0)
        region[atria & ~vent] = 2
    keep = np.nonzero(region > 0)[0]
    hx = np.stack(np.unravel_index(keep, tuple(n)), axis=1)
    # 5-tet split of the kept hexes on the global lattice (same rule as slab())
    ny1, nz1 = n[1] + 1, n[2] + 1

    def nid(a):
        return (a[:, 0] * ny1 + a[:, 1]) * nz1 + a[:, 2]

    even_local = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    odd_local = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]
    par = hx.sum(axis=1) & 1
    tets = np.empty((keep.size, 5, 4), np.int64)
    for hp in (0, 1):
        sel = par == hp
        base = hx[sel]
        cen_c = even_local if hp == 0 else odd_local
        cut = odd_local if hp == 0 else even_local
        tets[sel, 0, :] = np.stack([nid(base + np.array(q)) for q in cen_c], axis=1)
        for t, q in enumerate(cut):
            a, b, c = q
            tets[sel, 1 + t, 0] = nid(base + np.array(q))
            for m, r in enumerate([(1 - a, b, c), (a, 1 - b, c), (a, b, 1 - c)]):
                tets[sel, 1 + t, 1 + m] = nid(base + np.array(r))
    tets = tets.reshape(-1, 4)
    used, inv = np.unique(tets, return_inverse=True)
    tets = inv.reshape(-1, 4).astype(np.int32)
    gi = np.stack(np.unravel_index(used, (n[0] + 1, n[1] + 1, n[2] + 1)), axis=1)
    xyz = lo + gi * h
    reg = np.repeat(region[keep], 5)
    hcen = np.repeat(cen[keep], 5, axis=0)
    nt = tets.shape[0]
    # depth, layers and fibres of the ventricles (LV depth; RV free wall by its own shell)
    d_lv = _ellipsoid_depth(hcen, *lv)
    d_rv = _ellipsoid_depth(hcen - rv_off, *rv)
    in_rv = (hcen[:, 0] - rv_off[0]) ** 2 / rv[2] ** 2 + hcen[:, 1] ** 2 / rv[2] ** 2 + \
        (hcen[:, 2] - rv_off[2]) ** 2 / rv[3] ** 2 <= 1.0
    in_lv_wall = (hcen[:, 0] ** 2 + hcen[:, 1] ** 2) / lv[2] ** 2 + hcen[:, 2] ** 2 / lv[3] ** 2 <= 1.0
    d = np.where(in_lv_wall, d_lv, d_rv)
    d = np.clip(d, 0.0, 1.0)
    model = np.where(d < 0.3, TP06_ENDO, np.where(d < 0.7, TP06_MID, TP06_EPI)).astype(np.uint8)
    rng = np.random.default_rng(seed)
    alpha = np.deg2rad(-60.0 + 120.0 * d + rng.normal(0.0, 5.0, nt))
    # circumferential and meridional unit vectors of the local ellipsoid
    q = np.where(in_rv[:, None] & ~in_lv_wall[:, None], hcen - rv_off, hcen)
    rr = np.maximum(np.hypot(q[:, 0], q[:, 1]), 1e-9)
    e_t = np.stack([-q[:, 1] / rr, q[:, 0] / rr, np.zeros(nt)], axis=1)
    e_l = np.stack([q[:, 0] / rr * 0.3, q[:, 1] / rr * 0.3, np.ones(nt)], axis=1)
    e_l -= (e_l * e_t).sum(axis=1, keepdims=True) * e_t
    e_l /= np.linalg.norm(e_l, axis=1, keepdims=True)
    fibre = np.cos(alpha)[:, None] * e_t + np.sin(alpha)[:, None] * e_l
    scale_arr = np.ones(nt)
    atr = reg == 2
    if atr.any():
        model[atr] = CRN
        fibre[atr] = e_t[atr]                 # circumferential around the cap
        scale_arr[atr] = 1.05
    fibre /= np.linalg.norm(fibre, axis=1, keepdims=True)
    stimuli = []
    if atr.any():
        # sino-atrial-like ball of 1.5 mm on the cap at t = 0
        top = hcen[atr][np.argmax(hcen[atr][:, 0])]
        ids = np.nonzero(atr & (np.linalg.norm(hcen - top, axis=1) < 1.5 * max(L, h)))[0]
        stimuli.append(Stimulus(ids=ids.astype(np.int32), t0=0.0, dur=2.0, amp=-40.0))
    w = Workload(f"heart-h{h}-s{scale}", xyz, tets, fibre, model, sigma_l=SIGMA_L,
                 sigma_t=SIGMA_T, scale=scale_arr, stimuli=stimuli, dt=0.01,
                 n_steps=80000, hex_ijk=None, dims=())
    pk = purkinje_tree(lv, rv, rv_off, n_nodes=purkinje_nodes, n_pmj=n_pmj, seg=seg, branch_mm=branch_mm,
                       seed=seed, z_base=z_base)
    w.purkinje = pk
    # the His-bundle root is stimulated at 130 ms (AV conduction, Sec. 1); a
    # pulse into one graph node cannot charge the cable around it, so the
    # graph nodes within 0.5 mm of the root receive it
    root = np.nonzero(np.linalg.norm(pk.xyz - pk.xyz[0], axis=1) <= 0.5)[0].astype(np.int32)
    w.stimuli.append(Stimulus(ids=root, t0=130.0, dur=2.0, amp=-100.0, domain=1))
    # pacing-lead sites of Sec. 6 (mid-wall points of this geometry) and the
    # His root
    w.landmarks = {
        "his": pk.xyz[0].copy(),
        "rv_apex": np.array([rv_off[0], 0.0, rv_off[2] - 0.5 * (rv[1] + rv[3])]),
        "lv_apex": np.array([0.0, 0.0, -0.5 * (lv[1] + lv[3])]),
        "lv_lateral": np.array([-0.5 * (lv[0] + lv[2]), 0.0, -0.4 * lv[1]]),
    }
    if atr.any():
        w.landmarks["sa_node"] = top.copy()
        w.landmarks["ra_appendage"] = np.array([8 * L - (at_a + 0.5 * at_thick), 0.0,
                                                at_gap + 0.2 * at_c])
    return w


def config3() -> Workload:
    """The three-media heart at full size: ~9.6M TP06 + ~2M CRN tets at
    h = 0.375 mm, a 60,000-node Stewart tree at 0.1 mm whose branches of
    0.6-2.4 mm end in 2,000 junctions, dt = 0.01 ms."""
    return heart(h=0.375, scale=1.0, purkinje_nodes=60000, n_pmj=2000, branch_mm=(0.6, 2.4))


def purkinje_tree(lv, rv, rv_off, n_nodes=60000, n_pmj=2000, seg=0.1, seed=3, z_base=0.0,
                  branch_mm=(1.0, 4.0)):
    """Seeded fractal tree on the LV and RV endocardium: from a root near the
    base of the septum, branches of random length (branch_mm, 1-4 mm by
    default, x4 for the two bundle branches and their first split; segments of
    `seg` mm) split into two at +-20..50 deg, each point projected back onto
    the endocardial ellipsoid, until n_nodes nodes exist.  Leaves become the
    junctions, except those within 4 mm of the septal plane (the paper places
    none in the septum); at most n_pmj are kept, evenly subsampled."""
    rng = np.random.default_rng(seed)
    a_i, c_i = lv[0], lv[1]

    def project(p, side):
        if side == 0:
            q = p.copy()
            a, c = a_i * 1.01, c_i * 1.01
        else:
            q = p - rv_off
            a, c = rv[0] * 1.01, rv[1] * 1.01
        s = np.sqrt((q[0] ** 2 + q[1] ** 2) / a ** 2 + q[2] ** 2 / c ** 2)
        q = q / s
        q[2] = min(q[2], z_base - 1.0)
        return q if side == 0 else q + rv_off

    pts = [np.array([a_i * 0.9, 0.0, z_base - 2.0])]
    side_of = [0]
    edges = []
    e_side, e_depth = [], []
    leaves = []
    # two bundle branches, one per ventricle
    stack = []
    for side, direc in ((0, np.array([0.0, 0.3, -1.0])), (1, np.array([0.3, -0.3, -1.0]))):
        stack.append((0, side, direc / np.linalg.norm(direc), 0))
    while stack and len(pts) < n_nodes:
        start, side, direc, depth = stack.pop(0)
        length = rng.uniform(*branch_mm) * (4.0 if depth < 2 else 1.0)
        nseg = max(2, int(length / seg))
        prev = start
        for _ in range(nseg):
            if len(pts) >= n_nodes:
                break
            p = project(pts[prev] + seg * direc, side)
            step = p - pts[prev]
            nrm = np.linalg.norm(step)
            if nrm < 0.2 * seg:
                break
            direc = step / nrm
            p = pts[prev] + seg * direc       # every segment is exactly `seg` long
            pts.append(p)
            side_of.append(side)
            edges.append((prev, len(pts) - 1))
            e_side.append(side)
            e_depth.append(depth)
            prev = len(pts) - 1
        if len(pts) >= n_nodes or depth > 40:
            leaves.append(prev)
            continue
        for sgn in (-1.0, 1.0):
            ang = np.deg2rad(rng.uniform(20, 50)) * sgn
            axis = pts[prev] - (np.zeros(3) if side == 0 else rv_off)
            axis /= np.linalg.norm(axis)
            # rotate direc about the surface normal by ang (Rodrigues)
            nd = (direc * np.cos(ang) + np.cross(axis, direc) * np.sin(ang) +
                  axis * np.dot(axis, direc) * (1 - np.cos(ang)))
            stack.append((prev, side, nd / np.linalg.norm(nd), depth + 1))
    for item in stack:
        leaves.append(item[0])
    xyz = np.array(pts)
    edges = np.array(edges, np.int32).reshape(-1, 2)
    leaves = np.unique(np.array(leaves, np.int64))
    deg = np.bincount(edges.ravel(), minlength=xyz.shape[0])
    leaves = leaves[deg[leaves] == 1]
    septal = np.abs(xyz[leaves, 0] - 0.5 * (a_i + (rv_off[0] - rv[0]))) < 4.0
    leaves = leaves[~septal]
    if leaves.size > n_pmj:
        leaves = leaves[np.linspace(0, leaves.size - 1, n_pmj).astype(int)]
    return Purkinje(xyz=xyz, edges=edges, pmj_nodes=leaves.astype(np.int32),
                    edge_side=np.array(e_side, np.int8), edge_depth=np.array(e_depth, np.int32))


def purkinje_slab(nx: int = 16, ny: int = 8, nz: int = 2, h: float = 0.5, seg: float = 0.1,
                  two_way: bool = False, drive: str = "graph", n_steps: int = 750,
                  dt: float = 0.02, pmj_amp: float | None = None) -> Workload:
    """Slab of TP06-endocardial tissue (fibres along x) with a Y-shaped
    Stewart Purkinje graph lying at mid-depth: a trunk from x = 0.25 mm along
    +x to 40 % of the length, then two straight branches to leaves near the
    far corners (segments of at most `seg` mm).  The two leaves are the
    junctions (radius 0.6 mm, Sec. 3.3 delays and pulse).  drive="graph":
    -100 pA/pF for 1 ms on the graph nodes within 0.5 mm of the root;
    drive="tissue": -52 pA/pF for 1 ms on the cells within 1 mm of the first
    leaf (for the antidromic path with two_way).  The junction pulse is
    -200 pA/pF, or -1000 pA/pF with drive="tissue": a pulse into a single
    graph node must charge the cable around it, whose load is far larger
    than that of a tissue region."""
    xyz, tets, hijk = slab(nx, ny, nz, h)
    n = tets.shape[0]
    lx, ly, zm = nx * h, ny * h, 0.5 * nz * h
    root = np.array([0.25, 0.5 * ly, zm])
    fork = np.array([0.4 * lx, 0.5 * ly, zm])
    leaves = [np.array([lx - 0.5, 0.2 * ly, zm]), np.array([lx - 0.5, 0.8 * ly, zm])]
    pts, edges = [root], []

    def line(start_id, a, b):
        m = max(1, int(math.ceil(np.linalg.norm(b - a) / seg - 1e-9)))
        prev = start_id
        for s in range(1, m + 1):
            pts.append(a + (b - a) * (s / m))
            edges.append((prev, len(pts) - 1))
            prev = len(pts) - 1
        return prev

    f = line(0, root, fork)
    # branch labels: trunk -1, branch to leaf k: k (all generation 0)
    side = [-1] * len(edges)
    leaf_ids = []
    for k, q in enumerate(leaves):
        leaf_ids.append(line(f, fork, q))
        side += [k] * (len(edges) - len(side))
    side = np.array(side, np.int8)
    pxyz = np.array(pts)
    if pmj_amp is None:
        pmj_amp = -200.0 if drive == "graph" else -1000.0
    pk = Purkinje(xyz=pxyz, edges=np.array(edges, np.int32), pmj_nodes=np.array(leaf_ids, np.int32),
                  pmj_radius=0.6, two_way=two_way, pmj_amp=pmj_amp, edge_side=side,
                  edge_depth=np.zeros(len(edges), np.int32))
    stimuli = []
    if drive == "graph":
        ids = np.nonzero(np.linalg.norm(pxyz - root, axis=1) <= 0.5)[0].astype(np.int32)
        stimuli.append(Stimulus(ids=ids, t0=0.0, dur=1.0, amp=-100.0, domain=1))
    else:
        cen = xyz[tets].mean(axis=1)
        ids = np.nonzero(np.linalg.norm(cen - pxyz[leaf_ids[0]], axis=1) <= 1.0)[0].astype(np.int32)
        stimuli.append(Stimulus(ids=ids, t0=0.0, dur=1.0, amp=-52.0))
    w = Workload(f"purkinje-slab-{nx}x{ny}x{nz}-h{h}", xyz, tets, _uniform_fibre(n),
                 np.full(n, TP06_ENDO, np.uint8), stimuli=stimuli, dt=dt, n_steps=n_steps,
                 hex_ijk=hijk, dims=(nx, ny, nz, h))
    w.purkinje = pk
    return w
