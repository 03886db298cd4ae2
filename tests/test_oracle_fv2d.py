"""Pins of the oracle's 2D medium: cell-centred finite volumes on triangles
(Sec. 3.2: the 2D Purkinje shell uses the same scheme as the 3D myocardium
on triangles; node values by inverse distance, edge values as node means,
Gauss-Green cell gradients, alpha-weighted edge gradients with the eq.
gra2bis correction, fluxes through the edges).

Independent checks: closed-form geometry of the triangulated rectangle, the
exact gradient of linear fields, conservation and constants on flat and bent
sheets, the mean of the operator on quadratics against div(M grad q), the
slowest cosine mode's decay rate, the sheet's conduction velocity against a
1D chain of the same cells, a bent sheet against a flat one, and a mixed
mesh (tets plus triangles) against the two media run apart.
"""
import math

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

CHI, CM = M.CHI, M.CM


def passive_sheet(nx, ny, h=0.5, angle=0.0, R=0.0, sl=M.SIGMA_L, st=M.SIGMA_T, scale=None):
    w = M.sheet_workload(nx, ny, h, model=M.PASSIVE, sigma_l=sl, sigma_t=st,
                         curvature_radius=R, fibre_angle_deg=angle)
    w.stimuli = []
    w.scale = scale
    return w


def centroids(w):
    return w.xyz[w.tets[:, :3]].mean(axis=1)


def interior(w, rings=1):
    """Triangles whose square lies at least 1 + rings squares from the edge
    (their nodes and their neighbours' nodes are all interior)."""
    nx, ny, _, h = w.dims
    c = centroids(w)
    i = np.floor(c[:, 0] / h).astype(int)
    j = np.floor(c[:, 1] / h).astype(int)
    lo = 1 + rings
    return np.nonzero((i >= lo) & (i < nx - lo) & (j >= lo) & (j < ny - lo))[0]


def test_sheet_geometry_closed_forms(oracle_lib):
    nx, ny, h = 6, 4, 0.5
    w = passive_sheet(nx, ny, h)
    s = oracle_lib.Sim(w)
    area, S, nbr = s.geometry()
    assert area.sum() == pytest.approx(nx * ny * h * h, rel=1e-14)
    assert np.allclose(area, 0.5 * h * h)
    # per triangle: three in-plane edge vectors closing to zero, each of the
    # edge's length and pointing away from the centroid
    assert np.abs(S[:, :3].sum(axis=1)).max() < 1e-14
    assert np.abs(S[:, :, 2]).max() == 0.0 and np.abs(S[:, 3]).max() == 0.0
    c = centroids(w)
    for t in range(w.n_tets):
        tri = w.tets[t, :3]
        for j in range(3):
            a, b = w.xyz[tri[(j + 1) % 3]], w.xyz[tri[(j + 2) % 3]]
            assert np.linalg.norm(S[t, j]) == pytest.approx(np.linalg.norm(b - a), rel=1e-14)
            assert abs(np.dot(S[t, j], b - a)) < 1e-14
            assert np.dot(S[t, j], 0.5 * (a + b) - c[t]) > 0
    # neighbours: symmetric, 2 (nx + ny) boundary edges
    assert (nbr[:, 3] == -1).all()
    assert (nbr[:, :3] < 0).sum() == 2 * (nx + ny)
    for t in range(w.n_tets):
        for j in range(3):
            if nbr[t, j] >= 0:
                assert t in nbr[nbr[t, j], :3]


def test_linear_field_gradient_exact(oracle_lib):
    """Inverse-distance node values of a linear field are exact at interior
    nodes (their triangles' centroids are point-symmetric), and Gauss-Green
    with edge means is then the exact gradient."""
    w = passive_sheet(10, 8, 0.5)
    s = oracle_lib.Sim(w)
    g = s.gradients(centroids(w) @ np.array([1.5, -0.7, 0.0]) + 3.0)
    inner = interior(w, rings=0)
    assert np.abs(g[inner] - np.array([1.5, -0.7, 0.0])).max() < 1e-12


@pytest.mark.parametrize("R", [0.0, 3.0])
def test_constants_and_conservation(oracle_lib, R):
    """L 1 = 0, and sum_c A_c L_c = 0 for any field (the edge fluxes cancel
    in pairs, also on a bent sheet), with rotated anisotropic fibres and a
    cell-wise conductivity scale."""
    rng = np.random.default_rng(2)
    w = passive_sheet(9, 7, 0.5, angle=35.0, R=R, scale=rng.uniform(0.5, 2.0, 9 * 7 * 2))
    s = oracle_lib.Sim(w)
    area, _, _ = s.geometry()
    assert np.abs(s.apply_diffusion(np.full(w.n_tets, -80.0))).max() < 1e-12
    L = s.apply_diffusion(rng.normal(size=w.n_tets) * 30.0)
    assert abs((area * L).sum()) < 1e-11 * np.abs(area * L).sum()


def test_linear_field_null(oracle_lib):
    w = passive_sheet(10, 10, 0.5, angle=25.0)
    s = oracle_lib.Sim(w)
    L = s.apply_diffusion(centroids(w) @ np.array([1.0, -2.0, 0.0]) + 4.0)
    inner = interior(w, rings=1)
    assert inner.size > 50
    assert np.abs(L[inner]).max() < 1e-11


@pytest.mark.parametrize("angle,field,expect", [
    (0.0, "xx", "2l"), (0.0, "yy", "2t"), (90.0, "yy", "2l"), (45.0, "xy", "l-t")])
def test_quadratic_area_mean(oracle_lib, angle, field, expect):
    """Over interior triangles the area-weighted mean of L(q) equals
    div(M grad q)/(chi Cm) with the in-plane tensor M = s_t I + (s_l - s_t) f f^T."""
    w = passive_sheet(12, 12, 0.5, angle=angle)
    s = oracle_lib.Sim(w)
    area, _, _ = s.geometry()
    x = centroids(w)
    ax = {"x": 0, "y": 1}
    q = x[:, ax[field[0]]] * x[:, ax[field[1]]]
    L = s.apply_diffusion(q)
    inner = interior(w, rings=1)
    mean = (area[inner] * L[inner]).sum() / area[inner].sum()
    sl, st = M.SIGMA_L, M.SIGMA_T
    target = {"2l": 2 * sl, "2t": 2 * st, "l-t": sl - st}[expect] / (CHI * CM)
    assert abs(mean - target) < 1e-3 * abs(target)


def test_cosine_mode_decay(oracle_lib):
    """The slowest Neumann mode cos(pi x / Lx) decays at a rate converging
    to D_l pi^2 / Lx^2 under refinement (second-order scheme)."""
    Lx = 4.0
    errs = []
    for h in (0.5, 0.25):
        w = passive_sheet(int(Lx / h), 4, h)
        s = oracle_lib.Sim(w)
        area, _, _ = s.geometry()
        v = np.cos(math.pi * centroids(w)[:, 0] / Lx)
        L = s.apply_diffusion(v)
        rate = -(area * v * L).sum() / (area * v * v).sum()
        exact = M.SIGMA_L / (CHI * CM) * math.pi ** 2 / Lx ** 2
        errs.append(abs(rate - exact) / exact)
    assert errs[1] < 0.02 and errs[1] < 0.5 * errs[0]


def sheet_cv(oracle_lib, R=0.0, h=0.25):
    w = M.sheet_workload(56, 8, h, curvature_radius=R)
    s = oracle_lib.Sim(w)
    s.step(int(round(20.0 / w.dt)))
    at = s.activation()
    x = centroids(w)[:, 0]
    a = np.abs(x - 4.0) < h
    b = np.abs(x - 9.0) < h
    return (x[b].mean() - x[a].mean()) / (at[b].mean() - at[a].mean()), at


def test_sheet_velocity_matches_a_chain(oracle_lib):
    """A planar wave along the fibres of a TP06 sheet travels at the speed
    of a 1D chain of the same cells and conductivity (the 2D scheme reduces
    to the 1D one for a planar wave; 5 % band for the two discretisations)."""
    cv2, _ = sheet_cv(oracle_lib)
    from test_oracle_purkinje import chain_workload
    w = chain_workload(161, 0.1, model=M.TP06_ENDO, sigma=M.SIGMA_L, stim_nodes=list(range(10)),
                       stim_amp=-52.0, stim_dur=1.0)
    s = oracle_lib.Sim(w)
    s.step(int(round(20.0 / w.dt)))
    ta = s.purkinje_activation()
    x = w.purkinje.xyz[:, 0]
    i0, i1 = np.argmin(abs(x - 4.0)), np.argmin(abs(x - 9.0))
    cv1 = (x[i1] - x[i0]) / (ta[i1] - ta[i0])
    assert cv2 == pytest.approx(cv1, rel=0.05)


def test_bent_sheet_conducts_like_a_flat_one(oracle_lib):
    """Bending the sheet around its propagation axis changes no length along
    the wave: the activation times of the bent sheet equal the flat one's
    within 1 %."""
    cv_flat, at_flat = sheet_cv(oracle_lib)
    cv_bent, at_bent = sheet_cv(oracle_lib, R=2.0)
    assert cv_bent == pytest.approx(cv_flat, rel=0.01)
    both = np.isfinite(at_flat) & np.isfinite(at_bent)
    assert both.mean() > 0.9
    assert np.abs(at_bent[both] - at_flat[both]).max() < 0.02 * np.nanmax(at_flat)


def test_mixed_mesh_equals_media_apart(oracle_lib):
    """Tets and triangles in one simulation (disjoint nodes) evolve exactly
    as the two media do on their own."""
    w3 = M.config1(n_steps=0, nx=8, ny=6, nz=2)
    w2 = M.sheet_workload(12, 6, 0.5, model=M.CRN, n_steps=0)
    mix = M.mixed_workload(w3, w2)
    a, b, c = oracle_lib.Sim(mix), oracle_lib.Sim(w3), oracle_lib.Sim(w2)
    for o in (a, b, c):
        o.step(400)
    v = a.vm()
    assert np.array_equal(v[:w3.n_tets], b.vm())
    assert np.array_equal(v[w3.n_tets:], c.vm())
    at = a.activation()
    assert np.isfinite(at[w3.n_tets:]).any() and np.isfinite(at[:w3.n_tets]).any()


# ----------------------------------- communication nodes from the 2D shell
N3 = 16 * 8 * 2 * 5          # tets of the default shell_on_slab


def test_cell_junction_region_is_the_other_medium(oracle_lib):
    """Sec. 3.3: a communication node stimulates the cells of the other
    medium within R_S: brute-force centroid search restricted to tets; with
    a radius that holds no centroid, the tets sharing a node with the
    nearest tet."""
    w = M.shell_on_slab()
    s = oracle_lib.Sim(w)
    cen = w.xyz[np.where(w.tets >= 0, w.tets, w.tets[:, :1])].mean(axis=1)
    cen[N3:] = w.xyz[w.tets[N3:, :3]].mean(axis=1)
    for k, cj in enumerate(w.cell_junctions[:6]):
        d = np.linalg.norm(cen[:N3] - cen[cj.cell], axis=1)
        assert np.array_equal(np.sort(s.pmj_region(k)), np.nonzero(d <= cj.radius)[0])
    w0 = M.shell_on_slab(radius=0.0)
    s0 = oracle_lib.Sim(w0)
    cj = w0.cell_junctions[0]
    d = np.linalg.norm(cen[:N3] - cen[cj.cell], axis=1)
    near = w0.tets[int(np.argmin(d))]
    star = np.nonzero(np.isin(w0.tets[:N3], near).any(axis=1))[0]
    assert np.array_equal(np.sort(s0.pmj_region(0)), star)


def test_cell_junction_orthodromic_timing(oracle_lib):
    """The source triangle crossing the threshold during step n pulses the
    tets of its region from step n + 1 + round(5 ms / dt): at rest until
    then, then raised by about -amp dt per pulsed step."""
    w = M.shell_on_slab(drive="sheet")
    s = oracle_lib.Sim(w)
    dt = w.dt
    cj = w.cell_junctions[0]
    s.step(200)
    tn = s.activation()[cj.cell]
    assert np.isfinite(tn)
    fire = int(math.floor(tn / dt)) + 1 + int(round(cj.delay_ortho / dt))
    region = s.pmj_region(0)
    v_rest = s.vm()[region]
    s.step(fire - 200)
    v_before = s.vm()[region]
    assert np.all(abs(v_before - v_rest) < 0.05)
    s.step(1)
    assert np.all(s.vm()[region] - v_before > 0.5 * (-cj.amp) * dt)


def test_cell_junction_two_way(oracle_lib):
    """Driving the slab: with two-way nodes the region mean crossing during
    step n pulses the source triangle from n + 1 + round(3 ms / dt), and the
    shell then activates; one-way nodes leave the shell at rest."""
    w = M.shell_on_slab(drive="slab", two_way=True)
    s = oracle_lib.Sim(w)
    dt = w.dt
    region = s.pmj_region(0)
    cj = w.cell_junctions[0]
    m_prev = s.vm()[region].mean()
    n_cross = None
    for n in range(400):
        s.step(1)
        m = s.vm()[region].mean()
        if m_prev <= 0.0 < m:
            n_cross = n
            break
        m_prev = m
    assert n_cross is not None
    fire = n_cross + 1 + int(round(cj.delay_anti / dt))
    s.step(fire - s.step_index)               # steps 0 .. fire-1 done
    assert np.isnan(s.activation()[N3:]).all()   # no shell cell has fired yet
    v_src = s.vm()[cj.cell]
    s.step(1)                                 # step `fire`: first pulse on the source
    assert s.vm()[cj.cell] - v_src > 0.5 * (-cj.amp) * dt
    s.step(300)
    assert np.isfinite(s.activation()[N3:]).all()
    s1 = oracle_lib.Sim(M.shell_on_slab(drive="slab", two_way=False))
    s1.step(750)
    assert np.isnan(s1.activation()[N3:]).all()


# ------------------------------------- the 2D medium's own time step
def _fine(w, m):
    """The same workload stepping at dt / m (as m substeps would)."""
    import copy
    f = copy.copy(w)
    f.dt = w.dt / m
    f.medium_substeps = None
    return f


@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_medium_substeps_equal_a_sheet_at_the_small_step(oracle_lib, scheme):
    """A sheet with n_sub substeps per step of dt is the sheet stepped at
    dt / n_sub (Sec. 4: the shell runs at its own, smaller time step): the
    same potentials, activation times and APD90 bit for bit, with forward
    Euler, Adams-Bashforth 2 and the second-order Rush-Larsen variant."""
    m = 5
    w = M.sheet_workload(24, 6, 0.5, model=M.STEWART, dt=0.02)
    w.time_scheme = scheme
    w.medium_substeps = m
    a = oracle_lib.Sim(w)
    assert a.medium_substeps() == m
    b = oracle_lib.Sim(_fine(w, m))
    a.step(1300)
    b.step(1300 * m)
    assert np.array_equal(a.vm(), b.vm())
    assert np.array_equal(a.activation(), b.activation(), equal_nan=True)
    assert np.array_equal(a.apd90(), b.apd90(), equal_nan=True)
    assert np.isfinite(a.activation()).mean() > 0.9


def test_medium_substeps_leave_the_3d_medium_alone(oracle_lib):
    """In a mesh of tets and a separate sheet, substepping the sheet changes
    nothing in the tets (which step at dt) and makes the sheet evolve as it
    does alone at dt / n_sub."""
    m = 4
    w3 = M.config1(n_steps=0, nx=8, ny=6, nz=2)
    w2 = M.sheet_workload(12, 6, 0.5, model=M.CRN, n_steps=0)
    mix = M.mixed_workload(w3, w2)
    mix.medium_substeps = m
    a, b, c = oracle_lib.Sim(mix), oracle_lib.Sim(w3), oracle_lib.Sim(_fine(w2, m))
    a.step(400)
    b.step(400)
    c.step(400 * m)
    v = a.vm()
    assert np.array_equal(v[:w3.n_tets], b.vm())
    assert np.array_equal(v[w3.n_tets:], c.vm())
    at = a.activation()
    assert np.array_equal(at[w3.n_tets:], c.activation(), equal_nan=True)
    assert np.isfinite(at[w3.n_tets:]).any() and np.isfinite(at[:w3.n_tets]).any()


def _operator_matrix(s, n):
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = s.apply_diffusion(e)
    return A


@pytest.mark.parametrize("angle", [0.0, 30.0])
def test_derived_substeps_make_the_step_stable(oracle_lib, angle):
    """With n_sub <= 0 the count comes from the medium's own forward-Euler
    bound: on a fine, highly conducting sheet the step dt alone is unstable
    (some eigenvalue of the assembled operator has |1 + dt lambda| > 1), the
    derived substep dt / n_sub is stable for every eigenvalue, and the count
    is the smallest within 90 % of the bound computed here from the
    geometry (edge lengths, centroid distances, areas)."""
    w = passive_sheet(8, 6, 0.1, angle=angle, scale=np.full(96, 4.0))
    w.medium_substeps = 0
    s = oracle_lib.Sim(w)
    m = s.medium_substeps()
    lam = np.linalg.eigvals(_operator_matrix(s, w.n_tets))
    assert np.abs(1 + w.dt * lam).max() > 1.0
    assert np.abs(1 + (w.dt / m) * lam).max() <= 1.0 + 1e-12
    # the bound from the geometry
    T = w.tets[:, :3]
    P = w.xyz[T]
    cen = P.mean(axis=1)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    owner = {}
    for c in range(w.n_tets):
        for j in range(3):
            owner.setdefault(frozenset((T[c, (j + 1) % 3], T[c, (j + 2) % 3])), []).append(c)
    r = np.zeros(w.n_tets)
    for c in range(w.n_tets):
        for j in range(3):
            a, b = T[c, (j + 1) % 3], T[c, (j + 2) % 3]
            other = [k for k in owner[frozenset((a, b))] if k != c]
            if not other:
                continue
            edge = np.linalg.norm(w.xyz[b] - w.xyz[a])
            r[c] += edge / np.linalg.norm(cen[other[0]] - cen[c])
    r *= max(w.sigma_l, w.sigma_t) * 4.0 / (CHI * CM * area)
    dtmax = 1.0 / r.max()
    expect = 1
    while w.dt / expect > 0.9 * dtmax:
        expect += 1
    assert m == expect and m > 1
    # and the bound is one: every eigenvalue lies in [-2 max r, 0] (real part)
    assert lam.real.min() >= -2 * r.max() * (1 + 1e-9)


def test_passive_mode_decays_at_the_substep_rate(oracle_lib):
    """A passive sheet started on an eigenvector phi of its operator
    (eigenvalue lambda < 0) is (1 + h lambda)^k phi after k substeps of
    h = dt / n_sub: the substep count and size, checked on the potential."""
    m = 3
    w = passive_sheet(8, 4, 0.5)
    s0 = oracle_lib.Sim(w)
    A = _operator_matrix(s0, w.n_tets)
    lam, vec = np.linalg.eig(A)
    real = np.abs(lam.imag) < 1e-12
    i = np.argmin(np.where(real, lam.real, 0.0))
    phi, l = vec[:, i].real, lam[i].real
    assert l < 0
    w.medium_substeps = m
    s = oracle_lib.Sim(w)
    st = s.states()
    st[0] = phi
    s.set_states(st)
    n = 7
    s.step(n)
    expect = (1 + (w.dt / m) * l) ** (n * m) * phi
    assert np.abs(s.vm() - expect).max() < 1e-10 * np.abs(phi).max()
