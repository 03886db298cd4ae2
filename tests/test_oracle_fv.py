"""Pins of the oracle's geometry and finite-volume diffusion operator
(Sec. 3.2 of the paper: node values, Gauss-Green gradients, eq. gra2bis face
gradients, the face-flux balance of eq. electro2_3dmono) against closed
forms, invariants and brute force on tiny meshes."""
import math

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

CHI, CM = M.CHI, M.CM


def passive(nx, ny, nz, h=0.5, fibre=None, sl=M.SIGMA_L, st=M.SIGMA_T,
            dt=0.02, perm_seed=None, scale=None, split=5):
    xyz, tets, hijk = (M.slab if split == 5 else M.slab6)(nx, ny, nz, h)
    if perm_seed is not None:
        rng = np.random.default_rng(perm_seed)
        tets = np.array([t[rng.permutation(4)] for t in tets], dtype=np.int32)
    n = tets.shape[0]
    f = np.zeros((n, 3)); f[:, 0] = 1.0
    if fibre is not None:
        f[:] = fibre
    return M.Workload("passive", xyz, tets, f, np.full(n, M.PASSIVE, np.uint8),
                      sigma_l=sl, sigma_t=st, scale=scale, dt=dt, hex_ijk=hijk,
                      dims=(nx, ny, nz, h))


def centroids(w):
    return w.xyz[w.tets].mean(axis=1)


def interior_cells(w, rings=1):
    """Cells none of whose nodes, nor their face neighbours' nodes, lie on
    the boundary (stencil-interior, the cells where P5 must hold)."""
    nx, ny, nz, h = w.dims
    ijk = np.rint(w.xyz / h).astype(int)
    bnode = ((ijk == 0) | (ijk == np.array([nx, ny, nz]))).any(axis=1)
    hij = w.hex_ijk
    lo = 1 + rings
    sel = ((hij >= lo) & (hij < np.array([nx, ny, nz]) - lo)).all(axis=1)
    assert not bnode[w.tets[sel]].any()
    return np.nonzero(sel)[0]


# ---------------------------------------------------------------- geometry
@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 2, 2), (20, 20, 4)])
def test_geometry_closed_forms(oracle_lib, dims):
    nx, ny, nz = dims
    h = 0.5
    w = passive(nx, ny, nz, h, perm_seed=1)
    s = oracle_lib.Sim(w)
    vol, S, nbr = s.geometry()
    # P1: volumes add up to the box; each tet's four area vectors close
    assert math.isclose(vol.sum(), nx * ny * nz * h ** 3, rel_tol=1e-13)
    assert np.abs(S.sum(axis=1)).max() < 1e-14
    # every hex split into five tets: central tet has volume h^3/3
    v5 = vol.reshape(-1, 5)
    assert np.allclose(v5[:, 0], h ** 3 / 3, rtol=1e-13)
    assert np.allclose(v5[:, 1:], h ** 3 / 6, rtol=1e-13)
    # boundary triangles: 2 per boundary square
    assert (nbr < 0).sum() == 2 * 2 * (nx * ny + nx * nz + ny * nz)
    # neighbour relation is symmetric and area vectors are opposite
    c, j = np.nonzero(nbr >= 0)
    c2 = nbr[c, j]
    back = (nbr[c2] == c[:, None])
    assert back.sum(axis=1).min() == 1
    j2 = back.argmax(axis=1)
    assert np.abs(S[c, j] + S[c2, j2]).max() < 1e-14
    # outward: the area vector points away from the opposite vertex
    cen = centroids(w)
    opp = w.xyz[w.tets[c, j]]
    assert (np.einsum("ij,ij->i", S[c, j], cen[c] - opp) > 0).all()


def test_kuhn_split_geometry_and_operator(oracle_lib):
    """The 6-tet (Kuhn) split of the convergence study: six tets of volume
    h^3/6 per hex, the same boundary-triangle count, closed area vectors,
    and the operator invariants P3-P5 (constants steady, conservation,
    linear fields null at stencil-interior cells: every node of this lattice
    is point-symmetric too)."""
    nx, ny, nz, h = 8, 7, 7, 0.5
    w = passive(nx, ny, nz, h, fibre=np.array([math.cos(0.3), math.sin(0.3), 0.0]), split=6)
    s = oracle_lib.Sim(w)
    vol, S, nbr = s.geometry()
    assert np.allclose(vol, h ** 3 / 6, rtol=1e-13)
    assert np.abs(S.sum(axis=1)).max() < 1e-14
    assert (nbr < 0).sum() == 2 * 2 * (nx * ny + nx * nz + ny * nz)
    assert np.abs(s.apply_diffusion(np.full(w.n_tets, -80.0))).max() < 1e-11
    v = np.random.default_rng(2).normal(size=w.n_tets) * 30
    L = s.apply_diffusion(v)
    assert abs((vol * L).sum()) < 1e-12 * (vol * np.abs(L)).sum()
    lin = centroids(w) @ np.array([1.0, -2.0, 0.5]) + 4.0
    inner = interior_cells(w, rings=1)
    assert inner.size > 50
    assert np.abs(s.apply_diffusion(lin)[inner]).max() < 1e-11


def test_orientation_invariance(oracle_lib):
    """Results must not depend on the vertex order inside each tet."""
    rng = np.random.default_rng(3)
    outs = []
    for perm in (None, 7):
        w = passive(4, 3, 2, perm_seed=perm)
        s = oracle_lib.Sim(w)
        v = np.sin(centroids(w) @ np.array([0.7, 1.3, 2.1]))
        outs.append(s.apply_diffusion(v))
    assert np.abs(outs[0] - outs[1]).max() < 1e-13


# ------------------------------------------------------------- gradients
def test_gauss_green_equals_p1_gradient(oracle_lib):
    """P2: Gauss-Green with face values = mean of node values is the P1
    gradient; check against a linear solve through the four nodal values."""
    w = passive(3, 3, 3, 0.5, perm_seed=2)
    s = oracle_lib.Sim(w)
    rng = np.random.default_rng(0)
    v = rng.normal(size=w.n_tets)
    g = s.gradients(v)
    vn = s.node_values(v)
    X = w.xyz[w.tets]                       # [n,4,3]
    A = X[:, 1:, :] - X[:, :1, :]
    b = vn[w.tets[:, 1:]] - vn[w.tets[:, :1]]
    g_ref = np.linalg.solve(A, b[..., None])[..., 0]
    assert np.abs(g - g_ref).max() < 1e-11 * np.abs(g_ref).max()


def test_node_weights_partition_of_unity(oracle_lib):
    w = passive(3, 2, 2, perm_seed=4)
    s = oracle_lib.Sim(w)
    vn = s.node_values(np.full(w.n_tets, 3.25))
    assert np.abs(vn - 3.25).max() < 1e-14


def test_linear_field_exact_at_interior(oracle_lib):
    """Interior nodes of the alternating 5-tet lattice are point-symmetric,
    so inverse-distance node values (and hence gradients) of a linear cell
    field are exact there."""
    w = passive(6, 6, 6, 0.5)
    s = oracle_lib.Sim(w)
    a = np.array([0.3, -1.1, 0.7])
    v = centroids(w) @ a + 2.0
    g = s.gradients(v)
    inner = interior_cells(w, rings=0)
    assert np.abs(g[inner] - a).max() < 1e-12


# -------------------------------------------------------------- operator
def test_constants_are_steady(oracle_lib):
    """P3: L 1 = 0."""
    w = passive(5, 4, 3, perm_seed=5)
    s = oracle_lib.Sim(w)
    L = s.apply_diffusion(np.full(w.n_tets, -80.0))
    assert np.abs(L).max() < 1e-11


def test_conservation(oracle_lib):
    """P4: with no-flux boundaries sum_c V_c L_c = 0 for any field."""
    w = passive(5, 4, 3, perm_seed=6,
                fibre=np.array([0.6, 0.8, 0.0]))
    w.scale = np.random.default_rng(9).uniform(0.5, 2.0, w.n_tets)
    s = oracle_lib.Sim(w)
    vol, _, _ = s.geometry()
    v = np.random.default_rng(1).normal(size=w.n_tets) * 30
    L = s.apply_diffusion(v)
    assert abs((vol * L).sum()) < 1e-12 * (vol * np.abs(L)).sum()


def test_linear_field_null(oracle_lib):
    """P5: L(a.x + b) = 0 wherever the stencil avoids boundary nodes."""
    f = np.array([math.cos(0.4), math.sin(0.4), 0.0])
    w = passive(7, 7, 7, 0.5, fibre=f)
    s = oracle_lib.Sim(w)
    v = centroids(w) @ np.array([1.0, -2.0, 0.5]) + 4.0
    L = s.apply_diffusion(v)
    inner = interior_cells(w, rings=1)
    assert inner.size > 50
    assert np.abs(L[inner]).max() < 1e-11


@pytest.mark.parametrize("fdir,field,expect", [
    ((1, 0, 0), "xx", "2l"), ((1, 0, 0), "yy", "2t"), ((1, 0, 0), "zz", "2t"),
    ((0, 1, 0), "yy", "2l"), ((1, 1, 0), "xy", "l-t")])
def test_quadratic_volume_mean(oracle_lib, fdir, field, expect):
    """P6: over stencil-interior cells the volume-weighted mean of L applied
    to a quadratic equals div(M grad q)/(chi Cm); this pins the fibre tensor
    M = s_t I + (s_l - s_t) f f^T and the chi Cm scaling."""
    f = np.array(fdir, float) / np.linalg.norm(fdir)
    w = passive(8, 8, 8, 0.5, fibre=f)
    s = oracle_lib.Sim(w)
    vol, _, _ = s.geometry()
    x = centroids(w)
    ax = {"x": 0, "y": 1, "z": 2}
    q = x[:, ax[field[0]]] * x[:, ax[field[1]]]
    L = s.apply_diffusion(q)
    inner = interior_cells(w, rings=1)
    mean = (vol[inner] * L[inner]).sum() / vol[inner].sum()
    sl, st = M.SIGMA_L, M.SIGMA_T
    target = {"2l": 2 * sl, "2t": 2 * st, "l-t": sl - st}[expect] / (CHI * CM)
    assert abs(mean - target) < 1e-3 * abs(target) + 1e-12


def dense_operator(s, n):
    Ld = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n); e[k] = 1.0
        Ld[:, k] = s.apply_diffusion(e)
    return Ld


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (4, 2, 1)])
def test_dense_spectrum(oracle_lib, dims):
    """P15 brute force: the assembled operator has a one-dimensional kernel
    (constants), a real non-positive spectrum (stabilised face gradients),
    and V L is conservative column-wise."""
    f = np.array([math.cos(0.3), math.sin(0.3), 0.2]); f /= np.linalg.norm(f)
    w = passive(*dims, fibre=f, perm_seed=8)
    s = oracle_lib.Sim(w)
    n = w.n_tets
    Ld = dense_operator(s, n)
    vol, _, _ = s.geometry()
    assert np.abs(vol @ Ld).max() < 1e-12 * np.abs(Ld).max()
    ev = np.linalg.eigvals(Ld)
    scale = np.abs(ev).max()
    assert ev.real.max() < 1e-10 * scale
    assert np.abs(ev.imag).max() < 1e-8 * scale
    assert (np.abs(ev) < 1e-10 * scale).sum() == 1


def test_stability_limit(oracle_lib):
    """P7: forward Euler on the PASSIVE operator is stable below
    dt_max = 2/|lambda_max| and unstable above it (4 x 4 x 2 slab)."""
    w = passive(4, 4, 2, 0.5)
    s = oracle_lib.Sim(w)
    Ld = dense_operator(s, w.n_tets)
    lam = np.abs(np.linalg.eigvals(Ld).real).max()
    dtmax = 2.0 / lam
    # h = 0.5 mm with (0.17, 0.019) mS/mm gives a limit of order 0.1-0.2 ms
    assert 0.05 < dtmax < 0.4
    rng = np.random.default_rng(2)
    for fac, grows in ((0.98, False), (1.02, True)):
        ww = passive(4, 4, 2, 0.5, dt=fac * dtmax)
        ss = oracle_lib.Sim(ww)
        st = ss.states()
        st[0] = -80 + rng.normal(size=ww.n_tets)
        ss.set_states(st)
        ss.step(3000)
        amp = np.abs(ss.vm() - ss.vm().mean()).max()
        assert (amp > 10.0) == grows


def test_cosine_mode_decay(oracle_lib):
    """P8: the slowest Neumann mode cos(pi x / Lx) decays at a rate that
    converges to D_l pi^2 / Lx^2, D_l = sigma_l/(chi Cm), under refinement."""
    Lx = 4.0
    rates = []
    for h in (0.5, 0.25):
        nx = int(Lx / h)
        w = passive(nx, 2, 1, h, dt=0.005)
        s = oracle_lib.Sim(w)
        vol, _, _ = s.geometry()
        v = np.cos(math.pi * centroids(w)[:, 0] / Lx)
        L = s.apply_diffusion(v)
        rates.append(-(vol * v * L).sum() / (vol * v * v).sum())
    exact = M.SIGMA_L / (CHI * CM) * math.pi ** 2 / Lx ** 2
    err = [abs(r - exact) / exact for r in rates]
    assert err[1] < 0.05 and err[1] < err[0]


def test_passive_conserves_charge_over_time(oracle_lib):
    w = passive(4, 3, 2, perm_seed=3, fibre=np.array([0.0, 0.6, 0.8]))
    s = oracle_lib.Sim(w)
    vol, _, _ = s.geometry()
    st = s.states()
    st[0] = np.random.default_rng(5).normal(size=w.n_tets) * 20 - 60
    s.set_states(st)
    q0 = (vol * s.vm()).sum()
    s.step(200)
    assert abs((vol * s.vm()).sum() - q0) < 1e-11 * abs(q0)


@pytest.mark.parametrize("shear", [0.0, 0.6])
def test_quadratic_mean_sheared_isotropic(oracle_lib, shear):
    """P6 on an affine (sheared) lattice with isotropic conductivity: the
    interior volume mean of L(x^2), L(z^2) is 2 sigma/(chi Cm) and of L(xy)
    is 0.  Unlike the axis-aligned case this depends on the interpolated
    face gradient using both cell gradients."""
    nx = 8
    xyz, tets, hijk = M.slab(nx, nx, nx, 0.5)
    A = np.array([[1, shear, 0.2], [0, 1, 0.3], [0, 0, 1.0]])
    xyz = xyz @ A.T
    n = tets.shape[0]
    f = np.zeros((n, 3)); f[:, 0] = 1
    w = M.Workload("p", xyz, tets, f, np.full(n, M.PASSIVE, np.uint8),
                   sigma_l=0.1, sigma_t=0.1, hex_ijk=hijk, dims=(nx, nx, nx, 0.5))
    s = oracle_lib.Sim(w)
    vol, _, _ = s.geometry()
    x = centroids(w)
    sel = ((hijk >= 2) & (hijk < nx - 2)).all(axis=1)
    for q, target in ((x[:, 0] ** 2, 0.2), (x[:, 0] * x[:, 1], 0.0),
                      (x[:, 2] ** 2, 0.2)):
        L = s.apply_diffusion(q)
        mean = (vol[sel] * L[sel]).sum() / vol[sel].sum()
        assert abs(mean - target / (CHI * CM)) < 1e-9


# ------------------------------------------------- alpha off the lattice
def test_alpha_worked_example_two_tets(oracle_lib):
    """Face interpolation weight alpha (Sec. 3.2, the weights of eq. gra2bis)
    pinned where it matters: a face whose centre-to-centre line is not
    parallel to its normal.  Worked by hand:

    Nodes O = 0, X = e_x, Y = e_y, Z = e_z, Q = (1, 1, 0); tet A = OXYZ,
    tet B = XYZQ (both volume 1/6); shared face XYZ, outward from A
    S = (1, 1, 1)/2.  Centroids x_A = (1, 1, 1)/4, x_B = (2, 2, 1)/4,
    face centroid x_f = (1, 1, 1)/3, so |x_A - x_f| = sqrt(3)/12,
    |x_B - x_f| = 1/4 and alpha_A = (1/4)/(sqrt(3)/12 + 1/4) = (3 - sqrt 3)/2,
    alpha_B = (sqrt 3 - 1)/2.  d = |x_B - x_A| = sqrt(2)/4,
    e = (1, 1, 0)/sqrt 2, S.e = 1/sqrt 2, S - (S.e)e = (0, 0, 1/2).

    v_A = 1, v_B = 0.  Node values by inverse distance to the centroids:
    O -> 1, Q -> 0; X and Y lie sqrt(11)/4 from x_A and 3/4 from x_B, so
    p = v_X = v_Y = 3/(3 + sqrt 11); Z lies sqrt(11)/4 and sqrt(17)/4 away,
    q = v_Z = sqrt 17/(sqrt 17 + sqrt 11).  Cell gradients (the P1
    gradients of the node values): g_A = (p - 1, p - 1, q - 1),
    g_B = (-p, -p, q - 2p); their jump is along (1, 1, 1), the face normal.

    Isotropic conductivity sigma scaled by 1 in A and 3 in B: the face tensor
    is (alpha_A + 3 alpha_B) sigma I = sqrt(3) sigma I.  The stabilised face
    gradient keeps the part of gbar = alpha_A g_A + alpha_B g_B across e and
    replaces its e-component by (v_B - v_A)/d, so the flux out of A is
    sqrt(3) sigma (gbar_z / 2 - 2) with gbar_z = q - alpha_A - 2 p alpha_B,
    and L_A = 6 F / (chi Cm) = -L_B.

    Swapping alpha for 1 - alpha changes both the face tensor (to
    (4 - sqrt 3) sigma) and gbar_z (to q - alpha_B - 2 p alpha_A)."""
    s3, s11, s17 = math.sqrt(3.0), math.sqrt(11.0), math.sqrt(17.0)
    aA, aB = (3.0 - s3) / 2.0, (s3 - 1.0) / 2.0
    p, q = 3.0 / (3.0 + s11), s17 / (s17 + s11)
    sig = 0.1
    flux = s3 * sig * ((q - aA - 2.0 * p * aB) / 2.0 - 2.0)
    LA = 6.0 * flux / (CHI * CM)

    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0]], float)
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32)
    fib = np.array([[1.0, 0, 0], [0, 1.0, 0]])
    w = M.Workload("two-tets", xyz, tets, fib, np.full(2, M.PASSIVE, np.uint8),
                   sigma_l=sig, sigma_t=sig, scale=np.array([1.0, 3.0]), dt=0.01)
    s = oracle_lib.Sim(w)
    v = np.array([1.0, 0.0])
    vol, S, nbr = s.geometry()
    assert np.allclose(vol, 1.0 / 6.0, rtol=1e-15)
    assert np.allclose(s.node_values(v), [1.0, p, p, q, 0.0], rtol=1e-14)
    g = s.gradients(v)
    assert np.allclose(g[0], [p - 1, p - 1, q - 1], rtol=1e-14)
    assert np.allclose(g[1], [-p, -p, q - 2 * p], rtol=1e-14)
    L = s.apply_diffusion(v)
    assert math.isclose(L[0], LA, rel_tol=1e-13), (L[0], LA)
    assert math.isclose(L[1], -LA, rel_tol=1e-13)
    # the swapped reading gives a value the tolerance above excludes
    swapped = 6.0 * (4.0 - s3) * sig * ((q - aB - 2.0 * p * aA) / 2.0 - 2.0) / (CHI * CM)
    assert abs(swapped - LA) > 1e-3 * abs(LA)
