"""Pins of the oracle's bidomain step (Sec. 3.1 eq. electro, Sec. 3.2
eq. electro2_3d and the restarted GMRES solve of the extracellular potential).

* Proportional tensors (M_e = lambda M_i) reduce the bidomain model to the
  monodomain one with M = lambda M_i / (1 + lambda) (the paper's
  eq. electro2_3dmono); the discrete operator is linear in M, so the reduction
  holds step by step up to the solver tolerance, with
  phi_e = -v / (1 + lambda) + const.
* GMRES against a dense least-squares solve of the assembled operator.
* Charge conservation of the coupled flux, and the elliptic residual.
* With unequal anisotropy ratios the monodomain model with half the harmonic
  mean of the two conductivities approximates the bidomain activation
  (Sec. 1).
"""
import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M


def zero_mean(x, vol):
    return x - (vol * x).sum() / vol.sum()


@pytest.mark.parametrize("lam", [2.0, 0.5])
def test_proportional_tensors_reduce_to_monodomain(oracle_lib, lam):
    wb = M.config1(nx=10, ny=6, nz=2, n_steps=300)
    wb.fibre = np.tile([0.6, 0.8, 0.0], (wb.n_tets, 1))
    wb.bidomain = M.Bidomain(sigma_el=lam * 0.17, sigma_et=lam * 0.019, tol=1e-12)
    wm = M.config1(nx=10, ny=6, nz=2, n_steps=300)
    wm.fibre = wb.fibre
    wm.sigma_l, wm.sigma_t = lam * 0.17 / (1 + lam), lam * 0.019 / (1 + lam)
    b, m = oracle_lib.Sim(wb), oracle_lib.Sim(wm)
    b.step(300)
    m.step(300)
    assert np.abs(b.vm() - m.vm()).max() < 1e-8     # solver tolerance 1e-12, 300 steps
    vol, _, _ = b.geometry()
    phi = b.phi_e()
    np.testing.assert_allclose(phi, zero_mean(-b.vm() / (1 + lam), vol), atol=1e-8)
    assert abs((vol * phi).sum()) < 1e-9 * vol.sum()


def test_gmres_matches_dense_solve(oracle_lib):
    """Tiny mesh: assemble the flux operator from unit vectors, solve with
    dense least squares (minimum norm) and compare with restarted GMRES
    (restart 4, so restarts happen) up to the constant null space."""
    w = M.config1(nx=3, ny=2, nz=1)
    rng = np.random.default_rng(3)
    w.fibre = rng.normal(size=(w.n_tets, 3))
    w.fibre /= np.linalg.norm(w.fibre, axis=1, keepdims=True)
    s = oracle_lib.Sim(w)
    n = w.n_tets
    sl, st = 0.79, 0.259
    A = np.column_stack([s.apply_flux(np.eye(n)[k], sl, st) for k in range(n)])
    x_true = rng.normal(size=n)
    b = A @ x_true
    x, it, rr = s.gmres(b, np.zeros(n), sl, st, restart=4, tol=1e-12, max_iter=5000)
    assert rr <= 1e-12 and it > 4
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    np.testing.assert_allclose(x - x.mean(), ref - ref.mean(), atol=1e-8)
    # the operator annihilates constants and its columns sum to zero
    assert np.abs(A @ np.ones(n)).max() < 1e-12
    assert np.abs(A.sum(axis=0)).max() < 1e-12


def test_gmres_iteration_cap(oracle_lib):
    w = M.config1(nx=6, ny=4, nz=2)
    s = oracle_lib.Sim(w)
    rng = np.random.default_rng(1)
    b = s.apply_flux(rng.normal(size=w.n_tets), 0.79, 0.259)
    _, it, rr = s.gmres(b, np.zeros(w.n_tets), 0.79, 0.259, restart=5, tol=1e-30, max_iter=17)
    assert it == 17 and rr > 1e-30


def test_bidomain_charge_and_elliptic_residual(oracle_lib):
    """Passive cells and a stimulus pulse: the coupled flux moves no charge,
    sum_c V_c (v_c - v_0) = -amp dur sum_stim V_c; after each step phi_e
    solves the elliptic equation to the tolerance and has zero mean."""
    w = M.config1(nx=8, ny=6, nz=2, n_steps=100)
    w.model = np.full(w.n_tets, M.PASSIVE, np.uint8)
    w.stimuli = [M.Stimulus(ids=np.arange(0, 40, dtype=np.int32), t0=0.0, dur=0.2, amp=-30.0)]
    w.bidomain = M.Bidomain(tol=1e-11)
    s = oracle_lib.Sim(w)
    vol, _, _ = s.geometry()
    v0 = s.vm()
    s.step(50)
    v = s.vm()
    q = (vol * (v - v0)).sum()
    assert q == pytest.approx(30.0 * 0.2 * vol[:40].sum(), rel=1e-10)
    phi = s.phi_e()
    rhs = -s.apply_flux(v, 0.17, 0.019)
    res = s.apply_flux(phi, 0.17 + 0.62, 0.019 + 0.24) - rhs
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(rhs)
    assert abs((vol * phi).sum()) < 1e-9 * vol.sum()
    last, total, rr = s.bidomain_iterations()
    assert last > 0 and total >= last and rr <= 1e-11


def test_half_harmonic_mean_monodomain_approximates_bidomain(oracle_lib):
    """Unequal anisotropy (the paper's Niederer conductivities): the
    monodomain model with sigma = sigma_i sigma_e / (sigma_i + sigma_e) per
    direction activates a fibre-aligned slab within 10 % of the bidomain
    activation times (Sec. 1 recommends this approximation)."""
    def slab(bido):
        w = M.config1(nx=24, ny=4, nz=2, n_steps=900)
        if bido:
            w.bidomain = M.Bidomain(tol=1e-6)
        else:
            w.sigma_l = 0.17 * 0.62 / (0.17 + 0.62)
            w.sigma_t = 0.019 * 0.24 / (0.019 + 0.24)
        return w
    res = []
    for bido in (True, False):
        w = slab(bido)
        s = oracle_lib.Sim(w)
        s.step(w.n_steps)
        res.append(s.activation())
    far = M.hex_box_ids(slab(False).hex_ijk, (16, None, None), (17, None, None))
    tb, tm = res[0][far], res[1][far]
    assert np.isfinite(tb).all() and np.isfinite(tm).all()
    assert np.abs(tm / tb - 1).max() < 0.10
