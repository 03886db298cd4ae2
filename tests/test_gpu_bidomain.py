"""GPU bidomain step (Sec. 3.1 eq. electro, Sec. 3.2 eq. electro2_3d and the
restarted GMRES solve) through the C ABI against the FP64 oracle.

Bars: with the elliptic solves converged to 1e-12 (relative residual), the
transmembrane and extracellular potentials agree with the oracle's within
1e-6 mV; proportional tensors reproduce the GPU monodomain step with
M = lambda M_i / (1 + lambda) within 1e-8 mV.
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


def slab(n_steps=300, tol=1e-12, **kw):
    w = M.config1(nx=10, ny=6, nz=2, n_steps=n_steps)
    rng = np.random.default_rng(7)
    f = rng.normal(size=(w.n_tets, 3))
    w.fibre = f / np.linalg.norm(f, axis=1, keepdims=True)
    w.bidomain = M.Bidomain(tol=tol, **kw)
    return w


@pytest.mark.parametrize("restart", [20, 40])
def test_bidomain_fp64_parity(ep, oracle_lib, restart):
    """Both variants of the Arnoldi step against the oracle's plain GMRES:
    GMRES(20) on this small grid sums the Gram-Schmidt rows inside their
    consumer kernels (32 basis rows per pass), GMRES(40) (more rows than one
    pass holds) takes the separate row-sum kernels and 8-row passes."""
    w = slab(restart=restart)
    say(f"bidomain parity: {w.n_tets} tets, random fibres, GMRES({restart}) to 1e-12")
    g = ep.Sim(w, prec=ep.EP_FP64)
    o = oracle_lib.Sim(w)
    for chunk in range(3):
        g.step(100)
        o.step(100)
        dv = np.abs(g.vm() - o.vm()).max()
        dp = np.abs(g.phi_e() - o.phi_e()).max()
        say(f"  step {100 * (chunk + 1)}: max|dv| {dv:.2e}, max|dphi_e| {dp:.2e} mV, "
            f"GMRES steps gpu {g.bidomain_stats()[0]} oracle {o.bidomain_iterations()[0]}")
        assert dv <= TOL_MV and dp <= TOL_MV
    assert np.array_equal(np.isnan(g.activation()), np.isnan(o.activation()))
    assert np.nanmax(np.abs(g.activation() - o.activation())) <= 1e-6
    last, total, rr = g.bidomain_stats()
    assert last > 0 and total >= 300 and rr <= 1e-12
    assert np.abs(o.phi_e()).max() > 1.0            # a real extracellular field


def test_bidomain_proportional_is_monodomain(ep):
    lam = 2.0
    wb = M.config1(nx=10, ny=6, nz=2, n_steps=300)
    wb.bidomain = M.Bidomain(sigma_el=lam * 0.17, sigma_et=lam * 0.019, tol=1e-12)
    wm = M.config1(nx=10, ny=6, nz=2, n_steps=300)
    wm.sigma_l, wm.sigma_t = lam * 0.17 / (1 + lam), lam * 0.019 / (1 + lam)
    b, m = ep.Sim(wb, prec=ep.EP_FP64), ep.Sim(wm, prec=ep.EP_FP64)
    b.step(300)
    m.step(300)
    assert np.abs(b.vm() - m.vm()).max() < 1e-8


def test_bidomain_checkpoint_and_errors(ep):
    w = slab(n_steps=200, tol=1e-10)
    a = ep.Sim(w, prec=ep.EP_FP64)
    a.step(80)
    blob = a.checkpoint()
    a.step(40)
    c = ep.Sim(w, prec=ep.EP_FP64)
    c.restore(blob)
    c.step(40)
    assert np.array_equal(a.vm(), c.vm())
    assert np.array_equal(a.phi_e(), c.phi_e())
    with pytest.raises(ep.EPError) as e:
        ep.Sim(w, prec=ep.EP_FP32_MIXED)
    assert e.value.status == ep.EP_EINVAL
    mono = ep.Sim(M.config1(nx=4, ny=4, nz=2))
    with pytest.raises(ep.EPError) as e:
        mono.phi_e()
    assert e.value.status == ep.EP_ESTATE
    # the solver's state is staged in LDS: restarts up to 64
    for restart, ok in ((64, True), (65, False)):
        x = slab(n_steps=10, restart=restart)
        if ok:
            s = ep.Sim(x, prec=ep.EP_FP64)
            s.step(3)
            assert np.isfinite(s.phi_e()).all()
        else:
            with pytest.raises(ep.EPError) as e:
                ep.Sim(x, prec=ep.EP_FP64)
            assert e.value.status == ep.EP_EINVAL
