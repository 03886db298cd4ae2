"""Spatial convergence on the paper's verification box (Sec. 4): 20 x 7 x 3
mm, fibres along x, TP06, the 1.5 mm corner-cube stimulus, dt = 0.005 ms,
grid spacings 0.5, 0.25, 0.2, 0.125 and 0.1 mm (the paper's three and two
in between), 50 ms of activity.  The fine grids need ~4e10 cell-steps, which
the oracle would take half an hour for, so the study runs on the FP64 GPU
path, anchored to the oracle on the coarsest grid.

Checked against the paper's statements:
* refining the grid speeds the front up: the far corner activates earlier
  and the mean potential at 50 ms rises, monotonically, on every refinement;
* the error of the mean potential at 50 ms, measured as the paper measures
  it (against the finest grid, at 0.5 and 0.2 mm), falls with order about 2
  (band 1.6-2.4).
"""
import math

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M

pytestmark = pytest.mark.gpu

DT = 0.005
T_END = 50.0
HS = (0.5, 0.25, 0.2, 0.125, 0.1)


@pytest.fixture(scope="module")
def ep():
    from paper_2112_12854_amd import ep as _ep
    _ep.lib()
    return _ep


def say(msg):
    print(msg, flush=True)


def volumes(w):
    p = w.xyz[w.tets]
    e1, e2, e3 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    return np.abs(np.einsum("ij,ij->i", e1, np.cross(e2, e3))) / 6.0


def far_corner_cell(w):
    c = w.xyz[w.tets].mean(axis=1)
    return int(np.argmin(np.sum((c - np.array([20.0, 7.0, 3.0])) ** 2, axis=1)))


@pytest.fixture(scope="module")
def study(ep):
    n = int(round(T_END / DT))
    out = {}
    for h in HS:
        w = M.niederer_box(h=h, dt=DT, n_steps=n)
        s = ep.Sim(w, prec=ep.EP_FP64)
        s.step(n)
        vol = volumes(w)
        v = s.vm()
        vbar = float(np.dot(vol, v) / vol.sum())
        t_far = float(s.activation()[far_corner_cell(w)])
        say(f"h {h}: {w.n_tets} tets, vbar(50 ms) {vbar:.6f} mV, far corner {t_far:.4f} ms")
        out[h] = (vbar, t_far, v if h == HS[0] else None)
        s.close()
    return out


def test_coarse_grid_equals_oracle(oracle_lib, study):
    w = M.niederer_box(h=HS[0], dt=DT, n_steps=int(round(T_END / DT)))
    o = oracle_lib.Sim(w)
    o.step(w.n_steps)
    assert np.max(np.abs(study[HS[0]][2] - o.vm())) <= 1e-6
    assert abs(study[HS[0]][0] - o.mean_vm()) <= 1e-9


def test_refinement_speeds_the_front_monotonically(study):
    vbar = [study[h][0] for h in HS]
    t_far = [study[h][1] for h in HS]
    assert all(np.isfinite(t_far))
    assert all(a > b for a, b in zip(t_far, t_far[1:])), t_far
    assert all(a < b for a, b in zip(vbar, vbar[1:])), vbar
    # successive changes shrink faster than the spacing
    d = np.diff(vbar)
    assert d[0] / (HS[0] - HS[1]) > d[2] / (HS[2] - HS[3])


def test_second_order_error_against_the_finest_grid(study):
    ref = study[0.1][0]
    e_coarse, e_fine = abs(study[0.5][0] - ref), abs(study[0.2][0] - ref)
    p = math.log(e_coarse / e_fine) / math.log(0.5 / 0.2)
    say(f"observed order against the 0.1 mm grid: {p:.2f}")
    assert 1.6 <= p <= 2.4, p
