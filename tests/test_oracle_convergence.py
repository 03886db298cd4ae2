"""Temporal convergence of the oracle's explicit step (Sec. 4: the scheme is
first order in time; Rush-Larsen and forward Euler are both order 1).

The paper's box (20 x 7 x 3 mm, fibres along x, TP06, 1.5 mm corner
stimulus) at h = 1 mm; the mean potential at 50 ms for dt = 0.01, 0.005 and
0.0025 ms.  The observed order from three successive halvings,
p = log2((v(4h) - v(2h)) / (v(2h) - v(h))), needs no reference solution.
"""
import math

from paper_2112_12854_amd import meshgen as M


def vbar_at(oracle_lib, dt, t_end=50.0):
    w = M.niederer_box(h=1.0, dt=dt, n_steps=int(round(t_end / dt)))
    s = oracle_lib.Sim(w)
    s.step(w.n_steps)
    return s.mean_vm()


def test_first_order_in_time(oracle_lib):
    v = [vbar_at(oracle_lib, dt) for dt in (0.01, 0.005, 0.0025)]
    p = math.log2((v[0] - v[1]) / (v[1] - v[2]))
    assert 0.8 <= p <= 1.2, p
    # monotone approach: the error halves in the same direction
    assert (v[0] - v[1]) * (v[1] - v[2]) > 0
