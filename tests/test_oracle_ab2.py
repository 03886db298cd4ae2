"""The Adams-Bashforth alternative for the non-gating states (Sec. 4: the
paper's scheme is Rush-Larsen for the gates and forward Euler for the rest;
a second-order Adams-Bashforth step for the non-gating variables lowers the
time error, while the gates keep Rush-Larsen's first order).

Pins: the graph update equals the textbook AB2 recursion of the Neumann
finite-difference Laplacian (forward Euler on the first substep); on passive
tissue AB2 converges with order 2 in time where forward Euler has order 1;
on the paper's TP06 box AB2 is closer to the converged mean potential than
forward Euler at the same step.
"""
import math

import numpy as np
import pytest

from paper_2112_12854_amd import meshgen as M
from test_oracle_purkinje import CHI_CM, chain_workload


def test_graph_ab2_matches_textbook_recursion(oracle_lib):
    n, L, dt = 25, 0.1, 0.02
    w = chain_workload(n, L, model=M.PASSIVE, stim_nodes=[7], stim_amp=-40.0, stim_dur=0.1,
                       dt=dt)
    w.time_scheme = 1
    s = oracle_lib.Sim(w)
    nsub = s.purkinje_n_sub()
    dtp = dt / nsub
    A = np.zeros((n, n))
    for i in range(1, n - 1):
        A[i, i - 1], A[i, i], A[i, i + 1] = 1.0, -2.0, 1.0
    A[0, 0], A[0, 1] = -2.0, 2.0
    A[-1, -1], A[-1, -2] = -2.0, 2.0
    A *= 3.95 / (CHI_CM * L * L)
    v = s.purkinje_vm().copy()
    nstim = int(round(0.1 / dt))
    prev = None
    for step in range(40):
        for _ in range(nsub):
            ist = np.zeros(n)
            if step < nstim:
                ist[7] = -40.0
            F = A @ v - ist
            v = v + dtp * (F if prev is None else 1.5 * F - 0.5 * prev)
            prev = F
    s.step(40)
    np.testing.assert_allclose(s.purkinje_vm(), v, rtol=0, atol=1e-10)


def passive_mode(oracle_lib, dt, scheme, t_end=2.0):
    """Passive slab started from a smooth potential (a cosine along the
    fibres), no stimulus: a linear system whose only error is the time
    discretisation's."""
    w = M.config1(n_steps=0)
    w.model = np.full(w.n_tets, M.PASSIVE, np.uint8)
    w.stimuli = []
    w.dt = dt
    w.time_scheme = scheme
    s = oracle_lib.Sim(w)
    st = s.states()
    x = w.xyz[w.tets].mean(axis=1)[:, 0]
    st[0] = -80.0 + 20.0 * np.cos(np.pi * x / 10.0)
    s.set_states(st)
    s.step(int(round(t_end / dt)))
    return s.vm()


@pytest.mark.parametrize("scheme,order", [(0, 1.0), (1, 2.0)])
def test_passive_time_order(oracle_lib, scheme, order):
    v = [passive_mode(oracle_lib, dt, scheme) for dt in (0.01, 0.005, 0.0025)]
    e1 = np.abs(v[0] - v[1]).max()
    e2 = np.abs(v[1] - v[2]).max()
    p = math.log2(e1 / e2)
    assert abs(p - order) < 0.15, p


def vbar_at(oracle_lib, dt, scheme, t_end=50.0):
    w = M.niederer_box(h=1.0, dt=dt, n_steps=int(round(t_end / dt)))
    w.time_scheme = scheme
    s = oracle_lib.Sim(w)
    s.step(w.n_steps)
    return s.mean_vm()


def test_ab2_reduces_the_time_error_on_the_tp06_box(oracle_lib):
    """Reference: Richardson extrapolation of the first-order scheme,
    2 v(dt/2) - v(dt); AB2 at dt = 0.005 ms is closer to it than forward
    Euler at the same step (the paper's observation for its 1D case;
    observed: 0.54 of the forward-Euler error, the gates keeping their
    first-order part)."""
    fe1 = vbar_at(oracle_lib, 0.005, 0)
    fe2 = vbar_at(oracle_lib, 0.0025, 0)
    ref = 2.0 * fe2 - fe1
    ab = vbar_at(oracle_lib, 0.005, 1)
    assert abs(ab - ref) < 0.75 * abs(fe1 - ref), (ab, fe1, ref)


def test_second_order_rush_larsen_is_second_order(oracle_lib):
    """Sec. 4: with the non-gating states by AB2, a modified second-order
    Rush-Larsen step makes the whole scheme second order.  On the paper's
    TP06 box the mean potential at 50 ms converges with observed order
    2 (1.7 .. 2.3; observed 1.86) from dt = 0.01, 0.005, 0.0025 ms, against
    1.13 for the paper's scheme and 1.43 with AB2 alone."""
    v = [vbar_at(oracle_lib, dt, 2) for dt in (0.01, 0.005, 0.0025)]
    p = math.log2((v[0] - v[1]) / (v[1] - v[2]))
    assert 1.7 <= p <= 2.3, p
