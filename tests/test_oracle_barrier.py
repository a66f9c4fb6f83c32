"""Internal walls (tagged faces) in the oracle: a closed wall splits the
basin into two that exchange nothing, so the undisturbed one stays at rest
and each keeps its own mass; with an opening, water reaches the other side
and the total mass is conserved."""
from __future__ import annotations

import numpy as np

import workloads as W
from helpers import oracle_solver


def _halves(o):
    xc = o.mesh.x.mean(axis=1)
    return xc < 0.5, xc > 0.5


def _mass(o, sel):
    return float(np.sum(o.mesh.J[sel] * (o.q[0][sel] @ o.ref.w)))


def test_closed_wall_separates_basins():
    wl = W.barrier_basin(n=8, N=3, gap=(2.0, 2.0))   # no opening
    o = oracle_solver(wl)
    left, right = _halves(o)
    m_left, m_right = _mass(o, left), _mass(o, right)
    o.run(40)
    assert np.max(np.abs(o.q[0][right] - 1.0)) <= 1e-12
    assert np.max(np.abs(o.q[1][right])) <= 1e-12 and np.max(np.abs(o.q[2][right])) <= 1e-12
    assert abs(_mass(o, left) - m_left) <= 1e-12 * m_left
    assert abs(_mass(o, right) - m_right) <= 1e-12 * m_right
    # the disturbed side did move
    assert np.max(np.abs(o.q[1][left])) > 1e-3


def test_opening_lets_water_through():
    wl = W.barrier_basin(n=8, N=3)
    o = oracle_solver(wl)
    left, right = _halves(o)
    m0 = o.mass()
    o.run(60)
    assert np.max(np.abs(o.q[0][right] - 1.0)) > 1e-5   # the wave passed the opening
    assert abs(o.mass() - m0) <= 1e-12 * m0
