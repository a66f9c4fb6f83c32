"""The optional thin-film rule (momentum set to zero after the limiters at
nodes thinner than thin_cut) in the oracle: still water with a shoreline
that crosses elements stays bounded with it, and the rule is exact where it
applies and absent when switched off."""
from __future__ import annotations

import warnings

import numpy as np

import workloads as W
from helpers import oracle_solver


def _run(o, steps):
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        o.run(steps)


def test_shoreline_lake_stays_bounded_with_thin_cut():
    wl = W.shoreline_lake(n=12, N=2)
    o = oracle_solver(wl, thin_cut=1e-3)
    m0 = o.mass()
    _run(o, 600)
    assert np.all(np.isfinite(o.q)) and o.q[0].min() >= 0.0
    assert np.max(np.abs(o.q[1:])) <= 1e-2          # spurious momentum stays small
    assert abs(o.mass() - m0) <= 1e-12 * m0
    thin = o.q[0] < 1e-3
    assert thin.any() and np.all(o.q[1][thin] == 0.0) and np.all(o.q[2][thin] == 0.0)


def test_thin_cut_off_is_the_default_scheme():
    wl = W.small_wetdry(n=8, N=3)
    a = oracle_solver(wl)
    b = oracle_solver(wl, thin_cut=0.0)
    _run(a, 20)
    _run(b, 20)
    assert np.array_equal(a.q, b.q)
