"""Beds that jump across faces on the GPU (Section 5.1, Eq. 5.1-5.2): every
element of a jittered 8x8x2 unit square carries its own bed piece
(0.1 x + 0.04 r_k, plus a step), so B- != B+ at every face node and the
hydrostatic reconstruction h* = max(0, eta - max(B-, B+)) and the pressure
correction of the well-balanced flux are exercised at every face.  The beds
are plain FP64 values handed to dg_set_bathymetry.

* lake at rest over the stepped bed: bitwise steady on the GPU;
* a dam (surface step) over the stepped bed: parity with the FP64 oracle;
* a ledge whose dry elements' bed rises above the wet neighbours' surface,
  with a hump running into it: parity with the oracle, positivity codes
  compared element by element."""
import numpy as np
import pytest

import workloads as W
from helpers import flag_flips, gpu_solver, log, oracle_solver, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
PATHS = ["plain_fp32", "fused_fp32", "fused_mfma32"]


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("path", PATHS)
def test_stepped_lake_bitwise_steady(path, N):
    _require_gpu()
    wl = W.stepped_bed("lake", N=N)
    log(f"[stepped-lake] N={N} path={path}")
    g = gpu_solver(wl, precision=path)
    g.prepare()
    h0 = g.get_state(0)[0]
    g.advance(100)
    h1, hu1, hv1 = g.get_state(0)
    assert np.array_equal(h0, h1)
    assert np.all(hu1 == 0.0) and np.all(hv1 == 0.0)


def _parity(case, N, path):
    _require_gpu()
    wl = W.stepped_bed(case, N=N)
    log(f"[stepped-{case}] K={wl.n_elements} N={N} steps={wl.steps} path={path}")
    o = oracle_solver(wl)
    g = gpu_solver(wl, precision=path)
    _, dt = g.levels(0)
    assert abs(dt - o.dt_min) <= 1e-12 * o.dt_min
    g.advance(wl.steps)
    o.run(wl.steps)
    q = np.stack(g.get_state(0))
    err = rel_l2(o, q, o.q)
    pp, tv = flag_flips(g.flags(0), o.flags)
    d = g.diagnostics(0)
    log(f"[stepped-{case}] relL2 h={err['h']:.3e} m={err['m']:.3e} flips pp={pp} tvb={tv} "
        f"mass gpu={d['mass']:.12e} oracle={o.mass():.12e}")
    assert err["h"] <= TOL and err["m"] <= TOL, err
    assert abs(d["mass"] - o.mass()) <= 1e-6 * o.mass()
    return g, o, pp, tv


@pytest.mark.parametrize("N", [1, 3, 5])
@pytest.mark.parametrize("path", PATHS)
def test_stepped_dam_parity(path, N):
    g, o, pp, tv = _parity("dam", N, path)
    assert pp == 0 and tv == 0


@pytest.mark.parametrize("N", [1, 3, 5])
@pytest.mark.parametrize("path", PATHS)
def test_stepped_ledge_parity(path, N):
    g, o, pp, tv = _parity("ledge", N, path)
    assert pp == 0
    # the ledge is dry and stays dry: the reconstruction turned its faces into walls
    assert np.sum(o.flags.pp == 2) > 0
    assert g.diagnostics(0)["min_depth"] >= 0.0
