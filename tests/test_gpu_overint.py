"""The over-integrated weak form on the GPU (Section 3, Eq. 3.2 with the
cubature and Gauss rules; Section 7, Volume and Surface kernels) against the
FP64 oracle run with the same rules (parameter overint): the right-hand
side R = Pr cF1 + Ps cF2 + P cS - L^g Fn* on the vector-ALU kernel, followed
by the same update and limiters as the nodal path.  Tolerance: relative L2
of depth and momentum <= 1e-5; limiter flips counted and bounded.  The
right-hand side runs on the vector ALU (plain_fp32, fused_fp32) or with its
contractions on the matrix cores (fused_mfma32)."""
import numpy as np
import pytest

import workloads as W
from helpers import flag_flips, gpu_solver, log, oracle_solver, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
PATHS = ["plain_fp32", "fused_fp32", "fused_mfma32"]
# vector-ALU and matrix-core right-hand-side kernels
ENGINES = ["fused_fp32", "fused_mfma32"]


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _compare(tag, wl, steps, path="fused_fp32", flip_frac=0.01, **kw):
    _require_gpu()
    log(f"[oi-{tag}] K={wl.n_elements} N={wl.N} steps={steps} path={path}")
    o = oracle_solver(wl, overint=True, **kw)
    g = gpu_solver(wl, precision=path, overint=1, **kw)
    _, dt = g.levels(0)
    assert abs(dt - o.dt_min) <= 1e-12 * o.dt_min
    g.advance(steps)
    o.run(steps)
    q = np.stack(g.get_state(0))
    err = rel_l2(o, q, o.q)
    pp, tv = flag_flips(g.flags(0), o.flags)
    d = g.diagnostics(0)
    log(f"[oi-{tag}] relL2 h={err['h']:.3e} m={err['m']:.3e} flips pp={pp} tvb={tv} "
        f"mass gpu={d['mass']:.12e} oracle={o.mass():.12e}")
    assert err["h"] <= TOL and err["m"] <= TOL, err
    assert pp + tv <= flip_frac * wl.n_elements
    assert abs(d["mass"] - o.mass()) <= 1e-6 * o.mass()
    return g, o


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("path", PATHS)
def test_overint_lake_at_rest_bitwise(path, N):
    """Still water over a smooth bed and over a bed that jumps across every
    face stays bitwise at rest (perturbation form: every term is zero)."""
    _require_gpu()
    for wl in (W.lake_at_rest(n=6, N=N), W.stepped_bed("lake", N=N)):
        log(f"[oi-lake] {wl.name} N={N} path={path}")
        g = gpu_solver(wl, precision=path, overint=1)
        g.prepare()
        h0 = g.get_state(0)[0]
        g.advance(60)
        h1, hu1, hv1 = g.get_state(0)
        assert np.array_equal(h0, h1)
        assert np.all(hu1 == 0.0) and np.all(hv1 == 0.0)


@pytest.mark.parametrize("path", PATHS)
def test_overint_c1_trajectory(path):
    _compare("c1", W.c1(), 200, path=path)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("path", ENGINES)
def test_overint_wetdry_orders(path, N):
    g, o = _compare(f"wetdry-N{N}-{path}", W.small_wetdry(n=12, N=N), 60, path=path)
    assert g.diagnostics(0)["min_depth"] >= 0.0


@pytest.mark.parametrize("case", ["dam", "ledge"])
@pytest.mark.parametrize("N", [1, 3, 5])
@pytest.mark.parametrize("path", ENGINES)
def test_overint_stepped_bed(path, case, N):
    wl = W.stepped_bed(case, N=N)
    g, o = _compare(f"stepped-{case}-N{N}-{path}", wl, wl.steps, path=path)
    assert g.diagnostics(0)["min_depth"] >= 0.0


@pytest.mark.parametrize("N", [1, 3])
@pytest.mark.parametrize("path", ENGINES)
def test_overint_multirate_wetdry(path, N):
    """Multi-rate AB3 (the graded beach, four levels): coarser inactive
    neighbours supply their half-step face traces, interpolated to the Gauss
    points like the current traces."""
    g, o = _compare(f"mrab-N{N}-{path}", W.graded_beach(N=N), 10, path=path)
    lev, _ = g.levels(0)
    assert np.array_equal(lev.astype(int), o.levels)


@pytest.mark.parametrize("path", ENGINES)
def test_overint_reduced_c4(path):
    """The N = 5 precision workload (16 Fourier modes, fully wet) on a
    128x64x2 mesh, 30 steps."""
    _compare(f"c4-reduced-{path}", W.c4(nx=128, ny=64), 30, path=path)


@pytest.mark.parametrize("path", ENGINES)
def test_overint_ensemble(path):
    _require_gpu()
    wl = W.c5(n_inst=3, kmin=400, kmax=3000)
    log(f"[oi-ensemble] {path}")
    g = gpu_solver(wl, precision=path, overint=1)
    g.advance(40)
    for i in range(3):
        o = oracle_solver(wl, inst=i, overint=True)
        o.run(40)
        err = rel_l2(o, np.stack(g.get_state(i)), o.q)
        log(f"[oi-ensemble] inst {i} relL2 h={err['h']:.3e} m={err['m']:.3e}")
        assert err["h"] <= TOL and err["m"] <= TOL
