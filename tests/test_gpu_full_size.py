"""The HIP path at the full sizes of the multi-rate and precision workloads
against stored FP64 oracle states of 1024 sampled elements (written by
tests/golden/make_golden.py, which calls only the oracle):

* C4, 1048576 triangles at N = 5, fully wet, its configured 300 steps on
  every contraction engine -- the precision study: plain FP32, fused FP32,
  FP32 matrix cores, and the two- and three-part BF16 splits, each reported
  as relative L2 against the oracle;
* C3, the 496098-triangle graded band mesh with four multi-rate levels, its
  configured 100 coarse steps (800 ticks), levels compared bit for bit;
* C5 with the over-integrated operators (the paper's cubature and Gauss
  rules), all 64 instances for their 200 steps against the oracle run with
  the same rules (64 sampled elements per instance).

The launch shape is the one bench.py times (the autotuner's choice)."""
from __future__ import annotations

import os

import numpy as np
import pytest

import workloads as W
from helpers import gpu_solver, log

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
# two-part BF16 split: three products of up to 3 * 2^-16 relative error each
BF16_TOL = 5e-5


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle_samples.npz")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle samples for {name} not generated")
    return np.load(path)


def _compare(g, z):
    h, hu, hv = g.get_state(0)
    idx = z["elements"]
    M, J = z["mass_matrix"], z["J"]

    def nrm(a):
        return float(np.sum(J * np.einsum("ki,ij,kj->k", a, M, a)))

    eh = np.sqrt(nrm(h[idx] - z["h"]) / nrm(z["h"]))
    em = np.sqrt((nrm(hu[idx] - z["hu"]) + nrm(hv[idx] - z["hv"])) / (nrm(z["hu"]) + nrm(z["hv"])))
    flags = g.flags(0)[idx]
    flips = int(np.sum((flags & 3) != z["final_pp"])) + int(np.sum(((flags >> 2) & 3) != z["final_tvb"]))
    return eh, em, flips


@pytest.mark.parametrize("path", ["plain_fp32", "fused_fp32", "fused_mfma32", "fused_bf16x3", "fused_bf16x6"])
def test_c4_precision_study_300_steps(path):
    _require_gpu()
    z = _golden("c4")
    wl = W.c4()
    log(f"[c4-300] K={wl.n_elements} N=5 path={path}")
    g = gpu_solver(wl, precision=path)
    g.prepare()
    if path != "plain_fp32":
        g.autotune(reps=3)
    _, dt = g.levels(0)
    assert abs(dt - float(z["dt"])) <= 1e-12 * float(z["dt"])
    g.advance(int(z["steps"]))
    eh, em, flips = _compare(g, z)
    d = g.diagnostics(0)
    log(f"[c4-300] {path} relL2 h={eh:.3e} m={em:.3e} flips={flips} mass gpu={d['mass']:.12e} "
        f"oracle={float(z['mass']):.12e}")
    tol = BF16_TOL if path == "fused_bf16x3" else 1e-5
    assert eh <= tol and em <= tol
    assert flips == 0
    assert abs(d["mass"] - float(z["mass"])) <= 1e-6 * float(z["mass"])


@pytest.mark.parametrize("path", ["fused_fp32", "fused_mfma32"])
def test_c3_multirate_full_size(path):
    _require_gpu()
    z = _golden("c3")
    wl = W.c3()
    log(f"[c3-full] K={wl.n_elements} levels={wl.max_levels} path={path}")
    g = gpu_solver(wl, precision=path)
    g.prepare()
    g.autotune(reps=3)
    lev, dt = g.levels(0)
    assert np.array_equal(lev.astype(int), z["levels"].astype(int))
    assert abs(dt - float(z["dt"])) <= 1e-12 * float(z["dt"])
    g.advance(int(z["steps"]))
    eh, em, flips = _compare(g, z)
    d = g.diagnostics(0)
    log(f"[c3-full] {path} relL2 h={eh:.3e} m={em:.3e} flips={flips} mass gpu={d['mass']:.12e} "
        f"oracle={float(z['mass']):.12e}")
    assert eh <= 1e-5 and em <= 1e-5
    assert flips == 0
    assert abs(d["mass"] - float(z["mass"])) <= 1e-6 * float(z["mass"])


@pytest.mark.parametrize("path", ["fused_fp32", "fused_mfma32"])
def test_c5_overint_full_size(path):
    _require_gpu()
    z = _golden("c5_overint")
    wl = W.c5()
    Ks = [i.etov.shape[0] for i in wl.instances]
    log(f"[c5-overint] K={sum(Ks)} path={path}")
    g = gpu_solver(wl, precision=path, overint=1)
    g.prepare()
    g.advance(int(z["steps"]))
    M = z["mass_matrix"]
    worst_h = worst_m = 0.0
    flips = 0
    for i in range(len(Ks)):
        idx, J = z["elements"][i], z["J"][i]
        h, hu, hv = g.get_state(i)

        def nrm(a):
            return float(np.sum(J * np.einsum("ki,ij,kj->k", a, M, a)))

        eh = np.sqrt(nrm(h[idx] - z["h"][i]) / nrm(z["h"][i]))
        em = np.sqrt((nrm(hu[idx] - z["hu"][i]) + nrm(hv[idx] - z["hv"][i])) /
                     (nrm(z["hu"][i]) + nrm(z["hv"][i])))
        f = g.flags(i)[idx]
        flips += int(np.sum((f & 3) != z["final_pp"][i])) + int(np.sum(((f >> 2) & 3) != z["final_tvb"][i]))
        worst_h, worst_m = max(worst_h, eh), max(worst_m, em)
        d = g.diagnostics(i)
        assert d["min_depth"] >= 0.0
        assert abs(d["mass"] - float(z["mass"][i])) <= 1e-6 * float(z["mass"][i])
        assert eh <= 1e-5 and em <= 1e-5, (i, Ks[i], eh, em)
    log(f"[c5-overint] {path} 64 instances worst relL2 h={worst_h:.3e} m={worst_m:.3e} flips={flips}")
    assert flips <= 0.01 * z["elements"].size
