"""Shared drivers for the parity tests: the same seeded workload run through
the FP64 oracle and through the HIP library (C ABI), each evaluating the
analytic inputs at its own nodes."""
from __future__ import annotations

import sys
import time

import numpy as np

from oracle.swe import Params, Solver as OracleSolver


def oracle_solver(wl, inst=0, **kw):
    ins = wl.instances[inst]
    p = Params(g=wl.g, cfl=kw.pop("cfl", wl.cfl), max_levels=kw.pop("max_levels", wl.max_levels), **kw)
    s = OracleSolver(ins.vx, ins.vy, ins.etov, wl.N, p, bc=ins.bc)
    x, y = s.nodes()
    B = s.interpolate(ins.bathymetry)
    h, hu, hv = ins.initial(x, y)
    s.set_state(h, hu, hv, B)
    return s


def gpu_solver(wl, precision="fused_fp32", insts=None, **kw):
    from paper_1403_1661_amd import dgswe
    insts = list(range(len(wl.instances))) if insts is None else insts
    meshes = [(wl.instances[i].vx, wl.instances[i].vy, wl.instances[i].etov, wl.instances[i].bc) for i in insts]
    params = dict(g=wl.g, cfl=wl.cfl, max_levels=wl.max_levels, precision=precision)
    params.update(kw)
    s = dgswe.Solver(meshes, wl.N, **params)
    s.bind("cuda:0")
    for j, i in enumerate(insts):
        ins = wl.instances[i]
        x, y = s.node_coords(j)
        B = ins.bathymetry(x, y)
        s.set_bathymetry(j, B)
        h, hu, hv = ins.initial(x, y)
        s.set_state(j, h, hu, hv)
    return s


def closed_form_params(wl):
    """Solver parameters of a closed-form case: its desingularisation depth
    and whether the TVB limiter runs."""
    return {"hvel": wl.extra["hvel"], "tvb": wl.extra.get("tvb", True)}


def closed_form_oracle(wl):
    """Oracle on a closed-form case, started from the exact state at t0 (the
    instance's initial function)."""
    p = closed_form_params(wl)
    return oracle_solver(wl, hvel=p["hvel"], tvb=p["tvb"])


def closed_form_gpu(wl, precision="fused_fp32", **kw):
    from paper_1403_1661_amd import dgswe
    p = closed_form_params(wl)
    mask = dgswe.DG_LIMIT_PP | (dgswe.DG_LIMIT_TVB if p["tvb"] else 0)
    return gpu_solver(wl, precision=precision, hvel=p["hvel"], limiter_mask=mask, **kw)


def exact_errors(osolver, h, wl, t, region=None):
    """L2 error of the depth against the closed form at time t, relative to
    the L2 norm of the exact depth (nodal values, element mass matrices);
    with a region mask (elements), also over those elements only."""
    x, y = osolver.nodes()
    he = wl.extra["exact"](x, y, t)[0]
    M, J = osolver.ref.M, osolver.mesh.J
    e = np.asarray(h) - he
    w = J * np.einsum("ki,ij,kj->k", e, M, e)
    nrm = np.sqrt(float(np.sum(J * np.einsum("ki,ij,kj->k", he, M, he))))
    out = {"rel": np.sqrt(float(np.sum(w))) / nrm}
    if region is not None:
        out["local"] = np.sqrt(float(np.sum(w[region]))) / nrm
    return out


def rel_l2(osolver, q_test, q_ref):
    """Relative L2 of depth and of the momentum pair (absolute when the
    reference norm is below 1e-8)."""
    M = osolver.ref.M
    J = osolver.mesh.J

    def norm2(a):
        return float(np.sum(J * np.einsum("ki,ij,kj->k", a, M, a)))

    out = {}
    for name, fields in (("h", (0,)), ("m", (1, 2))):
        num = sum(norm2(q_test[c] - q_ref[c]) for c in fields)
        den = sum(norm2(q_ref[c]) for c in fields)
        out[name] = np.sqrt(num) / np.sqrt(den) if den > 1e-16 else np.sqrt(num)
    return out


def flag_flips(gpu_flags, oracle_flags):
    pp = int(np.sum((gpu_flags & 3) != oracle_flags.pp))
    tv = int(np.sum(((gpu_flags >> 2) & 3) != oracle_flags.tvb))
    return pp, tv


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Timer:
    def __enter__(self):
        self.t = time.time()
        return self

    def __exit__(self, *exc):
        self.dt = time.time() - self.t
