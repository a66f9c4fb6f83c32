"""Write stored oracle results used by the GPU parity tests and bench.py.

Calls only ``oracle/`` and ``workloads/``:

    python tests/golden/make_golden.py c2     # -> tests/golden/c2_oracle_samples.npz

c2: the 131072-triangle N=4 wet/dry workload run for its configured 500
single-rate AB3 steps by the FP64 oracle; stores the final depth and momenta
of 1024 elements drawn with numpy.random.default_rng(2024), the mass matrix,
the sampled elements' Jacobians, and the oracle's total mass and limiter
flag histograms.  Takes about 15 minutes on 8 cores.

c4: the 1048576-triangle N=5 fully wet precision workload for its
configured 300 steps (about 90 minutes on 8 cores, 11 GB); the same record
for 1024 sampled elements.

c3: the 496098-triangle graded band mesh with 4 multi-rate levels for its
configured 100 coarse steps (800 finest-level ticks); the same record plus
the level of every element.

c5: the 64-instance ensemble, every instance run by its own oracle (the
instances are independent, each with its own time step) for the configured
200 steps; 64 elements sampled from each instance (numpy.random.default_rng
seeded 2024 + instance number), with their final state, Jacobians, the
instance's mass and time step and the sampled elements' final limiter codes.
Runs the instances in a process pool (one BLAS thread each).

c5_overint: the same ensemble and record with the over-integrated weak form
(cubature and Gauss rules exact to degree 3N) instead of nodal collocation.

    python tests/golden/make_golden.py c3 c4 c5 c5_overint
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.swe import Params, Solver  # noqa: E402


def make_c2(n_samples=1024):
    wl = W.c2()
    ins = wl.instances[0]
    s = Solver(ins.vx, ins.vy, ins.etov, wl.N, Params(g=wl.g, cfl=wl.cfl))
    x, y = s.nodes()
    s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry))
    m0 = s.mass()
    t0 = time.time()
    for n in range(wl.steps):
        s.step()
        if n % 50 == 0:
            print(f"step {n} {time.time() - t0:.0f}s", flush=True)
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(s.K, size=n_samples, replace=False))
    pp = np.stack([fc[0] for fc in s.flag_counts])
    tv = np.stack([fc[1] for fc in s.flag_counts])
    out = os.path.join(HERE, "c2_oracle_samples.npz")
    np.savez_compressed(out, elements=idx, h=s.q[0][idx], hu=s.q[1][idx], hv=s.q[2][idx],
                        mass_matrix=s.ref.M, J=s.mesh.J[idx], steps=wl.steps, mass0=m0,
                        mass=s.mass(), dt=s.dt_min, pp_counts=pp, tvb_counts=tv,
                        final_pp=s.flags.pp, final_tvb=s.flags.tvb,
                        command="python tests/golden/make_golden.py c2")
    print("wrote", out, flush=True)


def make_sampled(name, wl, steps, n_samples=1024):
    """Run the oracle on a full-size workload and store 1024 sampled
    elements' final state (the c2 record without the flag histograms)."""
    ins = wl.instances[0]
    t0 = time.time()
    s = Solver(ins.vx, ins.vy, ins.etov, wl.N, Params(g=wl.g, cfl=wl.cfl, max_levels=wl.max_levels))
    x, y = s.nodes()
    s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry))
    print(f"{name}: K={s.K} setup {time.time() - t0:.0f}s dt={s.dt_min:.6e}", flush=True)
    m0 = s.mass()
    for n in range(steps):
        s.step() if wl.max_levels == 1 else s.run(1)
        if n % 10 == 0:
            print(f"{name}: step {n} {time.time() - t0:.0f}s", flush=True)
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(s.K, size=n_samples, replace=False))
    out = os.path.join(HERE, f"{name}_oracle_samples.npz")
    extra = {"levels": np.asarray(s.levels)} if wl.max_levels > 1 else {}
    np.savez_compressed(out, elements=idx, h=s.q[0][idx], hu=s.q[1][idx], hv=s.q[2][idx],
                        mass_matrix=s.ref.M, J=s.mesh.J[idx], steps=steps, mass0=m0,
                        mass=s.mass(), dt=s.dt_min, final_pp=s.flags.pp[idx],
                        final_tvb=s.flags.tvb[idx],
                        command=f"python tests/golden/make_golden.py {name}", **extra)
    print("wrote", out, f"{time.time() - t0:.0f}s", flush=True)


def _c5_instance(args):
    i, n_samples, overint = args
    wl = W.c5()
    ins = wl.instances[i]
    s = Solver(ins.vx, ins.vy, ins.etov, wl.N, Params(g=wl.g, cfl=wl.cfl, overint=overint))
    x, y = s.nodes()
    s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry))
    m0 = s.mass()
    t0 = time.time()
    for _ in range(wl.steps):
        s.step()
    rng = np.random.default_rng(2024 + i)
    idx = np.sort(rng.choice(s.K, size=min(n_samples, s.K), replace=False))
    print(f"c5[{i}] K={s.K} {wl.steps} steps {time.time() - t0:.0f}s", flush=True)
    return dict(elements=idx, h=s.q[0][idx], hu=s.q[1][idx], hv=s.q[2][idx], J=s.mesh.J[idx],
                mass0=m0, mass=s.mass(), dt=s.dt_min, final_pp=s.flags.pp[idx],
                final_tvb=s.flags.tvb[idx], M=s.ref.M)


def make_c5(n_samples=64, workers=4, overint=False):
    """Every instance of the ensemble through its own oracle; the records
    are stacked along a leading instance axis.  overint: the over-integrated
    weak form (cubature and Gauss rules) instead of nodal collocation."""
    from concurrent.futures import ProcessPoolExecutor
    from threadpoolctl import threadpool_limits
    n_inst = len(W.c5().instances)
    with threadpool_limits(limits=1), ProcessPoolExecutor(max_workers=workers) as ex:
        recs = list(ex.map(_c5_instance, [(i, n_samples, overint) for i in range(n_inst)]))
    name = "c5_overint" if overint else "c5"
    out = os.path.join(HERE, f"{name}_oracle_samples.npz")
    np.savez_compressed(out, elements=np.stack([r["elements"] for r in recs]),
                        h=np.stack([r["h"] for r in recs]), hu=np.stack([r["hu"] for r in recs]),
                        hv=np.stack([r["hv"] for r in recs]), J=np.stack([r["J"] for r in recs]),
                        mass_matrix=recs[0]["M"], steps=W.c5().steps,
                        mass0=np.array([r["mass0"] for r in recs]), mass=np.array([r["mass"] for r in recs]),
                        dt=np.array([r["dt"] for r in recs]),
                        final_pp=np.stack([r["final_pp"] for r in recs]),
                        final_tvb=np.stack([r["final_tvb"] for r in recs]),
                        command=f"python tests/golden/make_golden.py {name}")
    print("wrote", out, flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if not args:
        print(__doc__)
    for a in args:
        if a == "c2":
            make_c2()
        elif a == "c3":
            make_sampled("c3", W.c3(), 100)
        elif a == "c4":
            make_sampled("c4", W.c4(), 300)
        elif a == "c5":
            make_c5()
        elif a == "c5_overint":
            make_c5(overint=True)
        else:
            print(__doc__)
