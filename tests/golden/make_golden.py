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

c3: the 496098-triangle graded band mesh with 4 multi-rate levels for 10
coarse steps (80 ticks) of the full run; the same record plus the level of
every element.

    python tests/golden/make_golden.py c3 c4
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


if __name__ == "__main__":
    args = sys.argv[1:]
    if not args:
        print(__doc__)
    for a in args:
        if a == "c2":
            make_c2()
        elif a == "c3":
            make_sampled("c3", W.c3(), 10)
        elif a == "c4":
            make_sampled("c4", W.c4(), 300)
        else:
            print(__doc__)
