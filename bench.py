"""Throughput of the DG shallow-water hot path on one MI355X.

One step = one single-rate AB3 step of the whole path (multi-rate: one
coarse step, 2^(L-1) ticks) over every element of the workload: right-hand
side (volume + well-balanced LLF surface term + lift), AB update, positivity
limiter, TVB limiter.

Default workload (the bench line): the batched ensemble of 64 jittered unit
squares with 10k-200k triangles each (log-uniform, 4126216 triangles in
all), N = 3, a beach and a hump per instance, wet/dry, CFL 0.2, each
instance with its own time step, all advanced together.  --workload c4 times
the 1048576-triangle N = 5 fully wet mesh, c3 the graded four-level
multi-rate mesh, c2 the 131072-triangle N = 4 beach.  Inputs are resident in
HBM before the timed region; the replay graph is captured before it.

Prints one JSON line: node-updates/s (value) over the timed region; the
roofline of the fused step kernel (algorithmic bytes over its HIP-event
time, against 8 TB/s) and of the whole step (step + TVB kernels); the TVB
kernel's time; the plain (unfused) FP32 path and the other contraction
engines on the same workload; relative L2 against stored FP64 oracle samples
after the workload's configured step count (each solver is run on to that
count after its timed region); the measured stream-copy ceiling; and the
oracle's own throughput on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1403_1661_amd", "csrc", "dg_kernels.hip")
MAX_CPU_WORKERS = 16


def progress(msg: str):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload: str, precision: str, elems_per_block):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    record of this workload, or None when it is missing, was taken on another
    path or launch shape, or from a different kernel source."""
    path = os.path.join(PROFILES, f"step_kernel_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (rec.get("kernel_source_sha256") != kernel_source_hash() or rec.get("path") != precision
            or rec.get("elems_per_block") != elems_per_block):
        return None
    return rec.get("bytes_per_launch")


def copy_reference(n_bytes: int = 1 << 29, reps: int = 5):
    """A plain device copy of a known size (reference for the counters)."""
    import torch
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_reference_bytes_read": n_bytes, "copy_reference_bytes_written": n_bytes,
                      "reps": reps}), flush=True)


def copy_ceiling(torch, n_bytes: int = 1 << 29, reps: int = 20) -> float:
    """Measured stream-copy bandwidth of this GPU in GB/s (bytes read plus
    bytes written per second): a device-to-device copy of 512 MiB, twice the
    size of the last-level cache, timed with events after a warm-up."""
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    del src, dst
    return 2.0 * n_bytes * reps / sec / 1e9


def step_kernel_bytes(Np: int) -> int:
    """Algorithmic HBM bytes per element of one single-rate step (what the
    method has to move, each array once, FP32 nodal data): state h, hu, hv
    read + write 2*3*Np*4, bed Np*4, RHS history 1 write + 2 reads 3*3*Np*4,
    geometry 14 floats, connectivity 16, FP64 means 24, flag 1.  Neighbour
    face values (halo), the low word of the compensated surface level and the
    TVB deviations of candidate elements are implementation traffic on top."""
    return 64 * Np + 97


def make_solver(wl, precision, use_graph=1, tune=False, overint=0):
    """Solver over all instances of the workload, state set and prepared;
    with tune, the launch shape of the step kernel is picked by the
    library's autotuner (outside any timed region).  overint: the
    over-integrated weak form instead of nodal collocation."""
    from paper_1403_1661_amd import dgswe
    s = dgswe.Solver([(i.vx, i.vy, i.etov) for i in wl.instances], wl.N, g=wl.g, cfl=wl.cfl,
                     precision=precision, use_graph=use_graph, max_levels=wl.max_levels,
                     overint=overint)
    s.bind("cuda:0")
    for j, ins in enumerate(wl.instances):
        x, y = s.node_coords(j)
        s.set_bathymetry(j, ins.bathymetry(x, y))
        s.set_state(j, *ins.initial(x, y))
    s.prepare()
    s.tuning = s.autotune(reps=10) if tune else None
    s.steps_done = 0
    return s


def node_updates_per_step(s, wl) -> int:
    """Node-updates of one (coarse) step: every element advances 2^(L-l)
    times on level l of L."""
    total = 0
    for j in range(len(wl.instances)):
        lev, _ = s.levels(j)
        L = int(lev.max())
        total += int(np.sum(2 ** (L - lev.astype(np.int64)))) * wl.Np
    return total


def advance(s, n):
    s.advance(n)
    s.steps_done += n


def warm_and_capture(s, warmup, use_graph, torch):
    """Untimed warm-up steps, then the replay graph captured from the state
    the timed region starts in (needs the two start-up steps behind it)."""
    advance(s, warmup)
    captured = False
    if use_graph and warmup >= 2:
        s.capture_graph()
        captured = True
    torch.cuda.synchronize()
    return captured


def timed(s, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(s, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _oracle_worker(args):
    """One instance of the workload through the FP64 oracle: setup untimed,
    then steps until budget_s of wall time (one BLAS thread)."""
    name, inst, budget_s = args
    from threadpoolctl import threadpool_limits
    import workloads as W
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import oracle_solver
    wl = getattr(W, name)()
    with threadpool_limits(limits=1):
        o = oracle_solver(wl, inst=inst)
        o.step()
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            o.step()
            n += 1
        dt = time.perf_counter() - t0
    return o.K * o.ref.Np * n, dt, n, o.K


def cpu_baseline(name, wl, budget_s=15.0):
    """The FP64 oracle on this host.  Ensemble: one oracle process per
    instance for the first P instances (P = the host cores this process may
    use, at most 16), all running at once, each timed over about budget_s
    after its setup and one warm step; single mesh: one process on the whole
    mesh.  BLAS runs one thread per process, so P processes use P cores."""
    cores = len(os.sched_getaffinity(0))
    P = max(1, min(MAX_CPU_WORKERS, cores, len(wl.instances)))
    if P > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=P, mp_context=mp.get_context("fork")) as ex:
            res = list(ex.map(_oracle_worker, [(name, i, budget_s) for i in range(P)]))
    else:
        res = [_oracle_worker((name, 0, budget_s))]
    value = sum(nu / dt for nu, dt, _, _ in res)
    steps = [n for _, _, n, _ in res]
    Ks = [k for _, _, _, k in res]
    sample = (f"{P} instance(s) of the same workload (K = {min(Ks)}..{max(Ks)}), one oracle process each, "
              f"running concurrently, {min(steps)}-{max(steps)} AB3 steps each after one warm step, "
              f"~{budget_s:.0f} s each, NumPy FP64, one BLAS thread per process"
              if P > 1 else
              f"{steps[0]} AB3 steps (after one warm step) of the whole {Ks[0]}-element mesh, "
              f"~{budget_s:.0f} s, NumPy FP64, one BLAS thread")
    return {"value": value, "unit": "node-updates/s", "cores": P, "kind": "oracle",
            "host_cores_visible": cores, "sample": sample}


def rel_l2_vs_golden(s, name):
    """Relative L2 (depth, momentum pair) of the sampled elements against the
    stored oracle record of the workload, pooled over instances (and the
    worst instance), with the count of limiter codes that differ."""
    path = os.path.join(GOLDEN_DIR, f"{name}_oracle_samples.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    if s.steps_done != int(z["steps"]):
        return None
    M = z["mass_matrix"]
    idx_all, J_all = z["elements"], z["J"]
    multi = idx_all.ndim == 2
    n_inst = idx_all.shape[0] if multi else 1
    num = {"h": 0.0, "m": 0.0}
    den = {"h": 0.0, "m": 0.0}
    worst = {"h": 0.0, "m": 0.0}
    flips = 0

    def nrm(a, J):
        return float(np.sum(J * np.einsum("ki,ij,kj->k", a, M, a)))

    for i in range(n_inst):
        sel = (lambda a: a[i]) if multi else (lambda a: a)
        idx, J = sel(idx_all), sel(J_all)
        h, hu, hv = s.get_state(i)
        nh, dh = nrm(h[idx] - sel(z["h"]), J), nrm(sel(z["h"]), J)
        nm = nrm(hu[idx] - sel(z["hu"]), J) + nrm(hv[idx] - sel(z["hv"]), J)
        dm = nrm(sel(z["hu"]), J) + nrm(sel(z["hv"]), J)
        num["h"] += nh
        den["h"] += dh
        num["m"] += nm
        den["m"] += dm
        worst["h"] = max(worst["h"], np.sqrt(nh / dh))
        worst["m"] = max(worst["m"], np.sqrt(nm / dm) if dm > 0 else np.sqrt(nm))
        f = s.flags(i)[idx]
        fpp, ftv = sel(z["final_pp"]), sel(z["final_tvb"])
        if fpp.shape[0] != idx.shape[0]:      # codes stored for every element
            fpp, ftv = fpp[idx], ftv[idx]
        flips += int(np.sum((f & 3) != fpp)) + int(np.sum(((f >> 2) & 3) != ftv))
    return {"h": float(np.sqrt(num["h"] / den["h"])), "m": float(np.sqrt(num["m"] / den["m"])),
            "worst_instance_h": float(worst["h"]), "worst_instance_m": float(worst["m"]),
            "limiter_flips": flips, "instances": n_inst,
            "elements_sampled": int(idx_all.size), "steps": int(z["steps"])}


def accuracy_at_configured_steps(s, wl, name):
    """Run the solver on to the workload's configured step count and compare
    with the stored oracle samples (None when already past it or when no
    samples are stored for this workload)."""
    left = wl.steps - s.steps_done
    if left < 0 or not os.path.exists(os.path.join(GOLDEN_DIR, f"{name}_oracle_samples.npz")):
        return None
    advance(s, left)
    return rel_l2_vs_golden(s, name)


WORKLOADS = {
    "c2": ("256x256x2 jittered triangles (131072) on [0,1]^2, N=4 (Np=15), beach 0.8x + 8 bumps, "
           "still level 0.5, hump 0.05, wet/dry PP+TVB, single-rate AB3 at CFL 0.2, 500 configured steps",
           200, 20),
    "c3": ("graded band mesh of [0,4]x[0,1] (54*2^b cells per unit in band b, 496098 triangles), N=3, "
           "B=0.9(x/4)^2, N-wave, 4 MRAB levels, 100 configured coarse steps", 24, 6),
    "c4": ("1024x512x2 jittered triangles (1048576) on [0,2]x[0,1], N=5 (Np=21), 16 Fourier modes, "
           "fully wet, single-rate AB3, 300 configured steps", 60, 6),
    "c5": ("64 jittered unit squares, 10k-200k triangles each (log-uniform, 4126216 in all), N=3, "
           "beach + hump each, wet/dry PP+TVB, CFL 0.2, 200 configured steps each, one batched solver",
           60, 6),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--precision", default="fused_mfma32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain path and the other engines")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the run to the configured step count")
    ap.add_argument("--no-graph", action="store_true", help="eager launches (for counter runs)")
    ap.add_argument("--no-tune", action="store_true", help="default launch shape, no autotuning")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain copy of 512 MiB (counter reference)")
    args = ap.parse_args()
    if args.copy_ref:
        copy_reference()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is measured "
              "on one GPU's share and its multi-GPU sharding is a design note", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    name = args.workload
    desc, d_steps, d_warm = WORKLOADS[name]
    steps = args.steps if args.steps is not None else d_steps
    warmup = args.warmup if args.warmup is not None else d_warm
    wl = getattr(W, name)()
    Np = wl.Np
    use_graph = 0 if args.no_graph else 1

    # the oracle's processes are forked before this process touches the GPU
    cpu = None
    if not args.no_cpu:
        progress("oracle baseline on the host cores")
        cpu = cpu_baseline(name, wl)
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    progress(f"{name}: {wl.n_elements} elements, building the {args.precision} solver")
    s = make_solver(wl, args.precision, use_graph=use_graph, tune=not args.no_tune)
    tuning = s.tuning
    tuned = min(tuning, key=lambda t: t[1])[0] if tuning else None
    per_step = node_updates_per_step(s, wl)
    captured = warm_and_capture(s, warmup, use_graph, torch)
    t = timed(s, steps, torch)
    ms = 1e3 * t / steps
    value = per_step * steps / t

    # per-launch duration of the step and TVB kernels: start/stop events of
    # each launch on the stream it runs on, over a second (eager) region
    prof_steps = min(steps, 12)
    s.set_profiling(True)
    advance(s, prof_steps)
    torch.cuda.synchronize()
    avg_us, launches, elems = s.kernel_timing(0)
    tvb_us, tvb_launches, _ = s.kernel_timing(1)
    s.set_profiling(False)
    progress(f"timed {steps} steps: {ms:.4f} ms/step, step kernel {avg_us:.1f} us, TVB {tvb_us:.1f} us")
    accuracy = None if args.no_accuracy else accuracy_at_configured_steps(s, wl, name)
    diag = [s.diagnostics(i) for i in range(len(wl.instances))]
    del s
    torch.cuda.empty_cache()
    bytes_launch = step_kernel_bytes(Np) * elems
    achieved = bytes_launch / (avg_us * 1e-6) / 1e9
    elements = int(sum(i.etov.shape[0] for i in wl.instances))
    step_bytes = step_kernel_bytes(Np) * (per_step / Np)     # element-updates x bytes
    whole_gbps = step_bytes / (ms * 1e-3) / 1e9
    copy_gbps = copy_ceiling(torch)

    # the plain path and the other fused contraction engines on the same
    # workload: same timing, then each run on to the configured step count
    engines = None
    plain = None
    if not args.no_plain:
        engines = {}
        for prec in ("plain_fp32", "fused_fp32", "fused_mfma32", "fused_bf16x3", "fused_bf16x6"):
            if prec == args.precision:
                continue
            e = make_solver(wl, prec, use_graph=use_graph, tune=not args.no_tune and prec != "plain_fp32")
            warm_and_capture(e, warmup, use_graph, torch)
            te = timed(e, steps, torch)
            entry = {"value": per_step * steps / te, "ms_per_step": 1e3 * te / steps}
            if not args.no_accuracy:
                entry["rel_l2_vs_oracle"] = accuracy_at_configured_steps(e, wl, name)
            engines[prec] = entry
            progress(f"engine {prec}: {entry['ms_per_step']:.4f} ms/step")
            del e
            torch.cuda.empty_cache()
        plain = engines.get("plain_fp32")

    # the paper's own discretisation: the over-integrated weak form (cubature
    # volume term, Gauss surface term; N <= 5): its right-hand side kernel,
    # then the update and limiters of the matrix-core path
    overint = None
    if not args.no_plain and wl.N <= 5:
        e = make_solver(wl, "fused_mfma32", use_graph=use_graph, tune=False, overint=1)
        warm_and_capture(e, warmup, use_graph, torch)
        te = timed(e, steps, torch)
        e.set_profiling(True)
        advance(e, prof_steps)
        torch.cuda.synchronize()
        rhs_us, _, _ = e.kernel_timing(0)
        e.set_profiling(False)
        overint = {"value": per_step * steps / te, "ms_per_step": 1e3 * te / steps,
                   "rhs_kernel_avg_us": rhs_us,
                   "note": "weak form with cubature and Gauss rules exact to degree 3N; RHS kernel "
                           "with its contractions on the matrix cores, then the AB update, positivity "
                           "limiter and TVB hand-off in the matrix-core step kernel without its "
                           "right-hand side, then the TVB kernel"}
        if not args.no_accuracy:
            overint["rel_l2_vs_oracle"] = accuracy_at_configured_steps(e, wl, f"{name}_overint")
        progress(f"over-integrated: {overint['ms_per_step']:.4f} ms/step, RHS kernel {rhs_us:.1f} us")
        del e
        torch.cuda.empty_cache()

    kname = "step_mfma_kernel" if args.precision in ("fused_mfma32", "fused_bf16x3", "fused_bf16x6") \
        else "step_kernel"
    traffic = measured_traffic(name, args.precision, tuned)
    neg = sum(d["negative_means"] for d in diag)
    out = {
        "metric": "DG node-updates/s + HBM GB/s; FP32/BF16-split vs FP32 plain at rel-L2 1e-5",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": name, "elements": elements,
                   "instances": len(wl.instances), "N": wl.N, "path": args.precision,
                   "parallelism": "single GPU", "elems_per_block": tuned,
                   "graph_captured_before_timing": captured,
                   "autotune_us": {str(e): round(us, 2) for e, us in tuning} if tuning else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "copy_ceiling_gbps": copy_gbps, "frac_of_copy_ceiling": achieved / copy_gbps,
                     "kernel": f"{kname}<{wl.N}> (fused RHS + AB update + positivity limiter)",
                     "kernel_avg_us": avg_us, "launches_timed": launches,
                     "elements_per_launch": elems, "bytes_per_launch": bytes_launch,
                     "tvb_kernel_avg_us": tvb_us, "tvb_launches_timed": tvb_launches,
                     "whole_step": {"achieved": whole_gbps, "frac": whole_gbps / HBM_PEAK_GBS,
                                    "bytes_per_step": step_bytes,
                                    "note": "algorithmic bytes of the step over the timed ms_per_step "
                                            "(step kernel, TVB kernel and launch gaps)"}},
        "plain_fp32": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "engines": engines,
        "overint_fp32": overint,
        "rel_l2_vs_oracle": accuracy,
        "diagnostics": {"mass": sum(d["mass"] for d in diag), "min_depth": min(d["min_depth"] for d in diag),
                        "pp_counts": [sum(d["pp_counts"][c] for d in diag) for c in range(3)],
                        "tvb_counts": [sum(d["tvb_counts"][c] for d in diag) for c in range(4)],
                        "negative_means": neg},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
