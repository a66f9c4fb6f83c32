"""Throughput of the DG shallow-water hot path on one MI355X.

One step = one single-rate AB3 step of the whole path (multi-rate: one
coarse step, 2^(L-1) ticks): right-hand side (volume + well-balanced LLF
surface term + lift), AB update, positivity limiter, TVB limiter.  Default
workload (the bench line): 256x256x2 jittered triangles on the unit square
(131072 elements), N = 4 (15 nodes), sloping beach with eight bumps, still
level 0.5, Gaussian hump, wet/dry, CFL 0.2.  --workload c3 / c4 / c5 run the
graded multi-rate mesh (4 levels, N = 3), the 1,048,576-element N = 5 mesh
and the 64-instance ensemble instead.  Inputs are resident in HBM before the
timed region.

Prints one JSON line: node-updates/s (value), the roofline of the fused step
kernel (algorithmic bytes over its HIP-event time, against 8 TB/s), the
plain (unfused) FP32 path and the other fused contraction engines (vector
ALU, FP32 matrix cores, two- and three-part BF16 splits) on the same GPU,
relative L2 against the FP64 oracle after the configured 500 steps of the
default workload for each engine (when the stored oracle samples are
present), the measured stream-copy ceiling, and the oracle's own throughput
on this host's cores (default workload).
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
GOLDEN = os.path.join(ROOT, "tests", "golden", "c2_oracle_samples.npz")
TRAFFIC = os.path.join(ROOT, "profiles", "step_kernel_c2_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1403_1661_amd", "csrc", "dg_kernels.hip")


def kernel_source_hash() -> str:
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(precision: str):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    record, or None when it is missing, for another path, or was taken from a
    different kernel source."""
    if not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash() or rec.get("path") != precision:
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


def make_solver(wl, precision, use_graph=1, tune=False):
    """Solver over all instances of the workload, state set and prepared;
    with tune, the launch shape of the step kernel is picked by the
    library's autotuner (outside any timed region)."""
    from paper_1403_1661_amd import dgswe
    s = dgswe.Solver([(i.vx, i.vy, i.etov) for i in wl.instances], wl.N, g=wl.g, cfl=wl.cfl,
                     precision=precision, use_graph=use_graph, max_levels=wl.max_levels)
    s.bind("cuda:0")
    for j, ins in enumerate(wl.instances):
        x, y = s.node_coords(j)
        s.set_bathymetry(j, ins.bathymetry(x, y))
        s.set_state(j, *ins.initial(x, y))
    s.prepare()
    s.tuning = s.autotune(reps=10) if tune else None
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


def timed(s, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(wl, budget_s=20.0):
    """The FP64 oracle on this host: steps of the same workload until about
    budget_s of CPU work, BLAS pinned to one thread."""
    from threadpoolctl import threadpool_limits
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import oracle_solver
    with threadpool_limits(limits=1):
        o = oracle_solver(wl)
        o.step()
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            o.step()
            n += 1
        dt = time.perf_counter() - t0
    nodes = o.K * o.ref.Np
    return {"value": nodes * n / dt, "unit": "node-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} AB3 steps (after one warm step) of the same 131072-element N=4 "
                      f"workload, {dt:.1f} s, NumPy FP64, BLAS on 1 thread"}


def rel_l2_vs_golden(s, wl):
    if not os.path.exists(GOLDEN):
        return None
    z = np.load(GOLDEN)
    idx = z["elements"]
    h, hu, hv = s.get_state(0)
    M, J = z["mass_matrix"], z["J"]
    out = {}
    for name, test, ref in (("h", [h[idx]], [z["h"]]), ("m", [hu[idx], hv[idx]], [z["hu"], z["hv"]])):
        num = sum(float(np.sum(J * np.einsum("ki,ij,kj->k", a - b, M, a - b))) for a, b in zip(test, ref))
        den = sum(float(np.sum(J * np.einsum("ki,ij,kj->k", b, M, b))) for b in ref)
        out[name] = float(np.sqrt(num / den))
    out["elements_sampled"] = int(idx.size)
    out["steps"] = int(z["steps"])
    return out


WORKLOADS = {
    "c2": ("256x256x2 jittered triangles (131072) on [0,1]^2, N=4 (Np=15), beach 0.8x + 8 bumps, "
           "still level 0.5, hump 0.05, wet/dry PP+TVB, single-rate AB3 at CFL 0.2, 500 configured steps",
           480, 20),
    "c3": ("graded band mesh of [0,4]x[0,1] (54*2^b cells per unit in band b, 496098 triangles), N=3, "
           "B=0.9(x/4)^2, N-wave, 4 MRAB levels, 100 configured coarse steps", 96, 4),
    "c4": ("1024x512x2 jittered triangles (1048576) on [0,2]x[0,1], N=5 (Np=21), 16 Fourier modes, "
           "fully wet, single-rate AB3, 300 configured steps", 280, 20),
    "c5": ("64 jittered unit squares, 10k-200k triangles each (log-uniform), N=3, beach + hump, "
           "wet/dry PP+TVB, CFL 0.2, 200 configured steps each, one batched solver", 180, 20),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--precision", default="fused_mfma32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
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
    import torch
    import workloads as W
    assert torch.cuda.is_available(), "needs a GPU"
    desc, d_steps, d_warm = WORKLOADS[args.workload]
    steps = args.steps if args.steps is not None else d_steps
    warmup = args.warmup if args.warmup is not None else d_warm
    wl = getattr(W, args.workload)()
    Np = wl.Np

    s = make_solver(wl, args.precision, use_graph=0 if args.no_graph else 1, tune=not args.no_tune)
    tuning = s.tuning
    tuned = min(tuning, key=lambda t: t[1])[0] if tuning else None
    per_step = node_updates_per_step(s, wl)
    s.advance(warmup)
    torch.cuda.synchronize()
    t = timed(s, steps, torch)
    ms = 1e3 * t / steps
    value = per_step * steps / t
    accuracy = None
    if args.workload == "c2" and warmup + steps == wl.steps:
        accuracy = rel_l2_vs_golden(s, wl)
    diag = s.diagnostics(0)

    # per-launch duration of the fused step kernel: start/stop events of each
    # launch on the stream it runs on, over a second region of the same length
    s.set_profiling(True)
    s.advance(steps)
    torch.cuda.synchronize()
    avg_us, launches, elems = s.kernel_timing()
    s.set_profiling(False)
    bytes_launch = step_kernel_bytes(Np) * elems
    achieved = bytes_launch / (avg_us * 1e-6) / 1e9
    del s
    copy_gbps = copy_ceiling(torch)

    plain = None
    if not args.no_plain and args.precision != "plain_fp32":
        p = make_solver(wl, "plain_fp32")
        p.advance(warmup)
        tp = timed(p, steps, torch)
        plain = {"value": per_step * steps / tp, "ms_per_step": 1e3 * tp / steps}
        del p

    # the other fused contraction engines on the same workload (same timing,
    # and their accuracy against the stored oracle samples on the full C2 run)
    engines = None
    if not args.no_plain:
        engines = {}
        for prec in ("fused_fp32", "fused_mfma32", "fused_bf16x3", "fused_bf16x6"):
            if prec == args.precision:
                continue
            e = make_solver(wl, prec, tune=not args.no_tune)
            e.advance(warmup)
            te = timed(e, steps, torch)
            entry = {"value": per_step * steps / te, "ms_per_step": 1e3 * te / steps}
            if args.workload == "c2" and warmup + steps == wl.steps:
                entry["rel_l2_vs_oracle"] = rel_l2_vs_golden(e, wl)
            engines[prec] = entry
            del e

    kname = "step_mfma_kernel" if args.precision in ("fused_mfma32", "fused_bf16x3", "fused_bf16x6") \
        else "step_kernel"
    traffic = measured_traffic(args.precision) if args.workload == "c2" else None
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
        "config": {"workload": desc, "name": args.workload,
                   "elements": int(sum(i.etov.shape[0] for i in wl.instances)),
                   "instances": len(wl.instances), "N": wl.N, "path": args.precision,
                   "parallelism": "single GPU", "elems_per_block": tuned,
                   "autotune_us": {str(e): round(us, 2) for e, us in tuning} if tuning else None},
        "hbm_gbps_algorithmic_step": step_kernel_bytes(Np) * (per_step / Np) * steps / t / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "copy_ceiling_gbps": copy_gbps, "frac_of_copy_ceiling": achieved / copy_gbps,
                     "kernel": f"{kname}<{wl.N}> (fused RHS + AB3 + positivity)",
                     "kernel_avg_us": avg_us, "launches_timed": launches,
                     "elements_per_launch": elems, "bytes_per_launch": bytes_launch},
        "plain_fp32": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "engines": engines,
        "rel_l2_vs_oracle": accuracy,
        "diagnostics": {"mass": diag["mass"], "min_depth": diag["min_depth"],
                        "pp_counts": diag["pp_counts"], "tvb_counts": diag["tvb_counts"],
                        "negative_means": diag["negative_means"]},
    }
    if not args.no_cpu and args.workload == "c2":
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
