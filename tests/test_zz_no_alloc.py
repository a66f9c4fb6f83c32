"""The allocation-free diagnostics entry point against dg_get_diagnostics:
two calls in a row through the C ABI, the second on a smaller solver, each
compared field by field (same kernels, same reduction order: equal bit for
bit)."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_solver, log

pytestmark = pytest.mark.gpu


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(g, out, inst=0):
    import torch
    g.diagnostics_noalloc(inst, out.data_ptr())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = g.diagnostics(inst)
    ref = np.array([want["mass"], want["min_depth"]] + [float(c) for c in want["pp_counts"]]
                   + [float(c) for c in want["tvb_counts"]])
    log(f"[noalloc] K={g.K} mass={got[0]:.15e} min={got[1]:.3e} codes={got[2:]}")
    assert np.array_equal(got, ref), (got, ref)


def test_diagnostics_noalloc_matches_existing_entry_point():
    _require_gpu()
    import torch
    out = torch.full((9,), float("nan"), dtype=torch.float64, device="cuda")
    big = gpu_solver(W.small_wetdry(n=16, N=3), precision="fused_mfma32")
    big.advance(12)
    _check(big, out)
    small = gpu_solver(W.small_wetdry(n=6, N=2), precision="fused_fp32")
    small.advance(7)
    _check(small, out)
    # an ensemble instance other than the first, after the smaller call
    ens = gpu_solver(W.c5(n_inst=3, kmin=400, kmax=3000), precision="fused_mfma32")
    ens.advance(5)
    _check(ens, out, inst=2)
