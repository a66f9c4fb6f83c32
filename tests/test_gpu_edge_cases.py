"""Edge cases of the HIP path against the FP64 oracle: meshes smaller than one
block of the step kernels (1, 2 and 7 elements: every launch is ragged and
the clamped loads of the matrix-core kernel serve lanes past the last
element), an ensemble of such ragged instances, a fully dry domain (every
element takes the dry branch of Algorithm 5.2 and the TVB skip rule), and
orders 1 and 5 on the smallest meshes."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from helpers import flag_flips, gpu_solver, log, oracle_solver, rel_l2

pytestmark = pytest.mark.gpu

PATHS = ["plain_fp32", "fused_fp32", "fused_mfma32"]


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bed(x, y):
    return 0.3 * np.asarray(x) + 0.1 * np.asarray(y)


def _tiny(n_cells_x: int, n_cells_y: int, split_one: bool = False):
    """Triangles of a small structured patch; split_one keeps a single
    triangle of the first cell."""
    vx, vy, etov = W.structured_mesh(n_cells_x, n_cells_y, 0.0, 1.0, 0.0, 1.0)
    if split_one:
        etov = etov[:1]
    return vx, vy, etov


def _hump(x, y):
    eta = 1.0 + 0.05 * np.exp(-20.0 * ((x - 0.4) ** 2 + (y - 0.3) ** 2))
    h = eta - _bed(x, y)
    return h, np.zeros_like(h), np.zeros_like(h)


def _workload(meshes, N, init=_hump, steps=20):
    insts = [W.Instance(vx, vy, ev, _bed, init, f"tiny{i}") for i, (vx, vy, ev) in enumerate(meshes)]
    return W.Workload("tiny", N, insts, steps=steps, cfl=0.3)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N,shape", [(4, (1, 1, True)), (4, (1, 1, False)), (3, (2, 2, False)),
                                     (1, (1, 1, True)), (5, (1, 1, False)), (5, (2, 1, False))])
def test_tiny_meshes(path, N, shape):
    _require_gpu()
    wl = _workload([_tiny(*shape)], N)
    K = wl.n_elements
    g = gpu_solver(wl, precision=path)
    o = oracle_solver(wl)
    g.advance(wl.steps)
    o.run(wl.steps)
    err = rel_l2(o, np.stack(g.get_state(0)), o.q)
    log(f"[tiny] {path} N={N} K={K} relL2 h={err['h']:.3e} m={err['m']:.3e}")
    assert err["h"] <= 1e-5 and err["m"] <= 1e-5
    assert flag_flips(g.flags(0), o.flags) == (0, 0)


@pytest.mark.parametrize("path", ["fused_fp32", "fused_mfma32"])
def test_ragged_ensemble(path):
    """Instances of 1, 2, 7 and 18 elements advanced together: element
    blocks straddle instance boundaries."""
    _require_gpu()
    vx, vy, ev = _tiny(3, 3)
    meshes = [_tiny(1, 1, True), _tiny(1, 1), (vx, vy, ev[:7]), _tiny(3, 3)]
    wl = _workload(meshes, 4)
    g = gpu_solver(wl, precision=path)
    g.advance(wl.steps)
    for i in range(len(meshes)):
        o = oracle_solver(wl, inst=i)
        o.run(wl.steps)
        err = rel_l2(o, np.stack(g.get_state(i)), o.q)
        log(f"[ragged] {path} inst {i} K={meshes[i][2].shape[0]} relL2 h={err['h']:.3e} m={err['m']:.3e}")
        assert err["h"] <= 1e-5 and err["m"] <= 1e-5


@pytest.mark.parametrize("path", PATHS)
def test_all_dry_domain(path):
    """The bed is above the still level everywhere: every element is dry, the
    state stays exactly zero depth and momentum, the flags say dry and
    skipped, and nothing becomes non-finite."""
    _require_gpu()

    def dry(x, y):
        z = np.zeros_like(np.asarray(x, dtype=np.float64))
        return z, z.copy(), z.copy()

    vx, vy, ev = W.structured_mesh(6, 5, 0.0, 1.0, 0.0, 1.0)
    wl = _workload([(vx, vy, ev)], 3, init=dry)
    g = gpu_solver(wl, precision=path)
    g.advance(wl.steps)
    h, hu, hv = g.get_state(0)
    assert np.all(np.isfinite(h)) and np.all(h == 0.0)
    assert np.all(hu == 0.0) and np.all(hv == 0.0)
    f = g.flags(0)
    assert np.all((f & 3) == 2) and np.all((f >> 2) == 0)
    d = g.diagnostics(0)
    assert d["mass"] == 0.0 and d["pp_counts"][2] == wl.n_elements


@pytest.mark.parametrize("path", ["fused_fp32", "fused_mfma32"])
def test_multirate_tiny_levels(path):
    """Four MRAB levels of a few elements to a hundred (the coarsest smaller
    than one block of the step kernels): every level's part of a launch is
    ragged, and neighbours across level boundaries are read from the other
    parity or from half-step traces (Section 4)."""
    _require_gpu()
    wl = W.c3(n0=1)
    g = gpu_solver(wl, precision=path)
    o = oracle_solver(wl)
    lev, _ = g.levels(0)
    assert np.array_equal(lev.astype(int), o.levels)
    sizes = [int(np.sum(o.levels == l)) for l in range(1, wl.max_levels + 1)]
    log(f"[mrab-tiny] {path} K={wl.n_elements} level sizes {sizes}")
    g.advance(4)
    o.run(4)
    err = rel_l2(o, np.stack(g.get_state(0)), o.q)
    log(f"[mrab-tiny] relL2 h={err['h']:.3e} m={err['m']:.3e}")
    assert err["h"] <= 1e-5 and err["m"] <= 1e-5
    assert flag_flips(g.flags(0), o.flags) == (0, 0)


@pytest.mark.parametrize("path", ["plain_fp32", "fused_fp32", "fused_mfma32", "fused_bf16x6"])
@pytest.mark.parametrize("N", [1, 2, 4, 5])
def test_multirate_other_orders(path, N):
    """Multi-rate AB3 at the orders other than 3: the vector-ALU kernels and,
    on the matrix cores, the 16-lane groups (N = 1, 2, 4) and the packed
    21-lane groups (N = 5) of the multi-rate step kernel; four levels on the
    small graded band mesh, four coarse steps."""
    _require_gpu()
    import dataclasses
    wl = dataclasses.replace(W.c3(n0=2), N=N)
    g = gpu_solver(wl, precision=path)
    o = oracle_solver(wl)
    lev, _ = g.levels(0)
    assert np.array_equal(lev.astype(int), o.levels)
    g.advance(4)
    o.run(4)
    err = rel_l2(o, np.stack(g.get_state(0)), o.q)
    log(f"[mrab-N{N}] {path} K={wl.n_elements} relL2 h={err['h']:.3e} m={err['m']:.3e}")
    assert err["h"] <= 1e-5 and err["m"] <= 1e-5
    assert flag_flips(g.flags(0), o.flags) == (0, 0)


@pytest.mark.parametrize("path", ["fused_fp32", "fused_mfma32"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_tvb_fallback_stencil(path, N):
    """TVB limiting through the one-neighbour fallback of the stencil (two
    edges of the central element of the skewed patch) and next to a sliver:
    M = 0, every element limited at every step, 10 steps."""
    _require_gpu()
    wl = W.skewed_patch(N=N)
    g = gpu_solver(wl, precision=path, tvb_M=0.0)
    o = oracle_solver(wl, tvb_M=0.0)
    pair, _ = g.tvb_stencil(0)
    assert pair[0, 0, 0] == pair[0, 0, 1] and pair[0, 2, 0] == pair[0, 2, 1]
    g.advance(10)
    o.run(10)
    err = rel_l2(o, np.stack(g.get_state(0)), o.q)
    log(f"[tvb-fallback] N={N} {path} relL2 h={err['h']:.3e} m={err['m']:.3e} "
        f"flags {g.flags(0).tolist()}")
    assert err["h"] <= 1e-5 and err["m"] <= 1e-5
    assert flag_flips(g.flags(0), o.flags) == (0, 0)
    assert np.all((o.flags.tvb == 2) | (o.flags.tvb == 3))


@pytest.mark.parametrize("N,path", [(N, p) for N in (1, 2, 3, 4, 5) for p in ("fused_fp32", "fused_mfma32")]
                         + [(6, "fused_fp32")])
def test_near_dry_front(path, N):
    """Deep water against a thin film with M = 0 and h0 = 1e-3: the depth
    modification of Eq. 5.3 on limited elements next to the film, and at
    N = 4 elements whose nodes are all wet but whose mean is negative (made
    dry by the positivity limiter).  The initial limiting and 5 steps."""
    _require_gpu()
    wl = W.near_dry_front(N=N)
    g = gpu_solver(wl, precision=path, tvb_M=0.0, h0=1e-3)
    o = oracle_solver(wl, tvb_M=0.0, h0=1e-3)
    g.prepare()
    err0 = rel_l2(o, np.stack(g.get_state(0)), o.q)
    flips0 = flag_flips(g.flags(0), o.flags)
    tv_o = np.bincount(o.flags.tvb, minlength=4)
    g.advance(5)
    o.run(5)
    err = rel_l2(o, np.stack(g.get_state(0)), o.q)
    flips = flag_flips(g.flags(0), o.flags)
    log(f"[near-dry] N={N} {path} initial relL2 h={err0['h']:.3e} m={err0['m']:.3e} flips {flips0} "
        f"tvb codes {tv_o.tolist()}; 5 steps relL2 h={err['h']:.3e} m={err['m']:.3e} flips {flips}")
    assert tv_o[3] > 0 or N == 1
    assert err0["h"] <= 1e-5 and err0["m"] <= 1e-5 and flips0 == (0, 0)
    assert err["h"] <= 1e-5 and err["m"] <= 1e-5
    # M = 0 compares nearly equal characteristic increments: FP32 and FP64
    # part on a few keep-or-limit decisions (as in the TVD test of C1)
    assert sum(flips) <= 0.05 * wl.n_elements
    assert g.diagnostics(0)["min_depth"] >= 0.0


def test_multirate_block_shapes_bitwise():
    """The multi-rate launch cuts each level's element range into whole
    blocks; 1, 2, 4 or 8 waves per block change only that cut, so the MRAB
    trajectories agree bit for bit."""
    _require_gpu()
    wl = W.c3(n0=2)
    runs = []
    for epb in (5, 10, 20, 40):   # N = 3: five 12-lane elements per wave
        g = gpu_solver(wl, precision="fused_mfma32", elems_per_block=epb)
        g.advance(5)
        runs.append(g.get_state(0))
    for other in runs[1:]:
        for x, y in zip(other, runs[0]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("path", PATHS)
def test_internal_barrier(path):
    """Tagged internal walls (dg_mesh_desc.bc): with an opening the HIP path
    follows the oracle; with the wall closed the undisturbed basin stays
    bitwise at rest and keeps its mass."""
    _require_gpu()
    wl = W.barrier_basin(n=16, N=3)
    g = gpu_solver(wl, precision=path)
    o = oracle_solver(wl)
    etoe, _ = g.connectivity(0)
    assert np.array_equal(etoe, o.mesh.etoe)
    g.advance(60)
    o.run(60)
    err = rel_l2(o, np.stack(g.get_state(0)), o.q)
    log(f"[barrier] {path} relL2 h={err['h']:.3e} m={err['m']:.3e}")
    assert err["h"] <= 1e-5 and err["m"] <= 1e-5
    assert flag_flips(g.flags(0), o.flags) == (0, 0)

    closed = W.barrier_basin(n=16, N=3, gap=(2.0, 2.0))
    g = gpu_solver(closed, precision=path)
    g.prepare()   # the initial limiting; the state is on the device from here on
    h0, hu0, hv0 = g.get_state(0)
    g.advance(60)
    h, hu, hv = g.get_state(0)
    x, _ = g.node_coords(0)
    right = x.mean(axis=1) > 0.5
    assert np.array_equal(h[right], h0[right])
    assert np.all(hu[right] == 0.0) and np.all(hv[right] == 0.0)
    assert np.max(np.abs(hu[~right])) > 1e-3


def test_host_side_input_errors():
    """Inputs the library rejects before any kernel runs: depth or momentum
    that is negative or not finite, a state before its bathymetry, and
    checkpoints that are short or come from a solver of another shape."""
    _require_gpu()
    from paper_1403_1661_amd import dgswe
    wl = _workload([_tiny(2, 2), _tiny(3, 2)], 2)
    g = dgswe.Solver([(i.vx, i.vy, i.etov) for i in wl.instances], 2)
    g.bind("cuda:0")
    x, y = g.node_coords(0)
    h = np.ones_like(x)
    with pytest.raises(dgswe.DGError) as e:          # no bathymetry yet
        g.set_state(0, h, 0 * h, 0 * h)
    assert e.value.code == -7
    g.set_bathymetry(0, np.zeros_like(x))
    bad = h.copy()
    bad[0, 0] = -1e-3
    with pytest.raises(dgswe.DGError) as e:
        g.set_state(0, bad, 0 * h, 0 * h)
    assert e.value.code == -6
    mom = np.zeros_like(h)
    mom[1, 1] = np.inf
    with pytest.raises(dgswe.DGError) as e:
        g.set_state(0, h, mom, 0 * h)
    assert e.value.code == -6
    x1, _ = g.node_coords(1)
    g.set_bathymetry(1, np.zeros_like(x1))
    g.set_state(0, h, 0 * h, 0 * h)
    g.set_state(1, np.ones_like(x1), 0 * x1, 0 * x1)
    g.advance(2)
    blob = g.checkpoint()
    with pytest.raises(dgswe.DGError) as e:          # short blob
        g.restore(blob[:-8])
    assert e.value.code == -1
    other = gpu_solver(_workload([_tiny(2, 2)], 2))    # one instance, fewer elements
    other.prepare()
    with pytest.raises(dgswe.DGError) as e:
        other.restore(blob + bytes(max(0, len(other.checkpoint()) - len(blob))))
    assert e.value.code == -1
    g.restore(blob)                                    # its own blob still restores
    # a corrupt schedule state (state parity 5 at byte 40 of the header) is
    # rejected before anything is copied to the device
    bad_blob = bytearray(blob)
    bad_blob[40:44] = (5).to_bytes(4, "little", signed=True)
    with pytest.raises(dgswe.DGError) as e:
        g.restore(bytes(bad_blob))
    assert e.value.code == -1
    bad_blob = bytearray(blob)
    bad_blob[40 + 24:40 + 28] = (3).to_bytes(4, "little", signed=True)   # ring head 3
    with pytest.raises(dgswe.DGError) as e:
        g.restore(bytes(bad_blob))
    assert e.value.code == -1
    # a blob taken over another bathymetry is rejected
    h2 = gpu_solver(_workload([_tiny(2, 2), _tiny(3, 2)], 2))
    h2.set_bathymetry(0, 0.01 * np.ones_like(x))
    h2.set_state(0, h, 0 * h, 0 * h)
    h2.prepare()
    with pytest.raises(dgswe.DGError) as e:
        h2.restore(blob)
    assert e.value.code == -1
