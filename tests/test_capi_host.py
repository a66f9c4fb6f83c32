"""C-ABI library on the CPU: it loads, exports every declared symbol, and its
host setup (reference element, connectivity, levels, TVB stencil, node
coordinates) agrees with the oracle.  No device calls."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle.mesh import assign_levels, build_mesh, tvb_stencil
from oracle.refelem import reference_element
from paper_1403_1661_amd import dgswe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return dgswe.load_library()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "dgswe.h")).read()
    declared = set(re.findall(r"\b(dg_[a-z_]+)\s*\(", hdr))
    assert declared == set(dgswe.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_reference_element_matches_oracle(N):
    vx, vy, etov = W.structured_mesh(2, 2, 0, 1, 0, 1)
    s = dgswe.Solver([(vx, vy, etov)], N)
    ref = reference_element(N)
    r, sn = s.reference_nodes()
    assert np.max(np.abs(r - ref.r)) < 1e-14
    assert np.max(np.abs(sn - ref.s)) < 1e-14
    assert np.max(np.abs(s.reference(0) - ref.Dr)) < 1e-12
    assert np.max(np.abs(s.reference(1) - ref.Ds)) < 1e-12
    assert np.max(np.abs(s.reference(2) - ref.LIFT)) < 1e-12
    assert np.max(np.abs(s.reference(3) - ref.M)) < 1e-13
    assert np.max(np.abs(s.reference(4) - ref.w)) < 1e-13
    assert np.array_equal(s.reference(5).astype(int), ref.fmask)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_overint_operators_match_oracle(N):
    """The library's cubature and Gauss rules and the over-integrated
    operators (built on the host by its own Gauss-Jacobi Newton iteration and
    barycentric face interpolation) agree with the oracle's (SciPy rules,
    2D Vandermonde evaluation at the face points)."""
    from oracle.overint import overint_operators
    vx, vy, etov = W.structured_mesh(2, 2, 0, 1, 0, 1)
    s = dgswe.Solver([(vx, vy, etov)], N)
    oi = overint_operators(reference_element(N))
    cub = s.reference(6)
    assert np.max(np.abs(cub[0] - oi.rc)) < 1e-14 and np.max(np.abs(cub[1] - oi.sc)) < 1e-14
    assert np.max(np.abs(cub[2] - oi.wc)) < 1e-15
    gw = s.reference(11)
    xi = np.polynomial.legendre.leggauss(oi.NG)[0]
    assert np.max(np.abs(gw[0] - xi)) < 1e-14 and np.max(np.abs(gw[1] - oi.wg)) < 1e-14
    for which, want in ((7, oi.Ic), (8, oi.Pr), (9, oi.Ps), (10, oi.P), (13, oi.Lg)):
        got = s.reference(which)
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) < 1e-11 * max(1.0, np.max(np.abs(want))), which
    # face-node interpolation at the Gauss points reproduces I_g on face 0
    ref = reference_element(N)
    I1 = s.reference(12)
    assert np.max(np.abs(I1 - oi.Ig[:oi.NG][:, ref.fmask[0]])) < 1e-13


@pytest.mark.parametrize("case", ["c1", "wetdry", "c3small", "barrier", "skewed"])
def test_mesh_setup_matches_oracle(case):
    if case == "c1":
        wl, L = W.c1(), 1
    elif case == "skewed":   # TVB stencil fallback edges and a sliver
        wl, L = W.skewed_patch(N=2), 1
    elif case == "wetdry":
        wl, L = W.small_wetdry(n=12, N=4), 1
    elif case == "barrier":   # tagged internal walls
        wl, L = W.barrier_basin(n=16, N=3), 1
    else:
        wl, L = W.c3(n0=3), 4
    ins = wl.instances[0]
    s = dgswe.Solver([(ins.vx, ins.vy, ins.etov, ins.bc)], wl.N, max_levels=L)
    ref = reference_element(wl.N)
    m = build_mesh(ins.vx, ins.vy, ins.etov, ref, ins.bc)
    etoe, etof = s.connectivity(0)
    assert np.array_equal(etoe, m.etoe)
    assert np.array_equal(etof, m.etof)
    lev, _ = s.levels(0)
    assert np.array_equal(lev.astype(int), assign_levels(m, L))
    if L > 1:
        assert set(np.unique(lev)) == {1, 2, 3, 4}
    x, y = s.node_coords(0)
    assert np.max(np.abs(x - m.x)) < 1e-14
    assert np.max(np.abs(y - m.y)) < 1e-14
    st = tvb_stencil(m)
    pair, alpha = s.tvb_stencil(0)
    assert np.array_equal(pair.astype(int), st.pair)
    # relative: a sliver's wall-mirrored neighbours give weights in the thousands
    assert np.max(np.abs(alpha - st.alpha) / np.maximum(1.0, np.abs(st.alpha))) < 1e-13


def test_boundary_tags():
    """A tagged shared face becomes a wall on both sides (EToE = self);
    tags other than 0 and 1 are mesh errors."""
    wl = W.barrier_basin(n=8, N=2)
    ins = wl.instances[0]
    s = dgswe.Solver([(ins.vx, ins.vy, ins.etov, ins.bc)], 2)
    etoe, etof = s.connectivity(0)
    plain = dgswe.Solver([(ins.vx, ins.vy, ins.etov)], 2)
    etoe0, _ = plain.connectivity(0)
    K = ins.etov.shape[0]
    tagged = ins.bc.astype(bool)
    assert tagged.sum() > 0
    self_ref = etoe == np.arange(K)[:, None]
    assert np.all(self_ref[tagged])                      # tagged faces are walls
    assert np.all(etoe0[tagged] != np.arange(K)[:, None].repeat(3, 1)[tagged])   # they were shared
    assert np.array_equal(etoe[~tagged], etoe0[~tagged])   # the rest is unchanged
    bad = ins.bc.copy()
    bad[0, 0] = 2
    with pytest.raises(dgswe.DGError) as e:
        dgswe.Solver([(ins.vx, ins.vy, ins.etov, bad)], 2)
    assert e.value.code == -2


def test_ensemble_sizes():
    wl = W.c5(n_inst=3, kmin=50, kmax=300)
    s = dgswe.Solver([(i.vx, i.vy, i.etov) for i in wl.instances], 3)
    assert s.Ks == [i.etov.shape[0] for i in wl.instances]
    assert s.K == sum(s.Ks)
    assert s.workspace_bytes > 64 * s.K


def test_error_paths():
    vx = np.array([0.0, 1.0, 0.0, 1.0])
    vy = np.array([0.0, 0.0, 1.0, 1.0])
    with pytest.raises(dgswe.DGError) as e:
        dgswe.Solver([(vx, vy, np.array([[0, 2, 1]]))], 2)        # clockwise
    assert e.value.code == -2
    with pytest.raises(dgswe.DGError) as e:
        dgswe.Solver([(vx, vy, np.array([[0, 1, 2], [1, 0, 3], [0, 1, 3]]))], 2)
    assert e.value.code == -2
    with pytest.raises(dgswe.DGError) as e:
        dgswe.Solver([(vx, vy, np.array([[0, 1, 5]]))], 2)        # vertex out of range
    assert e.value.code == -2
    with pytest.raises(dgswe.DGError) as e:
        dgswe.Solver([(vx, vy, np.array([[0, 1, 2]]))], 9)        # N out of range
    assert e.value.code == -1
    with pytest.raises(dgswe.DGError) as e:
        dgswe.Solver([(vx, vy, np.array([[0, 1, 2]]))], 2, tvb_nu=0.5)
    assert e.value.code == -1
    tri = np.array([[0, 1, 2]])
    for epb in (5, 10, 20, 40):   # launch shapes of the matrix-core kernel (12-lane groups at N = 3)
        dgswe.Solver([(vx, vy, tri)], 3, precision="fused_mfma32", elems_per_block=epb)
    for epb in (4, 8, 16, 32):   # 16-lane groups at N = 4
        dgswe.Solver([(vx, vy, tri)], 4, precision="fused_mfma32", elems_per_block=epb)
    for bad, prec in ((12, "fused_mfma32"), (4, "fused_mfma32"), (16, "fused_fp32"), (-4, "fused_mfma32")):
        with pytest.raises(dgswe.DGError) as e:
            dgswe.Solver([(vx, vy, tri)], 3, precision=prec, elems_per_block=bad)
        assert e.value.code == -1
    dgswe.Solver([(vx, vy, tri)], 3, precision="fused_fp32", elems_per_block=25)   # 256 // Np
    for prec in ("fused_mfma32", "fused_bf16x3", "fused_bf16x6"):   # matrix cores: N <= 5
        dgswe.Solver([(vx, vy, tri)], 5, precision=prec)
        dgswe.Solver([(vx, vy, tri)], 5, precision=prec, elems_per_block=3)   # 21-lane elements
        dgswe.Solver([(vx, vy, tri)], 5, precision=prec, elems_per_block=24)
        for bad in (2, 16, 48):
            with pytest.raises(dgswe.DGError) as e:
                dgswe.Solver([(vx, vy, tri)], 5, precision=prec, elems_per_block=bad)
            assert e.value.code == -1
        with pytest.raises(dgswe.DGError) as e:
            dgswe.Solver([(vx, vy, tri)], 6, precision=prec)
        assert e.value.code == -1
    s = dgswe.Solver([(vx, vy, np.array([[0, 1, 3], [0, 3, 2]]))], 2)
    with pytest.raises(dgswe.DGError) as e:           # no state to tune on
        s.autotune(stream=_NoStream())
    assert e.value.code == -5
    x, _ = s.node_coords(0)
    s.set_bathymetry(0, np.zeros_like(x))
    with pytest.raises(dgswe.DGError) as e:           # nothing bound yet
        s.set_state(0, np.ones_like(x), 0 * x, 0 * x, stream=_NoStream())
    assert e.value.code == -5
    with pytest.raises(dgswe.DGError) as e:
        s.advance(1, stream=_NoStream())
    assert e.value.code == -5


class _NoStream:
    cuda_stream = 0


def test_instance_count_limit(lib):
    """The connectivity record holds the instance id in 23 bits: dg_create
    rejects more instances before it reads any mesh."""
    import ctypes as C
    one = (dgswe.MeshDesc * 1)()
    p = dgswe.default_params(2)
    h = C.c_void_p()
    assert lib.dg_create(one, 2 ** 23 + 1, C.byref(p), C.byref(h)) == -1
    assert b"2^23" in lib.dg_last_error()
    assert not h.value


def test_binding_shape_checks():
    """The binding rejects malformed arrays before they reach the library."""
    vx = np.array([0.0, 1.0, 0.0, 1.0])
    vy = np.array([0.0, 0.0, 1.0, 1.0])
    with pytest.raises(ValueError):
        dgswe.Solver([(vx, vy, np.array([0, 1, 2]))], 2)                      # etov not (K, 3)
    with pytest.raises(ValueError):
        dgswe.Solver([(vx, vy[:3], np.array([[0, 1, 2]]))], 2)               # vx, vy differ
    with pytest.raises(ValueError):
        dgswe.Solver([(vx, vy, np.array([[0, 1, 2]]), np.zeros((1, 2)))], 2)  # bc not (K, 3)
    s = dgswe.Solver([(vx, vy, np.array([[0, 1, 3], [0, 3, 2]]))], 2)
    x, _ = s.node_coords(0)
    with pytest.raises(ValueError):
        s.set_bathymetry(0, np.zeros((x.shape[0], x.shape[1] - 1)))
    with pytest.raises(IndexError):
        s.set_bathymetry(1, np.zeros_like(x))
    s.set_bathymetry(0, np.zeros_like(x))
    with pytest.raises(ValueError):
        s.set_state(0, np.ones_like(x)[:1], 0 * x, 0 * x, stream=_NoStream())


def test_non_finite_bathymetry_rejected():
    vx = np.array([0.0, 1.0, 0.0, 1.0])
    vy = np.array([0.0, 0.0, 1.0, 1.0])
    s = dgswe.Solver([(vx, vy, np.array([[0, 1, 3], [0, 3, 2]]))], 2)
    x, _ = s.node_coords(0)
    B = np.zeros_like(x)
    B[1, 2] = np.nan
    with pytest.raises(dgswe.DGError) as e:
        s.set_bathymetry(0, B)
    assert e.value.code == -6
