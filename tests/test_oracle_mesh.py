"""Pins for the oracle's mesh data: connectivity, geometry, levels, TVB stencil."""
import numpy as np
import pytest

import workloads as W
from oracle.mesh import MeshError, assign_levels, build_mesh, connect, tvb_stencil
from oracle.refelem import reference_element


def _mesh(n=6, jitter=0.2, seed=3, N=3):
    rng = np.random.default_rng(seed)
    vx, vy, etov = W.structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0, jitter=jitter, rng=rng)
    return build_mesh(vx, vy, etov, reference_element(N))


def test_euler_characteristic_and_pairing():
    m = _mesh()
    K = m.K
    n_int = int((~m.wall).sum())
    n_bnd = int(m.wall.sum())
    E = n_int // 2 + n_bnd
    V = m.vx.size
    assert V - E + K == 1
    for k in range(K):
        for f in range(3):
            if m.wall[k, f]:
                assert m.etoe[k, f] == k and m.etof[k, f] == f
            else:
                k2, f2 = m.etoe[k, f], m.etof[k, f]
                assert m.etoe[k2, f2] == k and m.etof[k2, f2] == f
                assert k2 != k


def test_paired_face_nodes_coincide():
    m = _mesh(N=4)
    ref = reference_element(4)
    fm = ref.fmask.reshape(-1)
    xM = m.x[:, fm]
    yM = m.y[:, fm]
    xP = m.x.reshape(-1)[m.vmapP]
    yP = m.y.reshape(-1)[m.vmapP]
    inner = ~np.repeat(m.wall, ref.Nfp, axis=1)
    assert inner.sum() > 0
    assert np.max(np.abs(xM - xP)[inner]) < 1e-14
    assert np.max(np.abs(yM - yP)[inner]) < 1e-14


def test_geometry():
    m = _mesh()
    assert abs(np.sum(2.0 * m.J) - 1.0) < 1e-13          # total area
    assert np.allclose(np.hypot(m.nx, m.ny), 1.0, atol=1e-15)
    k2 = m.etoe
    f2 = m.etof
    inner = ~m.wall
    assert np.max(np.abs((m.nx + m.nx[k2, f2])[inner])) < 1e-14
    assert np.max(np.abs((m.ny + m.ny[k2, f2])[inner])) < 1e-14
    # metric identities: d(x)/dx = 1 via the mapping of the vertices
    x1 = m.vx[m.etov[:, 0]]
    x2 = m.vx[m.etov[:, 1]]
    x3 = m.vx[m.etov[:, 2]]
    xr, xs = (x2 - x1) / 2, (x3 - x1) / 2
    assert np.allclose(m.rx * xr + m.sx * xs, 1.0, atol=1e-12)
    # inradius of a right isosceles triangle with legs a: a (2 - sqrt2) / 2
    mm = _mesh(n=4, jitter=0.0)
    assert np.allclose(mm.inradius, 0.25 * (2 - np.sqrt(2)) / 2, atol=1e-15)


def test_broken_meshes_raise():
    vx = np.array([0.0, 1.0, 0.0, 1.0])
    vy = np.array([0.0, 0.0, 1.0, 1.0])
    ref = reference_element(1)
    with pytest.raises(MeshError):
        build_mesh(vx, vy, np.array([[0, 2, 1]]), ref)       # clockwise
    with pytest.raises(MeshError):
        connect(np.array([[0, 1, 2], [1, 0, 3], [0, 1, 3]]))   # face shared three times


def test_levels_graded_bands():
    wl = W.c3(n0=4)
    inst = wl.instances[0]
    ref = reference_element(3)
    m = build_mesh(inst.vx, inst.vy, inst.etov, ref)
    lev = assign_levels(m, 4)
    assert lev.min() == 1 and lev.max() == 4
    xc = m.vx[m.etov].mean(axis=1)
    band = np.floor(xc).astype(int)
    # regular two-triangle cells keep their band's level 4 - b; in each
    # transition cell the two small triangles go one level finer.
    area = 2.0 * m.J
    for b in range(4):
        sel = band == b
        h = 1.0 / (4 * 2 ** b)
        regular = np.isclose(area, 0.5 * h * h) & sel
        assert np.all(lev[regular] == 4 - b)
        small = np.isclose(area, 0.25 * h * h) & sel
        if b < 3:
            assert small.sum() == 2 * 4 * 2 ** b
            assert np.all(lev[small] == 3 - b)
    # 2:1 grading across faces
    assert np.all(np.abs(lev[:, None] - lev[m.etoe]) <= 1)
    # single rate: everything at level 1
    assert np.all(assign_levels(m, 1) == 1)


def test_levels_smoothing_fixed_point():
    # a single tiny element in a coarse mesh forces its neighbourhood down
    vx, vy, etov = W.structured_mesh(8, 8, 0.0, 1.0, 0.0, 1.0)
    vx = vx.copy()
    c = 4 * 9 + 4                      # interior vertex (4,4)
    vx[c] += 0.115                     # squeeze elements touching the vertex
    m = build_mesh(vx, vy, etov, reference_element(2))
    lev = assign_levels(m, 6)
    assert np.all(np.abs(lev[:, None] - lev[m.etoe]) <= 1)
    r = m.inradius
    raw = 1 + np.floor(np.log2(r / r.min() * (1 + 1e-12))).astype(int)
    raw = np.minimum(raw, 6)
    # smoothing only lowers levels, and the result is min_j (raw_j + graph distance)
    assert np.all(lev <= raw)
    K = m.K
    dist = np.full((K, K), 10 ** 6)
    for k in range(K):
        dist[k, k] = 0
        frontier = [k]
        while frontier:
            nxt = []
            for a in frontier:
                for b in m.etoe[a]:
                    if dist[k, b] > dist[k, a] + 1:
                        dist[k, b] = dist[k, a] + 1
                        nxt.append(b)
            frontier = nxt
    assert np.array_equal(lev, np.min(raw[None, :] + dist, axis=1))


def test_tvb_stencil_reconstructs_linear_functions():
    m = _mesh(n=8)
    st = tvb_stencil(m)
    px = m.vx[m.etov]
    py = m.vy[m.etov]
    b0 = np.stack([px.mean(1), py.mean(1)], 1)
    mid = np.stack([0.5 * (px + np.roll(px, -1, 1)), 0.5 * (py + np.roll(py, -1, 1))], 2)
    nb = b0[m.etoe]
    interior = ~m.wall.any(axis=1)
    for i in range(3):
        pj, pk = st.pair[:, i, 0], st.pair[:, i, 1]
        aj, ak = st.alpha[:, i, 0], st.alpha[:, i, 1]
        K = m.K
        rec = aj[:, None] * (nb[np.arange(K), pj] - b0) + ak[:, None] * (nb[np.arange(K), pk] - b0)
        valid = interior & (pj != pk)
        assert np.max(np.abs((rec - (mid[:, i] - b0))[valid])) < 1e-13
        assert np.all(st.alpha[valid, i] >= -1e-10)
        assert np.allclose(np.linalg.norm(st.direction[:, i], axis=1), 1.0)
    # most interior edges find a valid pair on a jittered mesh
    assert np.mean(st.pair[interior, :, 0] != st.pair[interior, :, 1]) > 0.9


def test_tvb_stencil_fallback_on_skewed_neighbourhood():
    """Where the neighbour barycentres do not surround the element's own, no
    pair of them spans the direction to an edge midpoint with non-negative
    weights; that edge falls back to its face neighbour alone, with the weight
    that gives the neighbour direction the length of the midpoint offset."""
    wl = W.skewed_patch(N=2)
    ins = wl.instances[0]
    m = build_mesh(ins.vx, ins.vy, ins.etov, reference_element(2))
    st = tvb_stencil(m)
    px, py = m.vx[m.etov], m.vy[m.etov]
    b0 = np.stack([px.mean(1), py.mean(1)], 1)
    mid = np.stack([0.5 * (px + np.roll(px, -1, 1)), 0.5 * (py + np.roll(py, -1, 1))], 2)
    fb = st.pair[:, :, 0] == st.pair[:, :, 1]
    assert fb[0].tolist() == [True, False, True]
    for i in (0, 2):
        # no pair spans the offset with non-negative weights
        d = mid[0, i] - b0[0]
        nb = b0[m.etoe[0]] - b0[0]
        for j, k in ((0, 1), (0, 2), (1, 2)):
            w = np.linalg.solve(np.stack([nb[j], nb[k]], 1), d)
            assert w.min() < 0
        assert st.alpha[0, i, 1] == 0.0
        assert abs(st.alpha[0, i, 0] * np.linalg.norm(nb[i]) - np.linalg.norm(d)) < 1e-14
    # the middle edge spans exactly
    rec = st.alpha[0, 1, 0] * (b0[m.etoe[0, st.pair[0, 1, 0]]] - b0[0]) + \
        st.alpha[0, 1, 1] * (b0[m.etoe[0, st.pair[0, 1, 1]]] - b0[0])
    assert np.max(np.abs(rec - (mid[0, 1] - b0[0]))) < 1e-14
