"""Pins for the oracle's over-integrated weak form (Section 3, Eq. 3.2 and
the cubature/Gauss rules named after it; Section 7, Volume and Surface
kernels) against what the mathematics fixes: exactness of the rules against
closed-form integrals, the divergence theorem (weak form = strong form for
polynomial fluxes), the C-property with the plain bed source, convergence on
the translating vortex, conservation."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle.overint import conical_cubature, face_gauss_points, overint_operators, rule_points
from oracle.refelem import reference_element
from oracle.swe import Params, Solver


def _triangle_monomial(a: int, b: int) -> float:
    """Integral of r^a s^b over the reference triangle (-1,-1), (1,-1),
    (-1,1): with r = 2x - 1, s = 2y - 1 over the unit simplex (dr ds = 4 dx
    dy) and the Dirichlet integral of x^i y^j = i! j! / (i + j + 2)!."""
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = math.comb(a, i) * math.comb(b, j) * 2 ** (i + j) * (-1) ** (a - i + b - j)
            tot += Fraction(c * math.factorial(i) * math.factorial(j), math.factorial(i + j + 2))
    return float(4 * tot)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_cubature_exact_to_its_degree(N):
    q = rule_points(N)
    assert 2 * q - 1 >= 3 * N
    r, s, w = conical_cubature(q)
    assert r.size == q * q and np.all(w > 0)
    assert np.all(s >= -1) and np.all(r >= -1) and np.all(r + s <= 1e-15)
    for d in range(2 * q):
        for a in range(d + 1):
            exact = _triangle_monomial(a, d - a)
            assert abs(np.sum(w * r ** a * s ** (d - a)) - exact) < 1e-13 * max(1.0, abs(exact)), (a, d - a)
    # one degree beyond: no longer exact for every monomial
    d = 2 * q
    errs = [abs(np.sum(w * r ** a * s ** (d - a)) - _triangle_monomial(a, d - a)) for a in range(d + 1)]
    assert max(errs) > 1e-10


@pytest.mark.parametrize("N", [1, 3, 5])
def test_face_rule_exact_and_on_the_faces(N):
    q = rule_points(N)
    rf, sf, wg = face_gauss_points(q)
    xi = np.linspace(-1, 1, 3)
    for k in range(2 * q):
        t = np.polynomial.legendre.leggauss(q)[0]
        assert abs(np.sum(wg * t ** k) - (0.0 if k % 2 else 2.0 / (k + 1))) < 1e-14
    assert np.allclose(sf[0], -1.0) and np.allclose(rf[1] + sf[1], 0.0) and np.allclose(rf[2], -1.0)
    # counter-clockwise traversal: face 0 left to right, face 1 upwards, face 2 downwards
    assert np.all(np.diff(rf[0]) > 0) and np.all(np.diff(sf[1]) > 0) and np.all(np.diff(sf[2]) < 0)
    # symmetric points: point g of one side is point q-1-g traversed backwards
    assert np.allclose(rf[0], -rf[0][::-1])
    del xi


@pytest.mark.parametrize("N", [2, 3, 4])
def test_operators_reproduce_exact_integrals(N):
    """Pr, Ps, P, L^g against their definitions applied to polynomials: for
    a degree-N nodal f and degree-N fluxes, M P (f at the cubature nodes) is
    the exact integral of f phi_i; M (Pr c1 + Ps c2) + integration by parts
    equals the boundary integral through L^g (divergence theorem)."""
    ref = reference_element(N)
    oi = overint_operators(ref)
    rng = np.random.default_rng(N)
    f = rng.normal(size=ref.Np)
    g1 = rng.normal(size=ref.Np)
    # M P I_c f = M f  (exact integral of f phi_i, degree 2N)
    assert np.allclose(ref.M @ (oi.P @ (oi.Ic @ f)), ref.M @ f, atol=1e-12)
    # divergence theorem on the reference triangle for the field (g1, 0):
    # int dphi/dr g1 = -int phi dg1/dr + boundary int phi g1 n_r
    lhs = ref.M @ (oi.Pr @ (oi.Ic @ g1))
    vol = ref.M @ (ref.Dr @ g1)
    # outward reference normals n_r per face (s = -1: 0; r + s = 0: 1/sqrt2; r = -1: -1)
    # times the reference face Jacobians (1, sqrt2, 1)
    nr_sj = np.repeat([0.0, 1.0, -1.0], oi.NG)
    bnd = ref.M @ (oi.Lg @ (nr_sj * (oi.Ig @ g1)))
    assert np.allclose(lhs, -vol + bnd, atol=1e-11)


def _solver(wl, **kw):
    ins = wl.instances[0]
    return Solver(ins.vx, ins.vy, ins.etov, wl.N, Params(g=wl.g, cfl=wl.cfl, overint=True, **kw))


@pytest.mark.parametrize("N", [2, 3])
def test_weak_form_equals_strong_form_for_polynomial_fluxes(N):
    """Constant depth, linear momentum, flat bed: the fluxes are quadratic
    and continuous, so exact integration makes the weak form equal to the
    strong (nodal) form on interior elements; a transposed, mis-signed or
    mis-scaled operator breaks it."""
    wl = W.lake_at_rest(n=6, N=N)
    ins = wl.instances[0]
    a = Solver(ins.vx, ins.vy, ins.etov, N, Params(overint=True, pp=False, tvb=False))
    b = Solver(ins.vx, ins.vy, ins.etov, N, Params(overint=False, pp=False, tvb=False))
    x, y = a.nodes()
    q = np.stack([np.full_like(x, 1.3), 0.2 + 0.3 * x - 0.1 * y, -0.1 + 0.2 * y + 0.05 * x])
    B = np.zeros_like(x)
    Ra, Rb = a.rhs(q, B), b.rhs(q, B)
    inner = ~a.mesh.wall.any(axis=1)
    assert np.max(np.abs(Ra - Rb)[:, inner]) < 1e-11
    assert np.max(np.abs(Rb[:, inner])) > 1e-2


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_lake_at_rest_with_plain_source(N):
    """C-property through exact integration: still water over a smooth bed
    and over a bed that jumps across every face stays at rest with the plain
    source -g h grad B (no splitting).  The residual is roundoff: 1e-12 of
    the pressure term's own size (the same state over a flat bed)."""
    for wl in (W.lake_at_rest(n=5, N=N), W.stepped_bed("lake", N=N)):
        s = _solver(wl)
        B = s.interpolate(wl.instances[0].bathymetry)
        q = np.stack([np.maximum(1.0 - B, 0.0), 0 * B, 0 * B])
        scale = np.max(np.abs(s.rhs(q, 0 * B)))
        assert np.max(np.abs(s.rhs(q, B))) < 1e-12 * scale


def test_lake_at_rest_needs_the_rule_degree():
    """With a cubature of degree 2N instead of 3N the plain source no longer
    balances the pressure (the products are not integrated exactly)."""
    import oracle.overint as OI
    wl = W.lake_at_rest(n=5, N=3)
    s = _solver(wl)
    B = s.interpolate(wl.instances[0].bathymetry)
    q = np.stack([1.0 - B, 0 * B, 0 * B])
    scale = np.max(np.abs(s.rhs(q, 0 * B)))
    assert np.max(np.abs(s.rhs(q, B))) < 1e-12 * scale
    orig = OI.rule_points
    try:
        OI.rule_points = lambda N: N + 1          # exact to degree 2N + 1 only
        low = _solver(wl)
    finally:
        OI.rule_points = orig
    assert np.max(np.abs(low.rhs(q, B))) > 1e-8 * scale


def test_rhs_conserves_mass_with_walls():
    wl = W.small_wetdry(n=6, N=3)
    s = _solver(wl)
    x, y = s.nodes()
    rng = np.random.default_rng(0)
    q = np.stack([0.5 + rng.uniform(0, 0.5, x.shape), rng.normal(0, 0.3, x.shape), rng.normal(0, 0.3, x.shape)])
    B = s.interpolate(wl.instances[0].bathymetry)
    R = s.rhs(q, B)
    total = np.sum(s.mesh.J * (R[0] @ s.ref.w))
    scale = np.sum(s.mesh.J * (np.abs(R[0]) @ s.ref.w))
    assert abs(total) < 1e-13 * scale


@pytest.mark.parametrize("N", [2, 3])
def test_vortex_convergence_order_overint(N):
    """Translating vortex (g = 2, exact Dirichlet data, limiters off) with
    the over-integrated operators: least-squares EOC of the depth error at
    least N + 1/2 - 0.2 (Table 6.1's smooth-flow orders)."""
    beta = 5.0

    def exact(x, y, t):
        xx = x - t
        r2 = xx ** 2 + y ** 2
        h = 1 - beta ** 2 / (32 * np.pi ** 2) * np.exp(2 * (1 - r2))
        u = 1 - beta * np.exp(1 - r2) * y / (2 * np.pi)
        v = beta * np.exp(1 - r2) * xx / (2 * np.pi)
        return h, h * u, h * v

    T = 0.25
    errs, Hs = [], []
    for n in (10, 20, 40):
        vx, vy, etov = W.structured_mesh(int(1.5 * n), int(1.2 * n), -5, 10, -6, 6)
        s = Solver(vx, vy, etov, N, Params(g=2.0, cfl=0.5, pp=False, tvb=False, overint=True), ghost=exact)
        x, y = s.nodes()
        s.set_state(*exact(x, y, 0.0), 0 * x)
        nst = int(np.ceil(T / s.dt_min))
        dt = T / nst
        s.dt_min = dt
        for _ in range(nst):
            s.step()
        he = exact(x, y, T)[0]
        e = s.q[0] - he
        errs.append(np.sqrt(np.sum(s.mesh.J * np.einsum("ki,ij,kj->k", e, s.ref.M, e))))
        Hs.append(15.0 / (1.5 * n))
    p = np.polyfit(np.log(Hs), np.log(errs), 1)[0]
    assert p >= N + 0.5 - 0.2, (errs, p)


@pytest.mark.parametrize("N", [1, 3])
def test_wetdry_ledge_overint(N):
    """The ledge over a stepped bed (a dry bed above the wet neighbours'
    surface) with both limiters: mass conserved, depths non-negative."""
    wl = W.stepped_bed("ledge", N=N)
    s = _solver(wl)
    x, y = s.nodes()
    ins = wl.instances[0]
    s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry))
    m0 = s.mass()
    s.run(100)
    assert abs(s.mass() - m0) <= 1e-13 * m0
    assert s.q[0].min() >= 0.0
