"""Pins for the oracle's reference element against closed forms and textbook
routines (nodal DG on triangles, Section 3)."""
import itertools
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

from oracle.refelem import reference_element

NS = [1, 2, 3, 4, 5]


def tri_integral(a: int, b: int) -> float:
    """Exact integral of r^a s^b over the reference triangle (-1,-1),(1,-1),(-1,1)
    via r = 2 xi - 1, s = 2 eta - 1 and int xi^i eta^j = i! j! / (i+j+2)!."""
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = comb(a, i) * comb(b, j) * 2 ** (i + j) * (-1) ** (a - i + b - j)
            tot += c * Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    return float(4 * tot)


@pytest.mark.parametrize("N", NS)
def test_differentiation_exact_on_monomials(N):
    re = reference_element(N)
    r, s = re.r, re.s
    for a in range(N + 1):
        for b in range(N + 1 - a):
            f = r ** a * s ** b
            dfr = a * r ** (a - 1) * s ** b if a > 0 else 0 * r
            dfs = b * r ** a * s ** (b - 1) if b > 0 else 0 * r
            assert np.max(np.abs(re.Dr @ f - dfr)) < 1e-12
            assert np.max(np.abs(re.Ds @ f - dfs)) < 1e-12
    assert np.max(np.abs(re.Dr @ np.ones(re.Np))) < 1e-13


@pytest.mark.parametrize("N", NS)
def test_mass_matrix_integrates_products(N):
    re = reference_element(N)
    r, s = re.r, re.s
    assert abs(re.w.sum() - 2.0) < 1e-13
    mons = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    for (a1, b1), (a2, b2) in itertools.product(mons, mons):
        u = r ** a1 * s ** b1
        v = r ** a2 * s ** b2
        assert abs(u @ re.M @ v - tri_integral(a1 + a2, b1 + b2)) < 1e-12
    for (a, b) in mons:
        assert abs(re.w @ (r ** a * s ** b) - tri_integral(a, b)) < 1e-13


@pytest.mark.parametrize("N", NS)
def test_face_nodes_are_gll(N):
    re = reference_element(N)
    leg = np.polynomial.legendre.Legendre.basis(N).deriv().roots() if N > 1 else np.array([])
    gll = np.sort(np.concatenate([[-1.0, 1.0], np.real(leg)]))
    # face 0: s = -1 parameter r; face 1: parameter s; face 2: parameter -s
    t0 = re.r[re.fmask[0]]
    t1 = re.s[re.fmask[1]]
    t2 = -re.s[re.fmask[2]]
    for t in (t0, t1, t2):
        assert np.max(np.abs(t - gll)) < 1e-14
    # faces are traversed counter-clockwise: vertex f -> vertex f+1
    assert re.fmask[0][0] == re.fmask[2][-1]
    assert re.fmask[0][-1] == re.fmask[1][0]
    assert re.fmask[1][-1] == re.fmask[2][0]


@pytest.mark.parametrize("N", NS)
def test_node_set_symmetric(N):
    re = reference_element(N)
    lam = np.stack([-(re.r + re.s) / 2, (1 + re.r) / 2, (1 + re.s) / 2], axis=1)
    key = {tuple(np.round(l, 12)) for l in lam}
    for perm in itertools.permutations(range(3)):
        assert {tuple(np.round(l[list(perm)], 12)) for l in lam} == key


def test_low_order_nodes_closed_form():
    re1 = reference_element(1)
    assert np.allclose(np.stack([re1.r, re1.s], 1), [[-1, -1], [1, -1], [-1, 1]], atol=1e-15)
    re2 = reference_element(2)
    pts = {tuple(np.round(p, 14)) for p in np.stack([re2.r, re2.s], 1)}
    assert pts == {(-1.0, -1.0), (0.0, -1.0), (1.0, -1.0), (-1.0, 0.0), (0.0, 0.0), (-1.0, 1.0)}


@pytest.mark.parametrize("N", NS)
def test_lift_matches_integration_by_parts(N):
    """M Dr + Dr^T M equals the boundary form sum_f n_r,f sJ_f (face mass), which
    is M LIFT applied to n_r sJ times the face traces (independent routes: Dr from
    basis gradients, LIFT from the 1D face mass matrix)."""
    re = reference_element(N)
    Nfp = re.Nfp
    nr = [0.0, 1.0, -1.0]          # reference outward normals times face length/2
    ns = [-1.0, 1.0, 0.0]
    fm = re.fmask.reshape(-1)
    P = np.zeros((3 * Nfp, re.Np))
    P[np.arange(3 * Nfp), fm] = 1.0
    Dnr = np.repeat(nr, Nfp)
    Dns = np.repeat(ns, Nfp)
    lhs_r = re.M @ re.Dr + re.Dr.T @ re.M
    lhs_s = re.M @ re.Ds + re.Ds.T @ re.M
    rhs_r = re.M @ re.LIFT @ (Dnr[:, None] * P)
    rhs_s = re.M @ re.LIFT @ (Dns[:, None] * P)
    assert np.max(np.abs(lhs_r - rhs_r)) < 1e-12
    assert np.max(np.abs(lhs_s - rhs_s)) < 1e-12


@pytest.mark.parametrize("N", NS)
def test_p1_tools(N):
    re = reference_element(N)
    r, s = re.r, re.s
    lin = 0.3 - 1.7 * r + 0.6 * s
    assert np.max(np.abs(re.proj1 @ lin - lin)) < 1e-13
    verts = np.array([[-1, -1], [1, -1], [-1, 1]], float)
    assert np.max(np.abs(re.p1_vert @ lin - (0.3 - 1.7 * verts[:, 0] + 0.6 * verts[:, 1]))) < 1e-13
    mids = 0.5 * (verts + np.roll(verts, -1, 0))
    assert np.max(np.abs(re.p1_mid @ lin - (0.3 - 1.7 * mids[:, 0] + 0.6 * mids[:, 1]))) < 1e-13
    # L2 projection of a degree-N function by the normal equations on [1, r, s]
    u = np.cos(1.3 * r + 0.4) * np.exp(0.5 * s)
    L = np.stack([np.ones_like(r), r, s], 1)
    c = np.linalg.solve(L.T @ re.M @ L, L.T @ re.M @ u)
    if N >= 1:
        uh = u  # nodal interpolant
        assert np.max(np.abs(re.proj1 @ uh - L @ c)) < 1e-12
    # midpoint-Lagrange basis: phi_i(m_j) = delta_ij, each phi linear
    for i in range(3):
        assert np.max(np.abs(re.proj1 @ re.phi_mid[i] - re.phi_mid[i])) < 1e-13
        assert np.max(np.abs(re.p1_mid @ re.phi_mid[i] - np.eye(3)[i])) < 1e-13
    # the mean of the P1 projection equals the mean
    assert abs(re.w @ (re.proj1 @ u) - re.w @ u) < 1e-13
