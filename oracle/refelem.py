"""Reference triangle of the nodal DG discretisation (oracle, FP64).

Test infrastructure only (see the package header).

Section 3 of the paper: the solution on each triangle is a Lagrange
polynomial of degree N on Warp & Blend interpolation nodes (the node family
of Hesthaven & Warburton's book cited there).  Under the nodal-collocation
reading of the volume and surface terms the operators needed are:

* ``Dr``, ``Ds``  - nodal differentiation matrices on the reference triangle
  with vertices (-1,-1), (1,-1), (-1,1);
* ``M``           - nodal mass matrix;
* ``LIFT``        - M^{-1} E, with E the face mass matrices of the three
  faces (1D mass matrix on the Gauss-Lobatto face nodes);
* ``w``           - cell-mean weights, w = M 1, so that w.u = integral of u;
* P1 tools for the limiters of Section 5.2/5.3: L2 projection onto linear
  polynomials by modal truncation, its values at the vertices and at the
  edge midpoints, and the edge-midpoint Lagrange basis evaluated at the nodes.

Face f joins local vertices f and f+1 (mod 3); the face nodes are listed in
counter-clockwise traversal order, so a face shared by two counter-clockwise
elements is traversed in opposite directions and node j on one side meets
node Nfp-1-j on the other.

Numerics: Jacobi polynomials and Gauss-Jacobi roots come from SciPy
(``eval_jacobi``, ``roots_jacobi``) with the closed-form norm; Lagrange
interpolation in the warp function uses the product formula.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import eval_jacobi, gammaln, roots_jacobi

# Optimised blending parameters of the Warp & Blend family for N = 1..15
# (as tabulated in the node-construction chapter of the book the paper cites);
# any fixed value gives a valid node set, both sides of every parity test use
# these.
ALPHA_OPT = [0.0, 0.0, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832, 1.3648,
             1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258]


def jacobi_norm2(n: int, a: float, b: float) -> float:
    """Squared weighted L2 norm of the classical Jacobi polynomial P_n^{(a,b)}."""
    lg = (gammaln(n + a + 1) + gammaln(n + b + 1) - gammaln(n + a + b + 1) - gammaln(n + 1))
    return 2.0 ** (a + b + 1) / (2 * n + a + b + 1) * np.exp(lg)


def jacobi(x, a: float, b: float, n: int) -> np.ndarray:
    """Orthonormal Jacobi polynomial (weight (1-x)^a (1+x)^b on [-1,1])."""
    x = np.asarray(x, dtype=np.float64)
    return eval_jacobi(n, a, b, x) / np.sqrt(jacobi_norm2(n, a, b))


def jacobi_deriv(x, a: float, b: float, n: int) -> np.ndarray:
    """Derivative of :func:`jacobi`: d/dx P_n^{(a,b)} = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return 0.5 * (n + a + b + 1) * eval_jacobi(n - 1, a + 1, b + 1, x) / np.sqrt(
        jacobi_norm2(n, a, b))


def gll_nodes(N: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre nodes on [-1,1]: the endpoints and the roots of
    P_N' (= Gauss-Jacobi(1,1) nodes of degree N-1), ascending."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = roots_jacobi(N - 1, 1.0, 1.0)[0]
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


def warp_factor(N: int, rout: np.ndarray) -> np.ndarray:
    """Warp of the equidistant edge nodes onto the GLL nodes, interpolated at
    ``rout`` and divided by the edge blend 1 - r^2 (zero at the end points)."""
    rout = np.asarray(rout, dtype=np.float64)
    r_gll = gll_nodes(N)
    r_eq = np.linspace(-1.0, 1.0, N + 1)
    warp = np.zeros_like(rout)
    for i in range(N + 1):
        li = np.ones_like(rout)
        for j in range(N + 1):
            if j != i:
                li = li * (rout - r_eq[j]) / (r_eq[i] - r_eq[j])
        warp = warp + (r_gll[i] - r_eq[i]) * li
    interior = np.abs(rout) < 1.0 - 1.0e-10
    return np.where(interior, warp / np.where(interior, 1.0 - rout ** 2, 1.0), 0.0)


def warp_blend_nodes(N: int):
    """Warp & Blend nodes on the reference triangle, returned as (r, s).

    Built on the equilateral triangle from barycentric equidistant nodes
    (row by row: L1 = n/N outer, L3 = m/N inner), each edge's 1D warp blended
    into the interior with 4 L_a L_b (1 + (alpha L_c)^2), then mapped to the
    reference triangle.  Node order: rows of increasing s, r increasing
    within a row.
    """
    alpha = ALPHA_OPT[N - 1] if N <= len(ALPHA_OPT) else 5.0 / 3.0
    L1, L3 = [], []
    for n in range(N + 1):
        for m in range(N + 1 - n):
            L1.append(n / N)
            L3.append(m / N)
    L1 = np.array(L1)
    L3 = np.array(L3)
    L2 = 1.0 - L1 - L3
    x = -L2 + L3
    y = (-L2 - L3 + 2.0 * L1) / np.sqrt(3.0)
    blend1 = 4.0 * L2 * L3
    blend2 = 4.0 * L1 * L3
    blend3 = 4.0 * L1 * L2
    w1 = blend1 * warp_factor(N, L3 - L2) * (1.0 + (alpha * L1) ** 2)
    w2 = blend2 * warp_factor(N, L1 - L3) * (1.0 + (alpha * L2) ** 2)
    w3 = blend3 * warp_factor(N, L2 - L1) * (1.0 + (alpha * L3) ** 2)
    x = x + w1 + np.cos(2.0 * np.pi / 3.0) * w2 + np.cos(4.0 * np.pi / 3.0) * w3
    y = y + np.sin(2.0 * np.pi / 3.0) * w2 + np.sin(4.0 * np.pi / 3.0) * w3
    # equilateral (x,y) -> barycentric -> reference (r,s)
    l1 = (np.sqrt(3.0) * y + 1.0) / 3.0
    l2 = (-3.0 * x - np.sqrt(3.0) * y + 2.0) / 6.0
    l3 = (3.0 * x - np.sqrt(3.0) * y + 2.0) / 6.0
    r = -l2 + l3 - l1
    s = -l2 - l3 + l1
    return r, s


def _collapse(r, s):
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    top = np.abs(s - 1.0) < 1e-14
    a = np.where(top, -1.0, 2.0 * (1.0 + r) / np.where(top, 1.0, 1.0 - s) - 1.0)
    return a, s


def mode_list(N: int):
    """Orthonormal-basis mode indices (i, j), i+j <= N, i outer."""
    return [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]


def basis(r, s, i: int, j: int) -> np.ndarray:
    """Orthonormal Koornwinder-Dubiner mode
    psi_ij = sqrt(2) P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i on the reference triangle."""
    a, b = _collapse(r, s)
    return np.sqrt(2.0) * jacobi(a, 0, 0, i) * jacobi(b, 2 * i + 1, 0, j) * (1.0 - b) ** i


def basis_grad(r, s, i: int, j: int):
    """(d/dr, d/ds) of :func:`basis` by the chain rule through a = 2(1+r)/(1-s)-1, b = s."""
    a, b = _collapse(r, s)
    fa = jacobi(a, 0, 0, i)
    dfa = jacobi_deriv(a, 0, 0, i)
    gb = jacobi(b, 2 * i + 1, 0, j)
    dgb = jacobi_deriv(b, 2 * i + 1, 0, j)
    if i == 0:
        dr = np.zeros_like(a)
        ds = gb * 0.0 + fa * dgb
    else:
        om = 1.0 - b
        dr = 2.0 * dfa * gb * om ** (i - 1)
        ds = dfa * gb * (1.0 + a) * om ** (i - 1) + fa * dgb * om ** i - i * fa * gb * om ** (i - 1)
    return np.sqrt(2.0) * dr, np.sqrt(2.0) * ds


def vandermonde(N: int, r, s) -> np.ndarray:
    return np.stack([basis(r, s, i, j) for (i, j) in mode_list(N)], axis=1)


def grad_vandermonde(N: int, r, s):
    gr, gs = [], []
    for (i, j) in mode_list(N):
        dr, ds = basis_grad(r, s, i, j)
        gr.append(dr)
        gs.append(ds)
    return np.stack(gr, axis=1), np.stack(gs, axis=1)


VERTICES = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
MIDPOINTS = 0.5 * (VERTICES + np.roll(VERTICES, -1, axis=0))   # midpoint of face f


@dataclass
class RefElement:
    N: int
    Np: int
    Nfp: int
    r: np.ndarray
    s: np.ndarray
    V: np.ndarray
    Dr: np.ndarray
    Ds: np.ndarray
    M: np.ndarray
    fmask: np.ndarray        # (3, Nfp) volume-node index of face node j of face f
    LIFT: np.ndarray         # (Np, 3*Nfp)
    w: np.ndarray            # (Np,) cell-integral weights, sum = 2
    proj1: np.ndarray        # (Np, Np) nodal P1 L2 projection
    p1_vert: np.ndarray      # (3, Np) values of the P1 projection at the vertices
    p1_mid: np.ndarray       # (3, Np) values of the P1 projection at the face midpoints
    phi_mid: np.ndarray      # (3, Np) midpoint-Lagrange P1 basis phi_i at the nodes
    bary: np.ndarray         # (3, Np) barycentric coordinates of the nodes
    gll: np.ndarray          # (Nfp,) GLL nodes


def reference_element(N: int) -> RefElement:
    if N < 1:
        raise ValueError("N >= 1")
    Np = (N + 1) * (N + 2) // 2
    Nfp = N + 1
    r, s = warp_blend_nodes(N)
    V = vandermonde(N, r, s)
    Vr, Vs = grad_vandermonde(N, r, s)
    Vinv = np.linalg.inv(V)
    Dr = Vr @ Vinv
    Ds = Vs @ Vinv
    M = Vinv.T @ Vinv
    tol = 1e-10
    f0 = np.where(np.abs(s + 1.0) < tol)[0]
    f0 = f0[np.argsort(r[f0])]
    f1 = np.where(np.abs(r + s) < tol)[0]
    f1 = f1[np.argsort(s[f1])]
    f2 = np.where(np.abs(r + 1.0) < tol)[0]
    f2 = f2[np.argsort(-s[f2])]
    fmask = np.stack([f0, f1, f2]).astype(np.int64)
    if fmask.shape != (3, Nfp):
        raise RuntimeError("face node detection failed")
    gll = gll_nodes(N)
    # 1D mass matrix on the face GLL nodes (face parameter in [-1, 1])
    V1 = np.stack([jacobi(gll, 0, 0, n) for n in range(Nfp)], axis=1)
    V1inv = np.linalg.inv(V1)
    M1 = V1inv.T @ V1inv
    E = np.zeros((Np, 3 * Nfp))
    for f in range(3):
        for a in range(Nfp):
            E[fmask[f, a], f * Nfp:(f + 1) * Nfp] = M1[a]
    LIFT = V @ (V.T @ E)
    w = M @ np.ones(Np)
    modes = mode_list(N)
    lin = [modes.index((0, 0)), modes.index((0, 1)), modes.index((1, 0))]
    D1 = np.zeros((Np, Np))
    for m in lin:
        D1[m, m] = 1.0
    proj1 = V @ D1 @ Vinv
    Vv = vandermonde(N, VERTICES[:, 0], VERTICES[:, 1])
    Vm = vandermonde(N, MIDPOINTS[:, 0], MIDPOINTS[:, 1])
    p1_vert = Vv @ D1 @ Vinv
    p1_mid = Vm @ D1 @ Vinv
    bary = np.stack([-(r + s) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0])
    # phi_i = 1 at the midpoint of face i, 0 at the other two: 1 - 2*lambda_(opposite vertex)
    phi_mid = np.stack([1.0 - 2.0 * bary[(i + 2) % 3] for i in range(3)])
    return RefElement(N, Np, Nfp, r, s, V, Dr, Ds, M, fmask, LIFT, w, proj1, p1_vert,
                      p1_mid, phi_mid, bary, gll)
