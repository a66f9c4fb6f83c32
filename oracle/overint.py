"""Over-integrated weak-form operators of the paper's DG discretisation
(oracle, FP64).

Test infrastructure only (see the package header).

Section 3 (Eq. 3.2, and the sentence after it): the weak form

    (dQ/dt, phi) = (dphi/dx, F) + (dphi/dy, G) - (F* nx + G* ny, phi)_dK + (S, phi)

with the volume integrals evaluated by a cubature rule on the triangle and
the face integrals by Gauss quadrature; Section 7 (Volume and Surface
kernels): with affine elements this is

    N(Q) = Pr cF1 + Ps cF2 + P cS,          S(Q) = -L^g Fn*^g,

cF1 = rx F + ry G and cF2 = sx F + sy G the contravariant fluxes and cS the
source at the cubature nodes, Fn*^g the numerical flux at the Gauss nodes
scaled by the face Jacobian over the element Jacobian, and

    Pr = M^-1 Dr_c^T W,  Ps = M^-1 Ds_c^T W,  P = M^-1 I_c^T W,
    L^g = M^-1 [I_g0^T W_g, I_g1^T W_g, I_g2^T W_g],

where I_c, Dr_c, Ds_c evaluate the nodal basis and its r, s derivatives at
the cubature nodes, W and W_g are the cubature and Gauss weights and I_gf
evaluates the nodal basis at the Gauss nodes of face f.

Rules (the paper cites a compendium of triangle cubatures without naming a
rule or its degree): both are exact for polynomials of degree 3N, enough for
every product of three degree-N polynomials less one derivative in the
volume (flux times test-function gradient, depth times bed slope times test
function) and of three degree-N polynomials on a face, so that the lake at
rest is a discrete steady state with the plain source -g h grad B.

* cubature: the conical-product (collapsed-coordinate) rule of Stroud: q
  Gauss-Legendre points in a, q Gauss-Jacobi (1, 0) points in b, with
  r = (1 + a)(1 - b)/2 - 1, s = b; exact to degree 2q - 1, q = ceil((3N+1)/2);
* faces: q Gauss-Legendre points on [-1, 1] per face (exact to 2q - 1),
  listed in the counter-clockwise traversal of the face, so Gauss point g of
  one side meets point q - 1 - g of the other.

Gauss-Legendre and Gauss-Jacobi nodes and weights come from SciPy.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import roots_jacobi, roots_legendre

from .refelem import VERTICES, grad_vandermonde, vandermonde


def rule_points(N: int) -> int:
    """Points per direction (cubature) and per face (Gauss): exact to degree 3N."""
    return (3 * N + 2) // 2


def conical_cubature(q: int):
    """Stroud's conical product rule on the reference triangle with q points
    per direction: (r, s, w), exact for total degree <= 2q - 1, sum w = 2."""
    a, wa = roots_legendre(q)
    b, wb = roots_jacobi(q, 1.0, 0.0)      # weight (1 - b)
    A, Bb = np.meshgrid(a, b, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    r = 0.5 * (1.0 + A) * (1.0 - Bb) - 1.0
    s = Bb
    w = 0.5 * WA * WB                      # dr ds = (1 - b)/2 da db
    return r.ravel(), s.ravel(), w.ravel()


def face_gauss_points(q: int):
    """Reference coordinates (3, q) of the q Gauss-Legendre points on each
    face f (from vertex f to vertex f+1), and the weights on [-1, 1]."""
    xi, wg = roots_legendre(q)
    rf = np.empty((3, q))
    sf = np.empty((3, q))
    for f in range(3):
        v0, v1 = VERTICES[f], VERTICES[(f + 1) % 3]
        t = 0.5 * (1.0 + xi)
        rf[f] = v0[0] + t * (v1[0] - v0[0])
        sf[f] = v0[1] + t * (v1[1] - v0[1])
    return rf, sf, wg


@dataclass
class OverIntOps:
    q: int                 # points per cubature direction and per face
    Ncub: int
    NG: int                # Gauss points per face
    rc: np.ndarray
    sc: np.ndarray
    wc: np.ndarray         # (Ncub,) cubature weights
    Ic: np.ndarray         # (Ncub, Np) basis values at the cubature nodes
    Drc: np.ndarray        # (Ncub, Np) r-derivatives there
    Dsc: np.ndarray        # (Ncub, Np)
    Pr: np.ndarray         # (Np, Ncub)
    Ps: np.ndarray         # (Np, Ncub)
    P: np.ndarray          # (Np, Ncub)
    wg: np.ndarray         # (NG,) Gauss weights on [-1, 1]
    Ig: np.ndarray         # (3*NG, Np) basis values at the Gauss nodes of the faces
    Lg: np.ndarray         # (Np, 3*NG)


def overint_operators(ref) -> OverIntOps:
    N, Np = ref.N, ref.Np
    q = rule_points(N)
    rc, sc, wc = conical_cubature(q)
    Vinv = np.linalg.inv(ref.V)
    Ic = vandermonde(N, rc, sc) @ Vinv
    Vrc, Vsc = grad_vandermonde(N, rc, sc)
    Drc = Vrc @ Vinv
    Dsc = Vsc @ Vinv
    Minv = np.linalg.inv(ref.M)
    W = np.diag(wc)
    Pr = Minv @ Drc.T @ W
    Ps = Minv @ Dsc.T @ W
    P = Minv @ Ic.T @ W
    rf, sf, wg = face_gauss_points(q)
    Ig = vandermonde(N, rf.ravel(), sf.ravel()) @ Vinv
    Wg = np.diag(np.tile(wg, 3))
    Lg = Minv @ Ig.T @ Wg
    return OverIntOps(q, q * q, q, rc, sc, wc, Ic, Drc, Dsc, Pr, Ps, P, wg, Ig, Lg)


def gauss_exterior_map(mesh, NG: int) -> np.ndarray:
    """Flat index (into a (K, 3*NG) array) of the exterior Gauss point of
    every Gauss point: point g of face f of element k meets point NG-1-g of
    face EToF of element EToE (walls: the point itself)."""
    K = mesh.K
    out = np.empty((K, 3 * NG), dtype=np.int64)
    ks = np.arange(K)
    for f in range(3):
        nb = mesh.etoe[:, f]
        f2 = mesh.etof[:, f]
        for g in range(NG):
            own = ks * 3 * NG + f * NG + g
            other = nb * 3 * NG + f2 * NG + (NG - 1 - g)
            out[:, f * NG + g] = np.where(mesh.wall[:, f], own, other)
    return out
