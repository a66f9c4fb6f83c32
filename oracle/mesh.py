"""Mesh data of the nodal DG discretisation (oracle, FP64).

Test infrastructure only (see the package header).

* Connectivity of a conforming triangulation (Section 3): face f of element
  k joins vertices (v_f, v_{f+1}); two faces match when they share the same
  unordered vertex pair.  Unmatched faces are reflective walls.
* Affine geometry of each triangle: x = -(r+s)/2 x1 + (1+r)/2 x2 + (1+s)/2 x3,
  metric terms rx, ry, sx, sy, Jacobian J, outward unit normals from the
  edge vectors, face scale Fscale = (edge length / 2) / J, inradius
  r_K = 2 |K| / perimeter as the element length H^k of Eq. 4.1.
* Time step and levels (Section 4): dt_k = CFL r_K / ((N+1)^2 a_max) with
  the global wave speed a = |u| + sqrt(g h) of the initial data; element k
  joins level l when 2^{l-1} dt_min <= dt_k < 2^l dt_min (a relative tie
  tolerance of 1e-12 admits exact factor-of-two sizes), capped at the level
  count, then lowered to the fixed point of l_k <= l_neighbour + 1.
* TVB stencil (Section 5.3, the Cockburn-Shu limiter it cites): for edge i
  with midpoint m_i and element barycentre b0, coefficients alpha_j,
  alpha_k >= 0 with m_i - b0 = alpha_j (b_j - b0) + alpha_k (b_k - b0),
  b_j the neighbours' barycentres (a wall neighbour is b0 mirrored in the
  wall).  Pairs are tried in the order (i,i+1), (i,i+2), (i+1,i+2); when
  none has non-negative coefficients the edge falls back to its own face
  neighbour scaled by |m_i - b0| / |b_i - b0|.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .refelem import RefElement

LEVEL_TIE_TOL = 1e-12
ALPHA_TOL = -1e-10


class MeshError(ValueError):
    pass


def connect(etov: np.ndarray, bc: Optional[np.ndarray] = None):
    """EToE, EToF and wall flags from the element-to-vertex table.  ``bc``
    (K, 3), optional: 1 makes a face a reflective wall even where another
    element shares it (then on both sides); 0 leaves it to the matching."""
    K = etov.shape[0]
    etoe = np.repeat(np.arange(K, dtype=np.int64)[:, None], 3, axis=1)
    etof = np.tile(np.arange(3, dtype=np.int64), (K, 1))
    open_faces = {}
    closed = set()
    for k in range(K):
        for f in range(3):
            a = int(etov[k, f])
            b = int(etov[k, (f + 1) % 3])
            if a == b:
                raise MeshError(f"element {k} has a repeated vertex")
            key = (a, b) if a < b else (b, a)
            if key in closed:
                raise MeshError(f"face {key} is shared by more than two elements")
            other = open_faces.pop(key, None)
            if other is None:
                open_faces[key] = (k, f, a, b)
                continue
            k2, f2, a2, b2 = other
            if (a2, b2) != (b, a):
                raise MeshError(f"elements {k2} and {k} traverse face {key} the same way")
            etoe[k, f], etof[k, f] = k2, f2
            etoe[k2, f2], etof[k2, f2] = k, f
            closed.add(key)
    wall = np.zeros((K, 3), dtype=bool)
    for (k, f, _, _) in open_faces.values():
        wall[k, f] = True
    if bc is not None:
        bc = np.asarray(bc)
        if bc.shape != (K, 3) or not np.all((bc == 0) | (bc == 1)):
            raise MeshError("boundary tags must be (K, 3) with values 0 or 1")
        for k, f in zip(*np.nonzero(bc == 1)):
            if wall[k, f]:
                continue
            k2, f2 = etoe[k, f], etof[k, f]
            etoe[k, f], etof[k, f], wall[k, f] = k, f, True
            etoe[k2, f2], etof[k2, f2], wall[k2, f2] = k2, f2, True
    return etoe, etof, wall


@dataclass
class Mesh:
    K: int
    vx: np.ndarray
    vy: np.ndarray
    etov: np.ndarray
    etoe: np.ndarray
    etof: np.ndarray
    wall: np.ndarray
    rx: np.ndarray
    ry: np.ndarray
    sx: np.ndarray
    sy: np.ndarray
    J: np.ndarray
    nx: np.ndarray        # (K, 3)
    ny: np.ndarray
    sJ: np.ndarray
    fscale: np.ndarray
    x: np.ndarray         # (K, Np)
    y: np.ndarray
    inradius: np.ndarray
    longest_edge: np.ndarray
    vmapP: np.ndarray     # (K, 3*Nfp) flat index of the exterior node (self for walls)


def build_mesh(vx, vy, etov, ref: RefElement, bc=None) -> Mesh:
    vx = np.asarray(vx, dtype=np.float64)
    vy = np.asarray(vy, dtype=np.float64)
    etov = np.asarray(etov, dtype=np.int64)
    K = etov.shape[0]
    if etov.ndim != 2 or etov.shape[1] != 3:
        raise MeshError("etov must be (K, 3)")
    if etov.min() < 0 or etov.max() >= vx.size:
        raise MeshError("vertex index out of range")
    x1, x2, x3 = (vx[etov[:, i]] for i in range(3))
    y1, y2, y3 = (vy[etov[:, i]] for i in range(3))
    xr, xs = (x2 - x1) / 2.0, (x3 - x1) / 2.0
    yr, ys = (y2 - y1) / 2.0, (y3 - y1) / 2.0
    J = xr * ys - xs * yr
    if np.any(J <= 0.0):
        raise MeshError("element not counter-clockwise or degenerate")
    rx, ry, sx, sy = ys / J, -xs / J, -yr / J, xr / J
    px = np.stack([x1, x2, x3], axis=1)
    py = np.stack([y1, y2, y3], axis=1)
    ex = np.roll(px, -1, axis=1) - px          # edge f: vertex f -> vertex f+1
    ey = np.roll(py, -1, axis=1) - py
    elen = np.hypot(ex, ey)
    nx, ny = ey / elen, -ex / elen
    sJ = elen / 2.0
    fscale = sJ / J[:, None]
    area = 2.0 * J
    inradius = 2.0 * area / elen.sum(axis=1)
    r, s = ref.r, ref.s
    x = 0.5 * (-(r + s)[None, :] * x1[:, None] + (1 + r)[None, :] * x2[:, None]
               + (1 + s)[None, :] * x3[:, None])
    y = 0.5 * (-(r + s)[None, :] * y1[:, None] + (1 + r)[None, :] * y2[:, None]
               + (1 + s)[None, :] * y3[:, None])
    etoe, etof, wall = connect(etov, bc)
    Nfp = ref.Nfp
    vmapP = np.empty((K, 3 * Nfp), dtype=np.int64)
    for f in range(3):
        for j in range(Nfp):
            node = ref.fmask[etof[:, f], Nfp - 1 - j]
            vmapP[:, f * Nfp + j] = etoe[:, f] * ref.Np + node
    return Mesh(K, vx, vy, etov, etoe, etof, wall, rx, ry, sx, sy, J, nx, ny, sJ, fscale,
                x, y, inradius, elen.max(axis=1), vmapP)


def assign_levels(mesh: Mesh, max_levels: int) -> np.ndarray:
    """Multi-rate level of every element (1 = finest).

    dt_k is proportional to the inradius (global wave speed), so the level test
    2^j dt_min <= dt_k reduces to 2^j r_min <= r_k."""
    r = mesh.inradius
    rmin = r.min()
    lev = np.ones(mesh.K, dtype=np.int64)
    for k in range(mesh.K):
        j = 0
        while j + 1 < max_levels and (2.0 ** (j + 1)) * rmin <= r[k] * (1.0 + LEVEL_TIE_TOL):
            j += 1
        lev[k] = 1 + j
    while True:
        nb = lev[mesh.etoe]
        new = np.minimum(lev, nb.min(axis=1) + 1)
        if np.array_equal(new, lev):
            return lev
        lev = new


def element_wave_speeds(mesh: Mesh, h, hu, hv, g: float, hvel: float) -> np.ndarray:
    """Per-element wave speed for regrouping: the maximum of |(u,v)| + sqrt(g h)
    (desingularised velocity) over the nodes of the element and of its face
    neighbours (the speed that can enter it), floored at 1e-12."""
    f = 2.0 * h / (h * h + np.maximum(h * h, hvel * hvel))
    node = (np.hypot(hu * f, hv * f) + np.sqrt(g * np.maximum(h, 0.0))).max(axis=1)
    return np.maximum(np.maximum(node, node[mesh.etoe].max(axis=1)), 1e-12)


def speed_levels(mesh: Mesh, N: int, cfl: float, speeds: np.ndarray, max_levels: int):
    """Levels from each element's own allowable step (Eq. 4.1 with a per
    element): dt_k = CFL r_k / ((N+1)^2 a_k), dt_min = min dt_k, level l_k with
    2^(l-1) dt_min <= dt_k < 2^l dt_min (tie tolerance 1e-12), capped at
    max_levels, then the 2:1 rule across faces.  Returns (levels, dt_min)."""
    dt = cfl * mesh.inradius / ((N + 1) ** 2 * speeds)
    dtmin = float(dt.min())
    lev = np.ones(mesh.K, dtype=np.int64)
    for k in range(mesh.K):
        j = 0
        while j + 1 < max_levels and (2.0 ** (j + 1)) * dtmin <= dt[k] * (1.0 + LEVEL_TIE_TOL):
            j += 1
        lev[k] = 1 + j
    while True:
        new = np.minimum(lev, lev[mesh.etoe].min(axis=1) + 1)
        if np.array_equal(new, lev):
            return lev, dtmin
        lev = new


def time_step(mesh: Mesh, N: int, cfl: float, a_max: float) -> float:
    """dt_min of Eq. 4.1: min over elements of CFL r_K / ((N+1)^2 a_max)."""
    return cfl * mesh.inradius.min() / ((N + 1) ** 2 * max(a_max, 1e-12))


def wave_speed(h, hu, hv, g: float, hvel: float) -> float:
    """max |(u,v)| + sqrt(g h) over the nodes, with the desingularised
    velocity 2 h m / (h^2 + max(h^2, hvel^2))."""
    f = 2.0 * h / (h * h + np.maximum(h * h, hvel * hvel))
    return float(np.max(np.hypot(hu * f, hv * f) + np.sqrt(g * np.maximum(h, 0.0))))


@dataclass
class TVBStencil:
    pair: np.ndarray      # (K, 3, 2) face indices j, k used for edge i
    alpha: np.ndarray     # (K, 3, 2)
    direction: np.ndarray  # (K, 3, 2) unit vector (m_i - b0)/|m_i - b0|
    dk: np.ndarray        # (K,) longest edge


def tvb_stencil(mesh: Mesh) -> TVBStencil:
    K = mesh.K
    px = mesh.vx[mesh.etov]
    py = mesh.vy[mesh.etov]
    b0 = np.stack([px.mean(axis=1), py.mean(axis=1)], axis=1)          # (K, 2)
    mid = np.stack([0.5 * (px + np.roll(px, -1, axis=1)),
                    0.5 * (py + np.roll(py, -1, axis=1))], axis=2)      # (K, 3, 2)
    nbc = b0[mesh.etoe]                                                 # (K, 3, 2)
    # wall neighbour: b0 mirrored in the wall line
    n = np.stack([mesh.nx, mesh.ny], axis=2)
    pnt = np.stack([px, py], axis=2)
    dist = np.sum((b0[:, None, :] - pnt) * n, axis=2)
    mirror = b0[:, None, :] - 2.0 * dist[:, :, None] * n
    nbc = np.where(mesh.wall[:, :, None], mirror, nbc)
    pair = np.zeros((K, 3, 2), dtype=np.int64)
    alpha = np.zeros((K, 3, 2))
    direction = np.zeros((K, 3, 2))
    for i in range(3):
        d = mid[:, i, :] - b0
        direction[:, i, :] = d / np.linalg.norm(d, axis=1)[:, None]
        done = np.zeros(K, dtype=bool)
        for (j, k) in [(i, (i + 1) % 3), (i, (i + 2) % 3), ((i + 1) % 3, (i + 2) % 3)]:
            a = nbc[:, j, :] - b0
            b = nbc[:, k, :] - b0
            det = a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]
            scale = np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1)
            ok = np.abs(det) > 1e-12 * scale
            dets = np.where(ok, det, 1.0)
            aj = (d[:, 0] * b[:, 1] - d[:, 1] * b[:, 0]) / dets
            ak = (a[:, 0] * d[:, 1] - a[:, 1] * d[:, 0]) / dets
            good = ok & (aj >= ALPHA_TOL) & (ak >= ALPHA_TOL) & ~done
            pair[good, i] = (j, k)
            alpha[good, i, 0] = aj[good]
            alpha[good, i, 1] = ak[good]
            done |= good
        rest = ~done
        if np.any(rest):
            bi = nbc[rest, i, :] - b0[rest]
            pair[rest, i] = (i, i)
            alpha[rest, i, 0] = np.linalg.norm(d[rest], axis=1) / np.linalg.norm(bi, axis=1)
            alpha[rest, i, 1] = 0.0
    return TVBStencil(pair, alpha, direction, mesh.longest_edge.copy())
