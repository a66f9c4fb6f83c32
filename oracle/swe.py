"""FP64 nodal DG solver for the 2D shallow water equations (oracle).

Test infrastructure only (see the package header).  Every function follows a
passage of the paper; the nodal-collocation reading (volume term Dr/Ds on the
nodal fluxes, surface term LIFT on face-node fluxes) is used throughout.

Right-hand side (Section 2, Eq. 2.1-2.3; Section 3, Eq. 3.2-3.3), in strong
form with the numerical flux of Section 5.1:

    R(Q) = -(d/dx F + d/dy G) + S + LIFT [ Fscale (F(Q-).n - F*.n) ]

* velocities u = 2 h hu / (h^2 + max(h^2, hvel^2)) (likewise v): hu/h where
  h >= hvel, continuous down to zero at h = 0.  The paper does not say how
  the velocity is formed near dry nodes; a continuous form has no branch for
  rounding to flip, and hvel above the positivity limiter's vertex value h0
  keeps the velocity at that vertex bounded;
* S is the bathymetry source -g h grad B written as
  -g eta grad B + (g/2) grad(B^2) with eta = h + B (the splitting of the
  Xing & Shu paper the well-balanced flux is taken from), which keeps the
  lake at rest exactly steady under collocation;
* hydrostatic reconstruction h*^{+-} = max(0, h^{+-} + B^{+-} - max(B+, B-))
  and Q* = (h*, h* u, h* v) (Eq. 5.1);
* F* = F_LF(Q*+, Q*-) + (0, g/2 (h-)^2 - g/2 (h*-)^2, 0), likewise G*
  (Eq. 5.2), F_LF the local Lax-Friedrichs flux with the wave speed
  max |u.n| + sqrt(g h*) taken over both sides of all nodes of the face;
* reflective walls use the mirror state (h, m - 2 (m.n) n) with B+ = B-.

Limiters after every update (Algorithm 5.1): Q <- TVB(PP(Q)).

* PP (Algorithm 5.2): keep the element when min_j h_j > eps; otherwise
  project onto P1; when the mean depth is below h0 the element is dry
  (h = max(mean, 0), hu = hv = 0), else scale the P1 part about the mean by
  theta = min(1, (hbar - h0) / (hbar - min vertex h1)).
* TVB (Section 5.3): Cockburn-Shu characteristic TVB limiter on the P1 part
  with edge-midpoint deviations, then the positivity modification of Eq. 5.3
  on the depth increments; skipped on dry elements and their face
  neighbours; an element none of whose characteristic components was
  limited keeps its full degree-N solution.

Time stepping: Adams-Bashforth 3 (Algorithm 4.1 with one level), started by
forward Euler and AB2; multi-rate AB3 over levels that step with
2^{l-1} dt_min (Section 4, Algorithms 4.1 and 5.1) on a tick schedule, the
coarser neighbours of an active level supplying their AB3 interpolant at
the half step.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .mesh import (Mesh, assign_levels, build_mesh, element_wave_speeds, speed_levels, time_step,
                   tvb_stencil, wave_speed)
from .overint import gauss_exterior_map, overint_operators
from .refelem import reference_element

AB_COEFFS = {1: (1.0,), 2: (1.5, -0.5), 3: (23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0)}
# integral of the Adams-Bashforth interpolant over the first half step, in
# units of the full step: FE, AB2, AB3
HALF_COEFFS = {1: (0.5,), 2: (5.0 / 8.0, -1.0 / 8.0), 3: (17.0 / 24.0, -7.0 / 24.0, 2.0 / 24.0)}

PP_KEEP, PP_SCALED, PP_DRY = 0, 1, 2
TVB_SKIPPED, TVB_KEPT, TVB_LIMITED, TVB_POSITIVE = 0, 1, 2, 3


@dataclass
class Params:
    g: float = 9.81
    cfl: float = 0.5
    h0: float = 1e-5          # dry threshold
    eps: float = 1e-5         # positivity-limiter trigger
    hvel: float = 1e-3        # depth below which velocities are desingularised
    tvb_M: float = 10.0
    tvb_nu: float = 1.5
    pp: bool = True
    tvb: bool = True
    dry_literal: bool = False  # literal dry branch h = h0 instead of max(hbar, 0)
    thin_cut: float = 0.0      # > 0: momentum zeroed after the limiters where h < thin_cut
    max_levels: int = 1
    overint: bool = False      # weak form with cubature and Gauss rules (Section 3, Section 7)
    regroup_every: int = 0     # multi-rate: regroup levels from the current wave speeds every
                               # this many coarse steps (0: levels fixed from the mesh)


@dataclass
class StepFlags:
    pp: np.ndarray
    tvb: np.ndarray
    neg_mean: int = 0


def char_left(ub, vb, c, ex, ey):
    """Rows of the left eigenvectors L of the flux Jacobian A = F'(q) ex +
    G'(q) ey of Eq. 2.2 in direction (ex, ey) (unit), at the state with
    velocity (ub, vb) and celerity c = sqrt(g h): L A R = diag(un - c, un,
    un + c) with un = ub ex + vb ey.  Arrays of n states -> (n, 3, 3)."""
    un = ub * ex + vb * ey
    ut = -ub * ey + vb * ex
    return np.stack([
        np.stack([(un + c) / (2 * c), -ex / (2 * c), -ey / (2 * c)], axis=-1),
        np.stack([-ut, -ey, ex], axis=-1),
        np.stack([-(un - c) / (2 * c), ex / (2 * c), ey / (2 * c)], axis=-1)], axis=1)


def char_right(ub, vb, c, ex, ey):
    """Right eigenvectors R (columns) of the same Jacobian, R = L^-1:
    acoustic waves (1, ub -+ c ex, vb -+ c ey) and the shear wave
    (0, -ey, ex).  Arrays of n states -> (n, 3, 3)."""
    one = np.ones_like(ub * ex)
    return np.stack([
        np.stack([one, np.zeros_like(one), one], axis=-1),
        np.stack([ub - c * ex, -ey * one, ub + c * ex], axis=-1),
        np.stack([vb - c * ey, ex * one, vb + c * ey], axis=-1)], axis=1)


def char_minmod(ub, vb, c, ex, ey, dev, dbar, nu, M2):
    """One edge of the characteristic TVB limiter (Section 5.3, after Cockburn
    and Shu): the P1 deviation dev (3, n) of the conserved variables at the
    edge midpoint and the neighbour-mean increment dbar (3, n) go to
    characteristic variables a1 = L dev, a2 = nu L dbar; each component keeps
    a1 when |a1| <= M2 (the TVB bypass, M d_K^2) and otherwise takes
    minmod(a1, a2); the result goes back through R.  Returns the limited
    deviation (3, n) and whether every component kept a1."""
    L = char_left(ub, vb, c, ex, ey)
    Rm = char_right(ub, vb, c, ex, ey)
    a1 = np.einsum("nab,bn->an", L, dev)
    a2 = nu * np.einsum("nab,bn->an", L, dbar)
    small = np.abs(a1) <= M2[None, :]
    same = np.sign(a1) == np.sign(a2)
    mm = np.where(same, np.sign(a1) * np.minimum(np.abs(a1), np.abs(a2)), 0.0)
    mt = np.where(small, a1, mm)
    ret = small | (a1 == 0.0) | (same & (np.abs(a1) <= np.abs(a2)))
    return np.einsum("nab,bn->an", Rm, mt), ret.all(axis=0)


class Solver:
    """FP64 DG-SWE solver on one triangulation."""

    def __init__(self, vx, vy, etov, N: int, params: Optional[Params] = None,
                 ghost: Optional[Callable] = None, bc=None):
        self.p = params or Params()
        if self.p.regroup_every > 0 and self.p.max_levels < 2:
            raise ValueError("regrouping is a multi-rate option (max_levels >= 2)")
        if 0 < self.p.regroup_every < 3:
            # a level change re-samples three history values per element; by the
            # third coarse step after one they are all the element's own again
            raise ValueError("regroup_every must be 0 or at least 3 coarse steps")
        self.N = N
        self.ref = reference_element(N)
        self.mesh: Mesh = build_mesh(vx, vy, etov, self.ref, bc)
        self.levels = assign_levels(self.mesh, self.p.max_levels)
        self.stencil = tvb_stencil(self.mesh)
        self.ghost = ghost
        if self.p.overint:
            self.oi = overint_operators(self.ref)
            self.gmapP = gauss_exterior_map(self.mesh, self.oi.NG)
        self.t = 0.0
        self.q = None
        self.B = None
        self.dt_min = None
        self.flags = None
        self.history = []
        self.flag_counts = []

    # ------------------------------------------------------------------ data
    @property
    def K(self):
        return self.mesh.K

    def nodes(self):
        return self.mesh.x, self.mesh.y

    def interpolate(self, fn):
        """Nodal interpolation (the projection Pi_H of the initial data, read as
        interpolation at the nodes)."""
        return np.asarray(fn(self.mesh.x, self.mesh.y), dtype=np.float64)

    def set_state(self, h, hu, hv, B, limit: bool = True):
        """Q^0 = TVB(PP(Pi_H Q^0)) (first line of Algorithm 5.1); the time step
        uses the wave speed of the interpolated initial data."""
        self.B = np.array(B, dtype=np.float64)
        q = np.stack([np.asarray(h, np.float64), np.asarray(hu, np.float64),
                      np.asarray(hv, np.float64)]).copy()
        a_max = wave_speed(q[0], q[1], q[2], self.p.g, self.p.hvel)
        self.dt_min = time_step(self.mesh, self.N, self.p.cfl, a_max)
        if self.p.regroup_every > 0:
            # levels from the elements' own wave speeds, regrouped as the run goes
            sp = element_wave_speeds(self.mesh, q[0], q[1], q[2], self.p.g, self.p.hvel)
            self.levels, self.dt_min = speed_levels(self.mesh, self.N, self.p.cfl, sp, self.p.max_levels)
        self.coarse_steps = 0
        if limit:
            q, self.flags = self.limit(q)
        self.q = q
        self.t = 0.0
        self.history = []
        self.flag_counts = []
        self._mr = None

    # ------------------------------------------------------------------ RHS
    def ddr(self, f):
        return f @ self.ref.Dr.T

    def dds(self, f):
        return f @ self.ref.Ds.T

    def ddx(self, f):
        m = self.mesh
        return m.rx[:, None] * self.ddr(f) + m.sx[:, None] * self.dds(f)

    def ddy(self, f):
        m = self.mesh
        return m.ry[:, None] * self.ddr(f) + m.sy[:, None] * self.dds(f)

    def velocity(self, h, hu, hv):
        """Desingularised velocity 2 h m / (h^2 + max(h^2, hvel^2)): equal to
        m/h for h >= hvel, continuous in h, zero at h = 0."""
        den = h * h + np.maximum(h * h, self.p.hvel ** 2)
        f = 2.0 * h / den
        return hu * f, hv * f

    def traces(self, q, B, t, qP_override=None):
        """Interior (-) and exterior (+) traces at the 3*Nfp face nodes."""
        ref, m = self.ref, self.mesh
        fm = ref.fmask.reshape(-1)
        qM = q[:, :, fm]
        BM = B[:, fm]
        src = q if qP_override is None else qP_override
        qP = src.reshape(3, -1)[:, m.vmapP]
        BP = B.reshape(-1)[m.vmapP]
        Nfp = ref.Nfp
        nx = np.repeat(m.nx, Nfp, axis=1)
        ny = np.repeat(m.ny, Nfp, axis=1)
        wall = np.repeat(m.wall, Nfp, axis=1)
        if self.ghost is None:
            mn = qM[1] * nx + qM[2] * ny
            ghost = np.stack([qM[0], qM[1] - 2.0 * mn * nx, qM[2] - 2.0 * mn * ny])
        else:
            xf = m.x[:, fm]
            yf = m.y[:, fm]
            gh, ghu, ghv = self.ghost(xf, yf, t)
            ghost = np.stack([gh, ghu, ghv])
        qP = np.where(wall[None], ghost, qP)
        BP = np.where(wall, BM, BP)
        return qM, qP, BM, BP, nx, ny

    def rhs(self, q, B, t=0.0, qP_override=None):
        if self.p.overint:
            return self.rhs_overint(q, B, t, qP_override)
        return self.rhs_nodal(q, B, t, qP_override)

    def rhs_overint(self, q, B, t=0.0, qP_override=None):
        """Weak form with over-integration (Section 3, Eq. 3.2; Section 7,
        Volume and Surface kernels): N = Pr cF1 + Ps cF2 + P cS at the
        cubature nodes with the plain source cS = (0, -g h B_x, -g h B_y),
        S = -L^g (Fscale Fn*) at the Gauss nodes of the faces with the
        well-balanced flux of Eq. 5.1-5.2 (the wave speed maxed over the
        face's Gauss points of both sides)."""
        oi, m, p = self.oi, self.mesh, self.p
        g = p.g
        NG = oi.NG
        # volume: interpolate to the cubature nodes
        h, hu, hv = q @ oi.Ic.T
        Bx = m.rx[:, None] * (B @ oi.Drc.T) + m.sx[:, None] * (B @ oi.Dsc.T)
        By = m.ry[:, None] * (B @ oi.Drc.T) + m.sy[:, None] * (B @ oi.Dsc.T)
        u, v = self.velocity(h, hu, hv)
        F = np.stack([hu, hu * u + 0.5 * g * h * h, hu * v])
        G = np.stack([hv, hv * u, hv * v + 0.5 * g * h * h])
        cF1 = m.rx[:, None] * F + m.ry[:, None] * G
        cF2 = m.sx[:, None] * F + m.sy[:, None] * G
        cS = np.stack([np.zeros_like(h), -g * h * Bx, -g * h * By])
        R = cF1 @ oi.Pr.T + cF2 @ oi.Ps.T + cS @ oi.P.T
        # faces: traces at the Gauss nodes
        qM = q @ oi.Ig.T                          # (3, K, 3 NG)
        BM = B @ oi.Ig.T
        src = qM if qP_override is None else qP_override @ oi.Ig.T
        qP = src.reshape(3, -1)[:, self.gmapP]
        BP = BM.reshape(-1)[self.gmapP]
        nx = np.repeat(m.nx, NG, axis=1)
        ny = np.repeat(m.ny, NG, axis=1)
        wall = np.repeat(m.wall, NG, axis=1)
        if self.ghost is None:
            mn = qM[1] * nx + qM[2] * ny
            ghost = np.stack([qM[0], qM[1] - 2.0 * mn * nx, qM[2] - 2.0 * mn * ny])
        else:
            gh, ghu, ghv = self.ghost(m.x @ oi.Ig.T, m.y @ oi.Ig.T, t)
            ghost = np.stack([gh, ghu, ghv])
        qP = np.where(wall[None], ghost, qP)
        BP = np.where(wall, BM, BP)
        fstar = self._wb_flux(qM, qP, BM, BP, nx, ny, NG)
        fs = np.repeat(m.fscale, NG, axis=1)
        R -= (fs * fstar) @ oi.Lg.T
        return R

    def _wb_flux(self, qM, qP, BM, BP, nx, ny, npf):
        """Well-balanced Lax-Friedrichs flux F*.n of Eq. 5.1-5.2 at face
        points, npf points per face (wave speed maxed over each face)."""
        g = self.p.g
        hM, huM, hvM = qM
        hP, huP, hvP = qP
        uM, vM = self.velocity(hM, huM, hvM)
        uP, vP = self.velocity(hP, huP, hvP)
        Bmax = np.maximum(BM, BP)
        hsM = np.maximum(0.0, hM + BM - Bmax)
        hsP = np.maximum(0.0, hP + BP - Bmax)
        unM = uM * nx + vM * ny
        unP = uP * nx + vP * ny
        lam = np.maximum(np.abs(unM) + np.sqrt(g * hsM), np.abs(unP) + np.sqrt(g * hsP))
        lam = np.repeat(lam.reshape(self.K, 3, npf).max(axis=2), npf, axis=1)
        qsM = np.stack([hsM, hsM * uM, hsM * vM])
        qsP = np.stack([hsP, hsP * uP, hsP * vP])

        def flux_n(hs, u, v, un):
            return np.stack([hs * un,
                             hs * u * un + 0.5 * g * hs * hs * nx,
                             hs * v * un + 0.5 * g * hs * hs * ny])

        f_lf = 0.5 * (flux_n(hsM, uM, vM, unM) + flux_n(hsP, uP, vP, unP)) - 0.5 * lam * (qsP - qsM)
        corr = 0.5 * g * (hM * hM - hsM * hsM)
        return f_lf + np.stack([np.zeros_like(corr), corr * nx, corr * ny])

    def rhs_nodal(self, q, B, t=0.0, qP_override=None):
        ref, m, p = self.ref, self.mesh, self.p
        g = p.g
        h, hu, hv = q
        u, v = self.velocity(h, hu, hv)
        F = np.stack([hu, hu * u + 0.5 * g * h * h, hu * v])
        G = np.stack([hv, hv * u, hv * v + 0.5 * g * h * h])
        R = -(self.ddx(F) + self.ddy(G))
        eta = h + B
        R[1] += -g * eta * self.ddx(B) + 0.5 * g * self.ddx(B * B)
        R[2] += -g * eta * self.ddy(B) + 0.5 * g * self.ddy(B * B)

        qM, qP, BM, BP, nx, ny = self.traces(q, B, t, qP_override)
        hM, huM, hvM = qM
        hP, huP, hvP = qP
        uM, vM = self.velocity(hM, huM, hvM)
        uP, vP = self.velocity(hP, huP, hvP)
        Bmax = np.maximum(BM, BP)
        hsM = np.maximum(0.0, hM + BM - Bmax)
        hsP = np.maximum(0.0, hP + BP - Bmax)
        unM = uM * nx + vM * ny
        unP = uP * nx + vP * ny
        lam = np.maximum(np.abs(unM) + np.sqrt(g * hsM), np.abs(unP) + np.sqrt(g * hsP))
        Nfp = ref.Nfp
        lam = np.repeat(lam.reshape(self.K, 3, Nfp).max(axis=2), Nfp, axis=1)
        qsM = np.stack([hsM, hsM * uM, hsM * vM])
        qsP = np.stack([hsP, hsP * uP, hsP * vP])

        def flux_n(hs, u, v, un):
            return np.stack([hs * un,
                             hs * u * un + 0.5 * g * hs * hs * nx,
                             hs * v * un + 0.5 * g * hs * hs * ny])

        f_lf = 0.5 * (flux_n(hsM, uM, vM, unM) + flux_n(hsP, uP, vP, unP)) \
            - 0.5 * lam * (qsP - qsM)
        corr = 0.5 * g * (hM * hM - hsM * hsM)
        fstar = f_lf + np.stack([np.zeros_like(corr), corr * nx, corr * ny])
        fM = np.stack([huM * nx + hvM * ny,
                       (huM * uM + 0.5 * g * hM * hM) * nx + huM * vM * ny,
                       hvM * uM * nx + (hvM * vM + 0.5 * g * hM * hM) * ny])
        fs = np.repeat(m.fscale, Nfp, axis=1)
        R += (fs * (fM - fstar)) @ ref.LIFT.T
        return R

    # -------------------------------------------------------------- limiters
    def means(self, q):
        return (q @ self.ref.w) / 2.0

    def pp_limit(self, q, active=None):
        """Positivity-preserving limiter M Pi_H of Algorithm 5.2."""
        ref, p = self.ref, self.p
        q = q.copy()
        K = q.shape[1]
        code = np.zeros(K, dtype=np.uint8)
        hmin = q[0].min(axis=1)
        # Algorithm 5.2 keeps an element whose nodal depths all exceed eps.
        # At orders 4 and 6 three vertex weights of the nodal mean are
        # negative, so such an element can still have a mean below h0, even
        # a negative one, which the TVB stage cannot take (its wave speed is
        # sqrt(g hbar)); these elements take the rest of Algorithm 5.2 too
        # (the dry branch, since hbar < h0).  With positive weights and
        # eps <= h0 this adds nothing.
        trig = (hmin <= p.eps) | (self.means(q)[0] < p.h0)
        if active is not None:
            trig &= active
        neg = 0
        if np.any(trig):
            qt = q[:, trig, :]
            mt = self.means(qt)
            q1 = qt @ ref.proj1.T
            h1min = (qt[0] @ ref.p1_vert.T).min(axis=1)
            den = mt[0] - h1min
            theta = np.where(den > 0.0,
                             np.minimum(1.0, (mt[0] - p.h0) / np.where(den > 0.0, den, 1.0)),
                             1.0)
            new = mt[:, :, None] + theta[None, :, None] * (q1 - mt[:, :, None])
            dry = mt[0] < p.h0
            neg = int(np.sum(mt[0] < 0.0))
            hdry = np.full(mt[0].shape, p.h0) if p.dry_literal else np.maximum(mt[0], 0.0)
            new[0] = np.where(dry[:, None], hdry[:, None], new[0])
            new[1] = np.where(dry[:, None], 0.0, new[1])
            new[2] = np.where(dry[:, None], 0.0, new[2])
            q[:, trig, :] = new
            code[trig] = np.where(dry, PP_DRY, PP_SCALED)
        return q, code, neg

    def tvb_limit(self, q, pp_code, active=None, means=None):
        """Characteristic TVB limiter with the positivity modification (Eq. 5.3).

        ``means`` (3, K) are the neighbour means to use (the post-PP snapshot);
        ``active`` restricts which elements are limited (multi-rate)."""
        ref, m, st, p = self.ref, self.mesh, self.stencil, self.p
        K = m.K
        g = p.g
        q = q.copy()
        if means is None:
            means = self.means(q)
        own = self.means(q)
        dry = pp_code == PP_DRY
        nb_dry = np.where(m.wall, False, dry[m.etoe]).any(axis=1)
        work = ~dry & ~nb_dry
        if active is not None:
            work &= active
        code = np.zeros(K, dtype=np.uint8)
        idx = np.nonzero(work)[0]
        if idx.size == 0:
            return q, code
        qa = q[:, idx, :]
        qbar = own[:, idx]
        dev = np.einsum("ij,ckj->cki", ref.p1_mid, qa) - qbar[:, :, None]      # (3, n, 3 edges)
        nbm = means[:, m.etoe[idx]]                                            # (3, n, 3 faces)
        nxf, nyf = m.nx[idx], m.ny[idx]
        mn = qbar[1][:, None] * nxf + qbar[2][:, None] * nyf
        ghost = np.stack([np.broadcast_to(qbar[0][:, None], mn.shape),
                          qbar[1][:, None] - 2.0 * mn * nxf,
                          qbar[2][:, None] - 2.0 * mn * nyf])
        wall = m.wall[idx]
        nbm = np.where(wall[None], ghost, nbm)
        diff = nbm - qbar[:, :, None]                                          # (3, n, 3)
        hb = qbar[0]
        ub = qbar[1] / hb
        vb = qbar[2] / hb
        c = np.sqrt(g * hb)
        M2 = p.tvb_M * st.dk[idx] ** 2
        n = idx.size
        ar = np.arange(n)
        delta = np.zeros((3, n, 3))
        all_a1 = np.ones(n, dtype=bool)
        for i in range(3):
            pj = st.pair[idx, i, 0]
            pk = st.pair[idx, i, 1]
            dbar = st.alpha[idx, i, 0] * diff[:, ar, pj] + st.alpha[idx, i, 1] * diff[:, ar, pk]
            ex, ey = st.direction[idx, i, 0], st.direction[idx, i, 1]
            delta[:, :, i], ret = char_minmod(ub, vb, c, ex, ey, dev[:, :, i], dbar, p.tvb_nu, M2)
            all_a1 &= ret
        code_a = np.full(n, TVB_KEPT, dtype=np.uint8)
        lim = ~all_a1
        if np.any(lim):
            D = delta[:, lim, :]
            pos = np.maximum(D, 0.0).sum(axis=2)
            neg = np.maximum(-D, 0.0).sum(axis=2)
            thp = np.where(pos > 0.0, np.minimum(1.0, neg / np.where(pos > 0.0, pos, 1.0)), 1.0)
            thm = np.where(neg > 0.0, np.minimum(1.0, pos / np.where(neg > 0.0, neg, 1.0)), 1.0)
            Dh = thp[:, :, None] * np.maximum(D, 0.0) - thm[:, :, None] * np.maximum(-D, 0.0)
            # Eq. 5.3 on the depth increments
            hbl = hb[lim]
            d = Dh[0]
            S = d.sum(axis=1)
            dbar_h = S / 3.0
            vert = S[:, None] - 2.0 * d                    # -D_i + D_j + D_k
            vmin = vert.min(axis=1)
            fix = hbl + vmin < p.h0
            den = dbar_h - vmin
            theta = np.where(den > 0.0, (hbl + dbar_h - p.h0) / np.where(den > 0.0, den, 1.0), 0.0)
            theta = np.clip(theta, 0.0, 1.0)
            dfix = dbar_h[:, None] + theta[:, None] * (d - dbar_h[:, None])
            Dh[0] = np.where(fix[:, None], dfix, d)
            newq = qbar[:, lim, None] + np.einsum("cni,ij->cnj", Dh, ref.phi_mid)
            qa[:, lim, :] = newq
            code_a[lim] = np.where(fix, TVB_POSITIVE, TVB_LIMITED)
        q[:, idx, :] = qa
        code[idx] = code_a
        return q, code

    def limit(self, q, active=None):
        """Lambda Pi_H M Pi_H of Algorithm 5.1 (PP first, then TVB)."""
        p = self.p
        K = q.shape[1]
        pp = np.zeros(K, dtype=np.uint8)
        neg = 0
        if p.pp:
            q, pp, neg = self.pp_limit(q, active)
        tv = np.zeros(K, dtype=np.uint8)
        if p.tvb:
            q, tv = self.tvb_limit(q, pp, active)
        q = self.cut_thin_films(q, active)
        return q, StepFlags(pp, tv, neg)

    def cut_thin_films(self, q, active=None):
        """Optional thin-film rule (the paper is silent on velocities where
        the depth is tiny): after both limiters, zero the momentum at nodes
        whose depth is below thin_cut (elements that stepped only)."""
        if self.p.thin_cut <= 0.0:
            return q
        thin = q[0] < self.p.thin_cut
        if active is not None:
            thin &= active[:, None]
        q = q.copy()
        q[1] = np.where(thin, 0.0, q[1])
        q[2] = np.where(thin, 0.0, q[2])
        return q

    # ------------------------------------------------------------ stepping
    def step(self):
        """One single-rate AB3 step followed by the limiters."""
        R = self.rhs(self.q, self.B, self.t)
        self.history.insert(0, R)
        del self.history[3:]
        coeffs = AB_COEFFS[len(self.history)]
        incr = sum(c * r for c, r in zip(coeffs, self.history))
        qt = self.q + self.dt_min * incr
        self.q, self.flags = self.limit(qt)
        self.t += self.dt_min
        self.flag_counts.append((np.bincount(self.flags.pp, minlength=3),
                                 np.bincount(self.flags.tvb, minlength=4),
                                 self.flags.neg_mean))

    def run(self, steps: int):
        if self.p.max_levels > 1:
            for _ in range(steps):
                self.mrab_coarse_step()
        else:
            for _ in range(steps):
                self.step()
        return self.q

    # ----------------------------------------------------------- multi-rate
    def mrab_coarse_step(self):
        """One coarse step of multi-rate AB3 (Algorithms 4.1 and 5.1).

        Levels l = 1..L step with dt_l = 2^{l-1} dt_min.  A coarse step has
        2^{L-1} ticks of dt_min; at tick k the levels with k mod 2^{l-1} == 0
        are active.  All active levels first evaluate R at the common time
        (finer neighbours are always active and in step; an inactive coarser
        neighbour supplies its AB3 interpolant at its half step, written when
        it last stepped), then they update, coarsest first, then the limiters
        run on the active elements with the post-PP means of all elements.
        """
        L = self.p.max_levels
        lev = self.levels
        K = self.K
        if self._mr is None:
            self._mr = {"hist": [[] for _ in range(L + 1)],
                        "half": self.q.copy(), "tick": 0}
        st = self._mr
        for k in range(2 ** (L - 1)):
            active_levels = [l for l in range(1, L + 1) if k % (2 ** (l - 1)) == 0]
            active = np.isin(lev, active_levels)
            # exterior state: current state, except inactive elements supply
            # their half-step interpolant
            ext = np.where(active[None, :, None], self.q, st["half"])
            R = self.rhs(self.q, self.B, self.t, qP_override=ext)
            qt = self.q.copy()
            half = st["half"]
            for l in sorted(active_levels, reverse=True):
                sel = lev == l
                hist = st["hist"][l]
                hist.insert(0, R[:, sel, :])
                del hist[3:]
                dtl = self.dt_min * 2 ** (l - 1)
                coeffs = AB_COEFFS[len(hist)]
                qt[:, sel, :] = self.q[:, sel, :] + dtl * sum(c * r for c, r in zip(coeffs, hist))
                if l > 1:
                    hc = HALF_COEFFS[len(hist)]
                    half[:, sel, :] = self.q[:, sel, :] + dtl * sum(
                        c * r for c, r in zip(hc, hist))
            qt, flags = self.limit_multirate(qt, active)
            self.q = qt
            self.flags = flags
            self.t += self.dt_min
        self.coarse_steps += 1
        if self.p.regroup_every > 0 and self.coarse_steps % self.p.regroup_every == 0:
            self.regroup()
        return self.q

    def regroup(self):
        """Regroup the elements into levels from the current wave speeds (the
        option named after Algorithm 4.1), at a coarse-step boundary: every
        element's allowable step from Eq. 4.1 with its own wave speed (its
        nodes and its face neighbours'), then the level rule and the 2:1
        rule.  Needs a full history on every level (after the start-up
        steps); otherwise nothing changes."""
        st = self._mr
        L = self.p.max_levels
        if st is None or any(len(st["hist"][l]) < 3 for l in range(1, L + 1) if np.any(self.levels == l)):
            return
        q = self.q
        sp = element_wave_speeds(self.mesh, q[0], q[1], q[2], self.p.g, self.p.hvel)
        new_lev, new_dtmin = speed_levels(self.mesh, self.N, self.p.cfl, sp, L)
        self.set_levels(new_lev, new_dtmin)

    def set_levels(self, new_lev, new_dtmin):
        """Move the elements to new levels (and a new finest step) at a
        coarse-step boundary, where all levels are at the same time t.  Each
        element's Adams-Bashforth history R(t - dt), R(t - 2 dt), R(t - 3 dt) at
        its old step dt is replaced by the values at t - dt', t - 2 dt',
        t - 3 dt' of the quadratic through it, dt' the element's new step: the
        interpolant of the same degree as the AB3 rule, so a level change keeps
        the method third order in smooth flow (not conservative to roundoff:
        neighbours re-sample their histories at different times)."""
        st = self._mr
        L = self.p.max_levels
        old_lev = self.levels
        old_dt = self.dt_min * 2.0 ** (old_lev - 1)
        K, Np = self.K, self.ref.Np
        S = np.zeros((3, 3, K, Np))   # sample s (t - (s+1) dt), field, element, node
        for l in range(1, L + 1):
            sel = old_lev == l
            if not np.any(sel):
                continue
            for sidx in range(3):
                S[sidx][:, sel, :] = st["hist"][l][sidx]
        rho = (new_dtmin * 2.0 ** (np.asarray(new_lev) - 1)) / old_dt          # (K,)
        new = np.zeros_like(S)
        for sidx in range(3):
            tau = -(sidx + 1) * rho[None, :, None]
            l1 = (tau + 2.0) * (tau + 3.0) / 2.0
            l2 = -(tau + 1.0) * (tau + 3.0)
            l3 = (tau + 1.0) * (tau + 2.0) / 2.0
            new[sidx] = l1 * S[0] + l2 * S[1] + l3 * S[2]
        st["hist"] = [[] for _ in range(L + 1)]
        for l in range(1, L + 1):
            sel = new_lev == l
            if np.any(sel):
                st["hist"][l] = [new[sidx][:, sel, :] for sidx in range(3)]
        self.levels = np.asarray(new_lev)
        self.dt_min = new_dtmin

    def limit_multirate(self, q, active):
        p = self.p
        K = q.shape[1]
        pp = np.zeros(K, dtype=np.uint8)
        neg = 0
        prev_pp = self.flags.pp if self.flags is not None else np.zeros(K, np.uint8)
        if p.pp:
            q, pp_new, neg = self.pp_limit(q, active)
            pp = np.where(active, pp_new, prev_pp)
        tv = np.zeros(K, dtype=np.uint8)
        prev_tv = self.flags.tvb if self.flags is not None else tv
        if p.tvb:
            q, tv_new = self.tvb_limit(q, pp, active)
            tv = np.where(active, tv_new, prev_tv)
        q = self.cut_thin_films(q, active)
        return q, StepFlags(pp, tv, neg)

    # --------------------------------------------------------- diagnostics
    def mass(self, q=None):
        q = self.q if q is None else q
        return float(np.sum(self.mesh.J * (q[0] @ self.ref.w)))

    def rel_l2(self, q_test, q_ref=None, fields=(0,)):
        """sqrt(sum_k J_k e.M e) / sqrt(sum_k J_k q.M q) over the given fields."""
        q_ref = self.q if q_ref is None else q_ref
        M = self.ref.M
        num = 0.0
        den = 0.0
        for c in fields:
            e = q_test[c] - q_ref[c]
            num += float(np.sum(self.mesh.J * np.einsum("ki,ij,kj->k", e, M, e)))
            den += float(np.sum(self.mesh.J * np.einsum("ki,ij,kj->k", q_ref[c], M, q_ref[c])))
        return np.sqrt(num) / np.sqrt(den) if den > 0 else np.sqrt(num)
