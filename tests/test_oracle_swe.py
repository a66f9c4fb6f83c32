"""Pins for the oracle's DG-SWE solver against what the paper and the
mathematics fix: exact steady states, conservation, consistency with the PDE,
convergence order, exact Adams-Bashforth coefficients, limiter invariants."""
import numpy as np
import pytest

import workloads as W
from oracle.swe import AB_COEFFS, HALF_COEFFS, PP_DRY, PP_KEEP, PP_SCALED, Params, Solver


def make(wl, params=None, inst=0, **kw):
    ins = wl.instances[inst]
    p = params or Params(g=wl.g, cfl=wl.cfl, **kw)
    s = Solver(ins.vx, ins.vy, ins.etov, wl.N, p)
    x, y = s.nodes()
    B = s.interpolate(ins.bathymetry)
    h, hu, hv = ins.initial(x, y)
    s.set_state(h, hu, hv, B)
    return s


# --------------------------------------------------------------------- RHS
@pytest.mark.parametrize("N", [2, 3, 4])
def test_lake_at_rest_is_steady(N):
    """Exact C-property (Section 5.1): still water over a non-constant bed."""
    s = make(W.lake_at_rest(n=5, N=N))
    R = s.rhs(s.q, s.B)
    assert np.max(np.abs(R)) < 1e-12
    s.run(10)
    assert np.max(np.abs(s.q[0] + s.B - 1.0)) < 1e-13
    assert np.max(np.abs(s.q[1:])) < 1e-12


def test_lake_at_rest_discontinuous_bed():
    """With a bed that jumps across faces only the hydrostatic reconstruction
    and the pressure correction of Eq. 5.1-5.2 keep still water steady."""
    wl = W.lake_at_rest(n=6, N=3)
    ins = wl.instances[0]
    s = Solver(ins.vx, ins.vy, ins.etov, 3, Params())
    x, _ = s.nodes()
    rng = np.random.default_rng(5)
    B = np.repeat(rng.uniform(0.0, 0.4, s.K)[:, None], x.shape[1], axis=1) + 0.2 * x
    q = np.stack([1.0 - B, 0 * B, 0 * B])
    assert np.max(np.abs(s.rhs(q, B))) < 1e-12
    # a bed emerging above the still water (dry element next to wet ones)
    B[3] = 1.5
    q = np.stack([np.maximum(1.0 - B, 0.0), 0 * B, 0 * B])
    assert np.max(np.abs(s.rhs(q, B))) < 1e-12


@pytest.mark.parametrize("N", [1, 3, 5])
def test_stepped_bed_workloads(N):
    """The stepped-bed inputs of the GPU tests (a bed piece per element, a
    jump at every face): still water is a steady state of the oracle; over the
    ledge, whose dry elements' bed rises above the wet neighbours' surface, a
    wave conserves mass and keeps depths non-negative, and the ledge's faces
    are where Eq. 5.1 clips the reconstructed depth to zero."""
    s = make(W.stepped_bed("lake", N=N))
    assert np.max(np.abs(s.rhs(s.q, s.B))) < 1e-11
    s = make(W.stepped_bed("ledge", N=N))
    x, _ = s.nodes()
    eta = s.q[0] + s.B
    wet = s.q[0].min(axis=1) > 0.0
    nb = s.mesh.etoe
    above = [k for k in range(s.K) if wet[k] and any(not wet[nb[k, f]] and s.B[nb[k, f]].min() > eta[k].max()
                                                      for f in range(3))]
    assert len(above) >= 4
    m0 = s.mass()
    s.run(100)
    assert abs(s.mass() - m0) <= 1e-13 * m0
    assert s.q[0].min() >= 0.0


def test_uniform_flow_interior_residual_zero():
    wl = W.lake_at_rest(n=6, N=3)
    ins = wl.instances[0]
    s = Solver(ins.vx, ins.vy, ins.etov, 3, Params(pp=False, tvb=False))
    x, y = s.nodes()
    q = np.stack([np.full_like(x, 1.3), np.full_like(x, 0.4), np.full_like(x, -0.2)])
    R = s.rhs(q, np.zeros_like(x))
    inner = ~s.mesh.wall.any(axis=1)
    assert np.max(np.abs(R[:, inner, :])) < 1e-12


def test_rhs_conserves_mass_with_walls():
    wl = W.small_wetdry(n=6, N=3)
    s = make(wl)
    rng = np.random.default_rng(0)
    q = np.stack([0.5 + rng.uniform(0, 0.5, s.q[0].shape), rng.normal(0, 0.3, s.q[0].shape),
                  rng.normal(0, 0.3, s.q[0].shape)])
    R = s.rhs(q, s.B)
    total = np.sum(s.mesh.J * (R[0] @ s.ref.w))
    scale = np.sum(s.mesh.J * (np.abs(R[0]) @ s.ref.w))
    assert abs(total) < 1e-13 * scale


def _manufactured(g):
    def state(x, y):
        h = 1.0 + 0.2 * np.sin(2 * x + 1) * np.cos(3 * y)
        hu = 0.3 * np.cos(x - 2 * y)
        hv = -0.2 * np.sin(x * y + 0.5)
        return h, hu, hv

    def bed(x, y):
        return 0.1 * np.cos(x + y) + 0.05 * x

    def pde_rhs(x, y, d=1e-5):
        def F(x, y):
            h, hu, hv = state(x, y)
            u, v = hu / h, hv / h
            return np.stack([hu, hu * u + 0.5 * g * h * h, hu * v])

        def G(x, y):
            h, hu, hv = state(x, y)
            u, v = hu / h, hv / h
            return np.stack([hv, hv * u, hv * v + 0.5 * g * h * h])

        dFx = (F(x + d, y) - F(x - d, y)) / (2 * d)
        dGy = (G(x, y + d) - G(x, y - d)) / (2 * d)
        h = state(x, y)[0]
        Bx = (bed(x + d, y) - bed(x - d, y)) / (2 * d)
        By = (bed(x, y + d) - bed(x, y - d)) / (2 * d)
        S = np.stack([0 * h, -g * h * Bx, -g * h * By])
        return -(dFx + dGy) + S

    return state, bed, pde_rhs


@pytest.mark.parametrize("N", [2, 3])
def test_rhs_consistent_with_pde(N):
    """R(Q_H) approaches -div F + S of the PDE (Eq. 2.2) at order ~N on smooth
    data; a dropped term or wrong sign anywhere in volume, source or surface
    terms breaks this."""
    g = 9.81
    state, bed, pde_rhs = _manufactured(g)
    errs = []
    for n in (8, 16, 32):
        vx, vy, etov = W.structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0)
        s = Solver(vx, vy, etov, N, Params(g=g, pp=False, tvb=False))
        x, y = s.nodes()
        q = np.stack(state(x, y))
        B = bed(x, y)
        R = s.rhs(q, B)
        exact = pde_rhs(x, y)
        inner = ~s.mesh.wall.any(axis=1)
        errs.append(np.max(np.abs(R - exact)[:, inner, :]))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > N - 0.5), (errs, rates)


def _vortex_exact(beta=5.0):
    def exact(x, y, t):
        xx = x - t
        r2 = xx ** 2 + y ** 2
        h = 1 - beta ** 2 / (32 * np.pi ** 2) * np.exp(2 * (1 - r2))
        u = 1 - beta * np.exp(1 - r2) * y / (2 * np.pi)
        v = beta * np.exp(1 - r2) * xx / (2 * np.pi)
        return h, h * u, h * v
    return exact


@pytest.mark.parametrize("N", [2, 3])
def test_vortex_convergence_order(N):
    """Translating vortex of Section 6.2 (g = 2, Dirichlet data = exact
    solution, limiters off): least-squares EOC of the depth error at least
    N + 1/2 - 0.2 (Table 6.1)."""
    exact = _vortex_exact()
    T = 0.25
    errs, Hs = [], []
    for n in (10, 20, 40):
        vx, vy, etov = W.structured_mesh(int(1.5 * n), int(1.2 * n), -5, 10, -6, 6)
        s = Solver(vx, vy, etov, N, Params(g=2.0, cfl=0.5, pp=False, tvb=False), ghost=exact)
        x, y = s.nodes()
        s.set_state(*exact(x, y, 0.0), 0 * x)
        nst = int(np.ceil(T / s.dt_min))
        s.dt_min = T / nst
        s.run(nst)
        errs.append(s.rel_l2(np.stack(exact(x, y, T)), fields=(0,)))
        Hs.append(10.0 / n)
    eoc = np.polyfit(np.log(Hs), np.log(errs), 1)[0]
    assert eoc >= N + 0.5 - 0.2, (errs, eoc)


# --------------------------------------------------------------- time
def test_adams_bashforth_coefficients_exact_for_quadratics():
    """AB3 integrates the quadratic interpolant of the last three RHS values
    (Algorithm 4.1): exact for y' = c0 + c1 t + c2 t^2; the half-step weights
    integrate the same interpolant over the first half step."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        c = rng.normal(size=3)
        dt = rng.uniform(0.1, 2.0)
        t0 = rng.uniform(-1, 1)
        f = lambda t: c[0] + c[1] * t + c[2] * t * t  # noqa: E731
        prim = lambda t: c[0] * t + c[1] * t ** 2 / 2 + c[2] * t ** 3 / 3  # noqa: E731
        fs = [f(t0 - s * dt) for s in range(3)]
        assert abs(dt * sum(a * b for a, b in zip(AB_COEFFS[3], fs))
                   - (prim(t0 + dt) - prim(t0))) < 1e-12
        assert abs(dt * sum(a * b for a, b in zip(HALF_COEFFS[3], fs))
                   - (prim(t0 + dt / 2) - prim(t0))) < 1e-12
        g = lambda t: c[0] + c[1] * t  # noqa: E731
        gp = lambda t: c[0] * t + c[1] * t ** 2 / 2  # noqa: E731
        gs = [g(t0 - s * dt) for s in range(2)]
        assert abs(dt * sum(a * b for a, b in zip(AB_COEFFS[2], gs)) - (gp(t0 + dt) - gp(t0))) < 1e-12
        assert abs(dt * sum(a * b for a, b in zip(HALF_COEFFS[2], gs))
                   - (gp(t0 + dt / 2) - gp(t0))) < 1e-12


def test_solver_step_exact_for_quadratic_forcing():
    s = make(W.lake_at_rest(n=2, N=1), Params(pp=False, tvb=False))
    c = np.array([0.3, -1.2, 0.7])
    f = lambda t: c[0] + c[1] * t + c[2] * t * t  # noqa: E731
    prim = lambda t: c[0] * t + c[1] * t ** 2 / 2 + c[2] * t ** 3 / 3  # noqa: E731
    s.rhs = lambda q, B, t=0.0, qP_override=None: np.full_like(q, f(t))
    dt = s.dt_min = 0.05
    s.t = 2 * dt
    s.history = [np.full_like(s.q, f(dt)), np.full_like(s.q, f(0.0))]
    q0 = s.q.copy()
    for _ in range(4):
        s.step()
    assert np.max(np.abs(s.q - (q0 + prim(s.t) - prim(2 * dt)))) < 1e-12


def test_mrab_one_level_is_ab3_bitwise():
    wl = W.small_wetdry(n=6, N=2)
    a = make(wl, Params(g=wl.g, cfl=0.2))
    b = make(wl, Params(g=wl.g, cfl=0.2))
    for _ in range(15):
        a.step()
        b.mrab_coarse_step()
    assert np.array_equal(a.q, b.q)


def test_mrab_two_levels_third_order():
    """Two-level multi-rate AB3 (Section 4, Algorithm 4.1, on the tick
    schedule) converges at third order in dt_min.  The run starts from an
    exact history (the right-hand sides of a fine RK4 reference at the
    earlier step times of each level), so the forward Euler / AB2 start-up
    does not set the order; a wrong half-step weight of the coarse level's
    interpolant drops the ratio to about 2."""
    wl = W.c3(n0=2, n_bands=2)
    ins = wl.instances[0]

    def make_mr(levels):
        s = Solver(ins.vx, ins.vy, ins.etov, 2, Params(g=wl.g, cfl=0.3, max_levels=levels,
                                                      pp=False, tvb=False))
        x, y = s.nodes()
        s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry), limit=False)
        return s

    s0 = make_mr(2)
    assert np.unique(s0.levels).size == 2
    dt0, B = s0.dt_min, s0.B
    hq, T0, T, sub = dt0 / 4, 4 * dt0, 16 * dt0, 16

    def rk4(q, h):
        k1 = s0.rhs(q, B)
        k2 = s0.rhs(q + 0.5 * h * k1, B)
        k3 = s0.rhs(q + 0.5 * h * k2, B)
        k4 = s0.rhs(q + h * k3, B)
        return q + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    # reference states every dt0/4 from t = -T0 to T
    q = s0.q.copy()
    ref = []
    n_total = int(round((T0 + T) / hq))
    for i in range(n_total + 1):
        ref.append(q.copy())
        if i < n_total:
            for _ in range(sub):
                q = rk4(q, hq / sub)

    def at(t):
        return ref[int(round((t + T0) / hq))]

    errs = []
    for dt in (dt0, dt0 / 2, dt0 / 4):
        s = make_mr(2)
        s.dt_min = dt
        s.q = at(0.0).copy()
        hist = [[] for _ in range(3)]
        for l in (1, 2):
            dtl = dt * 2 ** (l - 1)
            sel = s.levels == l
            hist[l] = [s.rhs(at(-dtl), B)[:, sel, :], s.rhs(at(-2 * dtl), B)[:, sel, :]]
        s._mr = {"hist": hist, "half": s.q.copy(), "tick": 0}
        s.run(int(round(T / (2 * dt))))
        errs.append(np.max(np.abs(s.q - at(T))))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 6.5), (errs, ratios)


# --------------------------------------------------------------- limiters
def _pp_solver():
    return make(W.small_wetdry(n=6, N=3), Params(cfl=0.2))


def test_pp_limiter_invariants():
    s = _pp_solver()
    rng = np.random.default_rng(4)
    K, Np = s.q[0].shape
    q = np.stack([rng.uniform(-0.05, 0.3, (K, Np)), rng.normal(0, 0.1, (K, Np)),
                  rng.normal(0, 0.1, (K, Np))])
    q[0, :10] = rng.uniform(0.2, 0.3, (10, Np))          # some untouched elements
    q[0, 10:20] = rng.uniform(-0.02, 0.015, (10, Np))    # some dry, some negative means
    means = s.means(q)
    out, code, neg = s.pp_limit(q)
    mo = s.means(out)
    keep = code == PP_KEEP
    scaled = code == PP_SCALED
    dry = code == PP_DRY
    assert keep.sum() >= 10 and scaled.sum() > 0 and dry.sum() > 0
    assert np.array_equal(out[:, keep], q[:, keep])
    assert np.max(np.abs(mo[:, scaled] - means[:, scaled])) < 1e-14
    assert np.max(np.abs(mo[0, dry] - np.maximum(means[0, dry], 0))) < 1e-14
    assert np.all(out[1:, dry] == 0.0)
    assert np.all(out[0] >= 0.0)
    # theta < 1 puts the lowest vertex exactly on h0
    vert = out[0] @ s.ref.p1_vert.T
    tight = scaled & (vert.min(axis=1) < means[0] - 1e-12)
    h1 = (q[0] @ s.ref.p1_vert.T).min(axis=1)
    theta_lt1 = tight & (h1 < s.p.h0)
    assert theta_lt1.sum() > 0
    assert np.max(np.abs(vert[theta_lt1].min(axis=1) - s.p.h0)) < 1e-14
    assert np.all(out[0, scaled] >= s.p.h0 - 1e-14)
    # idempotent
    out2, _, _ = s.pp_limit(out)
    assert np.max(np.abs(out2 - out)) < 1e-14
    assert neg == int(np.sum(means[0][~keep] < 0))


def test_tvb_keeps_linear_and_constant_data():
    wl = W.lake_at_rest(n=8, N=3)
    ins = wl.instances[0]
    s = Solver(ins.vx, ins.vy, ins.etov, 3, Params(tvb_M=0.0))
    x, y = s.nodes()
    q = np.stack([1.0 + 0.3 * x - 0.2 * y, 0.1 + 0.05 * x + 0.02 * y, -0.03 + 0.04 * y])
    pp = np.zeros(s.K, dtype=np.uint8)
    out, code = s.tvb_limit(q, pp)
    st = s.stencil
    inner = ~s.mesh.wall.any(axis=1) & np.all(st.pair[:, :, 0] != st.pair[:, :, 1], axis=1)
    assert inner.sum() > 20
    assert np.max(np.abs(out[:, inner] - q[:, inner])) < 1e-13
    assert np.all(code[inner] == 1)
    qc = np.stack([np.full_like(x, 0.7), np.full_like(x, 0.1), np.full_like(x, -0.2)])
    outc, _ = s.tvb_limit(qc, pp)
    assert np.max(np.abs(outc - qc)) < 1e-14


def test_tvb_limits_discontinuity_preserving_means_and_positivity():
    wl = W.lake_at_rest(n=8, N=3)
    ins = wl.instances[0]
    s = Solver(ins.vx, ins.vy, ins.etov, 3, Params(tvb_M=0.0, h0=1e-3))
    x, y = s.nodes()
    rng = np.random.default_rng(7)
    h = np.where(x + 0.3 * y < 0.55, 1.0, 0.002) + 0.001 * rng.uniform(size=x.shape) * x
    q = np.stack([h, 0.3 * h * np.sin(3 * y), 0.1 * h])
    pp = np.zeros(s.K, dtype=np.uint8)
    before = s.means(q)
    out, code = s.tvb_limit(q, pp)
    after = s.means(out)
    assert np.sum(code >= 2) > 0 and np.sum(code == 3) > 0
    assert np.max(np.abs(after - before)) < 1e-13
    vert = out[0] @ s.ref.p1_vert.T
    lim = code >= 2
    assert np.all(vert[lim].min(axis=1) >= s.p.h0 - 1e-12)
    # limited elements are linear
    assert np.max(np.abs(out[:, lim] @ s.ref.proj1.T - out[:, lim])) < 1e-12


def test_tvb_skips_dry_and_their_neighbours():
    s = _pp_solver()
    q = s.q.copy()
    pp = s.flags.pp.copy()
    k = int(np.nonzero(~s.mesh.wall.any(axis=1) & (pp != PP_DRY))[0][0])
    pp[k] = PP_DRY
    _, code = s.tvb_limit(q, pp)
    assert code[k] == 0
    for k2, wall in zip(s.mesh.etoe[k], s.mesh.wall[k]):
        if not wall:
            assert code[k2] == 0


# ------------------------------------------------------------ whole solver
def test_wetdry_run_conserves_mass_and_positivity():
    s = make(W.small_wetdry(n=10, N=3), Params(cfl=0.2))
    m0 = s.mass()
    for _ in range(120):
        s.step()
        assert np.all(s.q[0] >= 0.0)
        assert np.all(np.isfinite(s.q))
    assert sum(fc[2] for fc in s.flag_counts) == 0
    assert abs(s.mass() - m0) / m0 < 1e-12
    pp_tot = sum(fc[0] for fc in s.flag_counts)
    assert pp_tot[1] > 0 and pp_tot[2] > 0


def test_mrab_wetdry_positivity_and_mass():
    """The graded beach with its hump, 10 coarse steps of the multi-rate
    schedule: depth stays non-negative after every coarse step, no mean goes
    negative, and mass is conserved to roundoff (walls all round; the dry
    coarse levels exchange no flux)."""
    wl = W.graded_beach(N=3)
    s = make(wl, Params(g=wl.g, cfl=wl.cfl, max_levels=4))
    m0 = s.mass()
    for _ in range(10):
        s.run(1)
        assert np.all(s.q[0] >= 0.0) and np.all(np.isfinite(s.q))
    assert abs(s.mass() - m0) / m0 < 1e-12
    assert s.flags.pp.max() == PP_DRY


def test_graded_beach_shoreline_conditioning():
    """How far the multi-rate wet/dry case at N = 1 (thin films on the
    shoreline) is determined by its data: perturbing the initial surface
    level by 6e-8 relative (the FP32 rounding of the stored level), once,
    moves the FP64 momentum after 10 coarse steps by more than 1e-6 relative.
    The GPU parity bound of that case rests on this figure."""
    from helpers import rel_l2
    wl = W.graded_beach(N=1)
    ins = wl.instances[0]

    def run(seed):
        s = Solver(ins.vx, ins.vy, ins.etov, 1, Params(g=wl.g, cfl=wl.cfl, max_levels=wl.max_levels))
        x, y = s.nodes()
        B = s.interpolate(ins.bathymetry)
        h, hu, hv = ins.initial(x, y)
        if seed:
            rng = np.random.default_rng(seed)
            eta = 0.55 + (h + B - 0.55) * (1.0 + rng.uniform(-6e-8, 6e-8, h.shape))
            h = np.where(h > 0.0, np.maximum(eta - B, 0.0), 0.0)
        s.set_state(h, hu, hv, B)
        s.run(10)
        return s

    a = run(0)
    errs = [rel_l2(a, run(seed).q, a.q)["m"] for seed in (1, 2)]
    assert max(errs) > 1e-6, errs
    assert max(errs) < 1e-5, errs


def test_pp_negative_mean_with_wet_nodes_is_dry():
    """At N = 4 the nodal mean weights of the three vertices are negative, so
    an element wet at its vertices and nearly dry elsewhere has every node
    above eps and a negative mean (checked here through the constant modal
    coefficient, not the nodal weights).  The limiter makes it dry instead of
    keeping it."""
    wl = W.lake_at_rest(n=3, N=4)
    ins = wl.instances[0]
    s = Solver(ins.vx, ins.vy, ins.etov, 4, Params())
    ref = s.ref
    assert np.sum(ref.w < 0) == 3
    h = np.full((s.K, ref.Np), 1e-4)
    vert = [int(np.argmin((ref.r - a) ** 2 + (ref.s - b) ** 2)) for a, b in ((-1, -1), (1, -1), (-1, 1))]
    h[0, vert] = 1.0
    mean_modal = np.linalg.solve(ref.V, h[0])[0] / np.sqrt(2.0)
    assert mean_modal < 0.0 and h[0].min() > s.p.eps
    q = np.stack([h, 0.1 * h, -0.1 * h])
    out, code, neg = s.pp_limit(q)
    assert code[0] == PP_DRY and neg == 1
    assert np.all(out[:, 0] == 0.0)
    assert np.all(code[1:] == PP_KEEP)


def test_near_dry_front_stays_finite_at_order_4():
    """The deep-water / thin-film front at N = 4 with M = 0: without the
    negative-mean rule above, the limiter's characteristic speed of such an
    element is the square root of a negative mean and the run fails in its
    first step."""
    wl = W.near_dry_front(N=4)
    s = make(wl, Params(cfl=wl.cfl, tvb_M=0.0, h0=1e-3))
    m0 = s.mass()
    for _ in range(5):
        s.step()
        assert np.all(np.isfinite(s.q)) and np.all(s.q[0] >= 0.0)
    tv = sum(fc[1] for fc in s.flag_counts)
    assert tv[3] > 0   # Eq. 5.3 at work
    assert abs(s.mass() - m0) / m0 < 1e-3


# ------------------------------------------------------------- regrouping
def test_regroup_history_remap_exact_for_quadratics():
    """The re-sampling of a level change: a right-hand side that is a
    quadratic in time is re-sampled exactly at the new step (coarser and
    finer), and an unchanged level is an exact identity."""
    wl = W.graded_beach(N=1)
    ins = wl.instances[0]
    s = Solver(ins.vx, ins.vy, ins.etov, 1, Params(max_levels=4, regroup_every=3, pp=False, tvb=False))
    x, y = s.nodes()
    s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry), limit=False)
    rng = np.random.default_rng(3)
    c = rng.normal(size=(3, 3, s.K, s.ref.Np))
    R = lambda t: c[0] + c[1] * t + c[2] * t * t   # noqa: E731
    lev0 = s.levels.copy()
    dt0 = s.dt_min * 2.0 ** (lev0 - 1)
    hist = [[] for _ in range(5)]
    for l in range(1, 5):
        sel = lev0 == l
        hist[l] = [R(-(i + 1) * dt0[None, :, None])[:, sel, :] for i in range(3)] if np.any(sel) else []
    s._mr = {"hist": [list(h) for h in hist], "half": s.q.copy(), "tick": 0}
    s.set_levels(lev0, s.dt_min)
    for l in range(1, 5):
        for a, b in zip(s._mr["hist"][l], hist[l]):
            assert np.array_equal(a, b)
    new = np.clip(lev0 + np.where(np.arange(s.K) % 2 == 0, 1, -1), 1, 4)
    s.set_levels(new, 0.75 * s.dt_min)
    dtn = s.dt_min * 2.0 ** (new - 1)
    for l in range(1, 5):
        sel = new == l
        for i, a in enumerate(s._mr["hist"][l]):
            want = R(-(i + 1) * dtn[None, :, None])[:, sel, :]
            assert np.max(np.abs(a - want)) < 1e-12 * np.max(np.abs(want))


def test_regroup_keeps_third_order():
    """Two-level multi-rate AB3 from an exact history, with every element
    moved to the other level every third coarse step (the shortest regroup
    period: by then each level's three history samples are its own right-hand
    sides again): the error against a fine RK4 reference still falls at
    third order.  Each move re-samples the history with an O(dt^3) error, so a
    linear re-sampling would leave O(dt^2) after the O(1/dt) moves."""
    wl = W.c3(n0=2, n_bands=2)
    ins = wl.instances[0]

    def make_mr():
        s = Solver(ins.vx, ins.vy, ins.etov, 2, Params(g=wl.g, cfl=0.3, max_levels=2, pp=False, tvb=False))
        x, y = s.nodes()
        s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry), limit=False)
        return s

    s0 = make_mr()
    dt0, B = s0.dt_min, s0.B
    hq, T0, T, sub = dt0 / 4, 4 * dt0, 24 * dt0, 16

    def rk4(q, h):
        k1 = s0.rhs(q, B)
        k2 = s0.rhs(q + 0.5 * h * k1, B)
        k3 = s0.rhs(q + 0.5 * h * k2, B)
        k4 = s0.rhs(q + h * k3, B)
        return q + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    q = s0.q.copy()
    ref = []
    n_total = int(round((T0 + T) / hq))
    for i in range(n_total + 1):
        ref.append(q.copy())
        if i < n_total:
            for _ in range(sub):
                q = rk4(q, hq / sub)

    def at(t):
        return ref[int(round((t + T0) / hq))]

    errs = []
    for dt in (dt0, dt0 / 2, dt0 / 4):
        s = make_mr()
        s.dt_min = dt
        s.q = at(0.0).copy()
        hist = [[] for _ in range(3)]
        for l in (1, 2):
            dtl = dt * 2 ** (l - 1)
            sel = s.levels == l
            hist[l] = [s.rhs(at(-dtl), B)[:, sel, :], s.rhs(at(-2 * dtl), B)[:, sel, :],
                       s.rhs(at(-3 * dtl), B)[:, sel, :]]
        s._mr = {"hist": hist, "half": s.q.copy(), "tick": 0}
        for c in range(int(round(T / (2 * dt)))):
            s.run(1)
            if c % 3 == 2:
                # every element to the other level; the finest step stays dt
                # (levels 1 and 2 swap, which the 2:1 rule allows for two levels)
                s.set_levels(3 - s.levels, dt)
        errs.append(np.max(np.abs(s.q - at(T))))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 6.5), (errs, ratios)


def test_regroup_follows_the_wave_speeds():
    """On the graded wet/dry beach the regrouped levels move with the flow
    (some element changes level within 8 coarse steps), the run stays
    non-negative, and regrouping every step equals never regrouping while no
    level changes (the re-sampling is then the identity)."""
    wl = W.graded_beach(N=2)
    ins = wl.instances[0]

    def make(regroup):
        s = Solver(ins.vx, ins.vy, ins.etov, 2, Params(g=wl.g, cfl=wl.cfl, max_levels=4, regroup_every=regroup))
        x, y = s.nodes()
        s.set_state(*ins.initial(x, y), s.interpolate(ins.bathymetry))
        return s

    a = make(3)
    lev0 = a.levels.copy()
    changed = False
    m0 = a.mass()
    for _ in range(12):
        a.run(1)
        changed |= not np.array_equal(a.levels, lev0)
    assert changed
    assert a.q[0].min() >= 0.0
    assert abs(a.mass() - m0) < 1e-5 * m0
    b, c = make(3), make(10 ** 6)
    b.run(3)
    c.run(3)
    assert np.array_equal(b.q, c.q)
    if np.array_equal(b.levels, c.levels):
        b.run(1)
        c.run(1)
        assert np.array_equal(b.q, c.q)
    with pytest.raises(ValueError):
        make(2)
