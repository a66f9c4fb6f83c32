"""The FP64 oracle against the closed-form wet/dry solutions of the paper's
numerical section: the rarefaction into a dry bed (PP limiter only), the
oscillating lake in a paraboloid (PP and TVB) and Thacker's parabolic bowl
(PP and TVB).  Each run starts from the exact state at t0 and is compared
with the exact depth after a fraction of the case's time scale on two or
three meshes: the error must be small, fall under refinement, conserve mass
to roundoff and keep every nodal depth non-negative.  A sign error in the
split bed source fails them; with a continuous bed the hydrostatic
reconstruction of Eq. 5.1 is the identity, so its face correction cannot be
probed here (the lake-at-rest and jump tests of the oracle cover it), and
the size of the Lax-Friedrichs dissipation moves these errors by a few per
cent only.  The error bounds are set about a third above the values these
runs give (rarefaction 1.41 %, 0.41 %, 0.15 %; lake 10.9 %, 5.9 %; bowl
9.4 %, 4.5 %)."""
from __future__ import annotations

import math
import warnings

import numpy as np
import pytest

import workloads as W
from helpers import closed_form_oracle, exact_errors


def _run(wl, t_end):
    o = closed_form_oracle(wl)
    mass0 = float(np.sum(o.mesh.J * (o.q[0] @ o.ref.w)))
    steps = int(round((t_end - wl.extra["t0"]) / o.dt_min))
    with warnings.catch_warnings():
        # the vectorised positivity limiter evaluates theta for every
        # triggered element and discards it for dry ones
        warnings.simplefilter("ignore", RuntimeWarning)
        o.run(steps)
    mass1 = float(np.sum(o.mesh.J * (o.q[0] @ o.ref.w)))
    assert np.all(np.isfinite(o.q))
    assert o.q[0].min() >= 0.0
    assert abs(mass1 - mass0) <= 1e-12 * mass0
    return o, wl.extra["t0"] + steps * o.dt_min


def test_rarefaction_converges_to_closed_form():
    """Dam break into a dry bed (Section 6, rarefaction wave), N = 2, from
    t = 2 to t = 4; the local region x in (17, 26) lies inside the smooth
    part of the fan at t = 4 (it spans 16 < x < 28)."""
    errs = []
    for nx, bound in ((20, 0.019), (40, 0.0055), (80, 0.0021)):
        wl = W.rarefaction(nx, 2)
        o, t = _run(wl, 4.0)
        x, _ = o.nodes()
        region = np.all((x > 17.0) & (x < 26.0), axis=1)
        e = exact_errors(o, o.q[0], wl, t, region)
        assert e["rel"] <= bound, (nx, e)
        errs.append(e)
        # the still-water side well behind the fan's tail (x = 20 - t) keeps
        # its depth up to the scheme's small precursors
        far = np.all(x < 10.0, axis=1)
        assert np.max(np.abs(o.q[0][far] - 1.0)) <= 1e-4
    for a, b in zip(errs, errs[1:]):
        assert math.log2(a["rel"] / b["rel"]) >= 1.2
        assert math.log2(a["local"] / b["local"]) >= 1.2


def test_rarefaction_dry_front_position():
    """The wet region ends at the front x = 20 + 2 sqrt(g h0) t: the last
    element holding water lies within two cells of it."""
    wl = W.rarefaction(40, 2)
    o, t = _run(wl, 4.0)
    x, _ = o.nodes()
    wet = o.q[0].max(axis=1) > 1e-4
    front = 20.0 + 2.0 * t
    cell = 50.0 / 40
    assert abs(x[wet].max() - front) <= 2.0 * cell


@pytest.mark.parametrize("case,meshes,bounds", [
    ("lake", (8, 16), (0.145, 0.079)),
    ("bowl", (8, 16), (0.125, 0.060)),
])
def test_curved_bed_cases_converge(case, meshes, bounds):
    """Oscillating lake (an eighth of a period) and parabolic bowl (a quarter
    of a period), N = 2, both limiters on."""
    errs = []
    for n, bound in zip(meshes, bounds):
        wl = W.oscillating_lake(n, 2) if case == "lake" else W.parabolic_bowl(n, 2)
        frac = 0.125 if case == "lake" else 0.25
        o, t = _run(wl, frac * wl.extra["period"])
        e = exact_errors(o, o.q[0], wl, t)
        assert e["rel"] <= bound, (n, e)
        errs.append(e["rel"])
    assert errs[1] < 0.65 * errs[0]
