"""Seeded synthetic inputs for the DG shallow-water hot path.

This module only builds inputs: conforming triangulations (vertex coordinates
and counter-clockwise element-to-vertex lists) and the analytic bathymetry and
initial-state functions that each side evaluates at its own nodes.  It holds
none of the method's arithmetic (no reference element, no fluxes, no limiters,
no time stepping) and is the only code shared by the FP64 oracle and the HIP
path.

Workloads (all seeded with ``numpy.random.default_rng(seed)``):

* ``c1``  unit square, 16x16 cells split in two, N=3, flat bed, Gaussian hump
          on depth 1, reflective walls, 200 AB3 steps at CFL 0.5, limiters on.
* ``c2``  unit square, 256x256 jittered cells (131072 triangles), N=4,
          sloping beach B = 0.8x plus eight Gaussian bumps, still level 0.5,
          wet/dry, 500 steps at CFL 0.2 (AB3 at a wet/dry front is unstable
          at 0.3 and above).
* ``c3``  [0,4]x[0,1] in four bands whose cell size halves per band
          (496098 triangles), N=3, B = 0.9 (x/4)^2, right-going N-wave,
          100 coarse steps of multi-rate AB3.
* ``c4``  [0,2]x[0,1], 1024x512 jittered cells (1048576 triangles), N=5,
          smooth random bed of 16 Fourier modes, fully wet, 300 steps.
* ``c5``  ensemble of 64 jittered unit squares with log-uniform sizes in
          [1e4, 2e5] triangles, N=3, per-instance beach slope and hump,
          200 steps each.

Bathymetry ``B`` is bed elevation; the free surface is ``eta = h + B``.
Bathymetry functions return plain FP64 values (no rounding to a grid the FP32
device could represent exactly).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

G_DEFAULT = 9.81


@dataclass
class Instance:
    """One triangulated domain with its analytic data."""

    vx: np.ndarray            # (Nv,) float64
    vy: np.ndarray            # (Nv,) float64
    etov: np.ndarray          # (K, 3) int32, counter-clockwise
    bathymetry: Callable[[np.ndarray, np.ndarray], np.ndarray]
    initial: Callable[[np.ndarray, np.ndarray], tuple]   # -> (h, hu, hv)
    label: str = ""
    bc: Optional[np.ndarray] = None   # (K, 3) face tags, 1 = wall (internal barriers)


@dataclass
class Workload:
    name: str
    N: int
    instances: List[Instance]
    steps: int
    cfl: float = 0.5
    g: float = G_DEFAULT
    limiters: bool = True
    max_levels: int = 1
    seed: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return int(sum(inst.etov.shape[0] for inst in self.instances))

    @property
    def Np(self) -> int:
        return (self.N + 1) * (self.N + 2) // 2


# --------------------------------------------------------------------------
# triangulations
# --------------------------------------------------------------------------

def structured_mesh(nx: int, ny: int, x0: float, x1: float, y0: float, y1: float,
                    jitter: float = 0.0, rng: Optional[np.random.Generator] = None):
    """nx-by-ny cells on [x0,x1]x[y0,y1]; each cell is cut along its
    lower-left to upper-right diagonal into (v00, v10, v11) and (v00, v11, v01).

    Vertices are numbered row-major (index j*(nx+1)+i), cells row-major, two
    triangles per cell.  With ``jitter > 0`` every interior vertex moves by
    independent U[-jitter*dx, jitter*dx] and U[-jitter*dy, jitter*dy] offsets;
    boundary vertices stay fixed.
    """
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(xs, ys)            # (ny+1, nx+1)
    vx = X.ravel().copy()
    vy = Y.ravel().copy()
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs an rng")
        dx = (x1 - x0) / nx
        dy = (y1 - y0) / ny
        jx = rng.uniform(-jitter * dx, jitter * dx, size=(ny + 1, nx + 1))
        jy = rng.uniform(-jitter * dy, jitter * dy, size=(ny + 1, nx + 1))
        interior = np.zeros((ny + 1, nx + 1), dtype=bool)
        interior[1:-1, 1:-1] = True
        vx = vx + np.where(interior, jx, 0.0).ravel()
        vy = vy + np.where(interior, jy, 0.0).ravel()
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    v00 = (j * (nx + 1) + i).ravel()
    v10 = v00 + 1
    v01 = v00 + (nx + 1)
    v11 = v01 + 1
    etov = np.empty((2 * nx * ny, 3), dtype=np.int32)
    etov[0::2] = np.stack([v00, v10, v11], axis=1)
    etov[1::2] = np.stack([v00, v11, v01], axis=1)
    return vx, vy, etov


def graded_band_mesh(n0: int, n_bands: int, height: float = 1.0):
    """[0, n_bands] x [0, height] in unit-wide bands; band b holds
    (n0*2^b) x (n0*2^b*height) square cells.  Interior cells are cut in two
    as in :func:`structured_mesh`; the last cell column of every band except
    the finest meets twice as many vertices on its right edge, so each such
    cell is cut into three triangles (v00,v10,m), (v00,m,v01), (v01,m,v11)
    with m the midpoint vertex of its right edge.  Element order: band by
    band, then row-major.
    """
    vx_list, vy_list = [], []
    etov_list = []
    vid = {}

    def vertex(x: float, y: float) -> int:
        # exact keys: every coordinate is a dyadic rational times 1/n0
        key = (round(x * n0 * 2 ** (n_bands + 1)), round(y * n0 * 2 ** (n_bands + 1)))
        idx = vid.get(key)
        if idx is None:
            idx = len(vx_list)
            vid[key] = idx
            vx_list.append(x)
            vy_list.append(y)
        return idx

    for b in range(n_bands):
        n = n0 * 2 ** b
        ny = int(round(n * height))
        h = 1.0 / n
        for j in range(ny):
            for i in range(n):
                xa, xb = b + i * h, b + (i + 1) * h
                ya, yb = j * h, (j + 1) * h
                v00, v10 = vertex(xa, ya), vertex(xb, ya)
                v01, v11 = vertex(xa, yb), vertex(xb, yb)
                if i == n - 1 and b < n_bands - 1:
                    m = vertex(xb, 0.5 * (ya + yb))
                    etov_list += [(v00, v10, m), (v00, m, v01), (v01, m, v11)]
                else:
                    etov_list += [(v00, v10, v11), (v00, v11, v01)]
    return (np.asarray(vx_list, dtype=np.float64), np.asarray(vy_list, dtype=np.float64),
            np.asarray(etov_list, dtype=np.int32))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def _zeros_like(x):
    return np.zeros_like(np.asarray(x, dtype=np.float64))


def c1(nx: int = 16) -> Workload:
    vx, vy, etov = structured_mesh(nx, nx, 0.0, 1.0, 0.0, 1.0)

    def bath(x, y):
        return _zeros_like(x)

    def init(x, y):
        h = 1.0 + 0.1 * np.exp(-100.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2))
        return h, _zeros_like(x), _zeros_like(x)

    return Workload("c1", 3, [Instance(vx, vy, etov, bath, init, "c1")], steps=200,
                    cfl=0.5, seed=1,
                    notes="unit square 16x16x2, N=3, flat bed, Gaussian hump on depth 1")


def beach_bathymetry(rng: np.random.Generator, n_bumps: int = 8, slope: float = 0.8,
                     amp: float = 0.05, width: float = 0.05):
    cx = rng.uniform(0.0, 1.0, size=n_bumps)
    cy = rng.uniform(0.0, 1.0, size=n_bumps)

    def bath(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        b = slope * x
        for k in range(n_bumps):
            b = b + amp * np.exp(-((x - cx[k]) ** 2 + (y - cy[k]) ** 2) / width ** 2)
        return b

    return bath, (cx, cy)


def c2(n: int = 256, seed: int = 2) -> Workload:
    rng = np.random.default_rng(seed)
    vx, vy, etov = structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0, jitter=0.2, rng=rng)
    bath, _ = beach_bathymetry(rng)

    def init(x, y):
        eta = 0.5 + 0.05 * np.exp(-100.0 * ((x - 0.6) ** 2 + (y - 0.5) ** 2))
        h = np.maximum(0.0, eta - bath(x, y))
        return h, _zeros_like(x), _zeros_like(x)

    return Workload("c2", 4, [Instance(vx, vy, etov, bath, init, "c2")], steps=500,
                    cfl=0.2, seed=seed,
                    notes=f"unit square {n}x{n}x2 jittered, N=4, beach 0.8x + 8 bumps, "
                          "still level 0.5, hump 0.05 at (0.6,0.5), wet/dry")


def c3(n0: int = 54, seed: int = 3, n_bands: int = 4) -> Workload:
    rng = np.random.default_rng(seed)
    vx, vy, etov = graded_band_mesh(n0, n_bands)
    xc = rng.uniform(0.4, 0.6)
    w = rng.uniform(0.05, 0.1)
    g = G_DEFAULT
    L = float(n_bands)

    def bath(x, y):
        return 0.9 * (np.asarray(x, dtype=np.float64) / L) ** 2

    def init(x, y):
        x = np.asarray(x, dtype=np.float64)
        d = 1.0 - bath(x, y)
        z = (x - xc) / w
        etap = -0.02 * z * np.exp(0.5 - 0.5 * z * z)
        return d + etap, etap * np.sqrt(g * d), _zeros_like(x)

    return Workload("c3", 3, [Instance(vx, vy, etov, bath, init, "c3")], steps=100,
                    cfl=0.5, max_levels=n_bands, seed=seed,
                    notes=f"graded bands n0={n0}, N=3, B=0.9(x/4)^2, N-wave xc={xc:.4f} w={w:.4f}",
                    extra={"xc": xc, "w": w})


def fourier_bathymetry(rng: np.random.Generator, n_modes: int = 16, amp: float = 0.1,
                       mean_depth: float = 1.0, lx: float = 2.0, ly: float = 1.0):
    k = rng.integers(1, 5, size=n_modes)
    l = rng.integers(1, 5, size=n_modes)
    a = rng.uniform(-1.0, 1.0, size=n_modes)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)

    def f(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        s = np.zeros(np.broadcast(x, y).shape)
        for m in range(n_modes):
            s = s + a[m] * np.cos(2.0 * np.pi * (k[m] * x / lx + l[m] * y / ly) + phi[m])
        return s

    # normalisation over a fixed lattice, independent of any node set
    gx, gy = np.meshgrid(np.linspace(0.0, lx, 1025), np.linspace(0.0, ly, 513))
    fmax = float(np.max(np.abs(f(gx, gy))))

    def bath(x, y):
        return -mean_depth + amp * f(x, y) / fmax

    return bath


def c4(nx: int = 1024, ny: int = 512, seed: int = 4) -> Workload:
    rng = np.random.default_rng(seed)
    vx, vy, etov = structured_mesh(nx, ny, 0.0, 2.0, 0.0, 1.0, jitter=0.2, rng=rng)
    bath = fourier_bathymetry(rng)

    def init(x, y):
        eta = 0.1 * np.exp(-100.0 * ((x - 1.0) ** 2 + (y - 0.5) ** 2))
        return eta - bath(x, y), _zeros_like(x), _zeros_like(x)

    return Workload("c4", 5, [Instance(vx, vy, etov, bath, init, "c4")], steps=300,
                    cfl=0.5, seed=seed,
                    notes=f"[0,2]x[0,1] {nx}x{ny}x2 jittered, N=5, 16 Fourier modes amp 0.1 "
                          "about depth 1, hump 0.1 at (1,0.5), fully wet")


def c5(n_inst: int = 64, seed: int = 5, kmin: float = 1e4, kmax: float = 2e5) -> Workload:
    rng = np.random.default_rng(seed)
    ktil = np.exp(rng.uniform(np.log(kmin), np.log(kmax), size=n_inst))
    ns = np.maximum(2, np.rint(np.sqrt(ktil / 2.0)).astype(int))
    insts = []
    for i in range(n_inst):
        n = int(ns[i])
        vx, vy, etov = structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0, jitter=0.2, rng=rng)
        slope = rng.uniform(0.3, 1.0)
        amp = rng.uniform(0.01, 0.1)
        cx, cy = rng.uniform(0.0, 1.0, size=2)

        def bath(x, y, slope=slope):
            return slope * np.asarray(x, dtype=np.float64)

        def init(x, y, slope=slope, amp=amp, cx=cx, cy=cy):
            x = np.asarray(x, dtype=np.float64)
            y = np.asarray(y, dtype=np.float64)
            eta = 0.5 + amp * np.exp(-100.0 * ((x - cx) ** 2 + (y - cy) ** 2))
            return np.maximum(0.0, eta - bath(x, y)), _zeros_like(x), _zeros_like(x)

        insts.append(Instance(vx, vy, etov, bath, init, f"c5[{i}] n={n}"))
    return Workload("c5", 3, insts, steps=200, cfl=0.2, seed=seed,
                    notes="64 jittered unit squares, log-uniform sizes, beach + hump each")


def lake_at_rest(n: int = 4, N: int = 3, jitter: float = 0.2, seed: int = 11,
                 level: float = 1.0) -> Workload:
    """Fully wet still water over a non-constant bed (exact steady state)."""
    rng = np.random.default_rng(seed)
    vx, vy, etov = structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0, jitter=jitter, rng=rng)

    def bath(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return 0.2 * np.sin(2.0 * np.pi * x) * np.cos(np.pi * y) + 0.1 * x * y

    def init(x, y):
        return level - bath(x, y), _zeros_like(x), _zeros_like(x)

    return Workload("lake", N, [Instance(vx, vy, etov, bath, init, "lake")], steps=50,
                    cfl=0.5, seed=seed, notes="lake at rest")


def graded_beach(n0: int = 2, N: int = 3, n_bands: int = 4) -> Workload:
    """Multi-rate wet/dry case: the graded band mesh of ``c3`` under a plane
    beach B = 0.3 (4 - x) whose shoreline (still level 0.55, x ~ 2.17) runs
    through the second-finest band next to the interface with the coarser
    bands, which are dry; a hump 0.1 exp(-100 r^2) at (2.3, 0.5) straddles
    the shoreline.  Walls all round."""
    vx, vy, etov = graded_band_mesh(n0, n_bands)

    def bath(x, y):
        return 0.3 * (float(n_bands) - np.asarray(x, dtype=np.float64))

    def init(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        eta = 0.55 + 0.1 * np.exp(-100.0 * ((x - 2.3) ** 2 + (y - 0.5) ** 2))
        h = np.maximum(0.0, eta - bath(x, y))
        return h, _zeros_like(x), _zeros_like(x)

    return Workload("graded_beach", N, [Instance(vx, vy, etov, bath, init, "graded_beach")],
                    steps=10, cfl=0.3, max_levels=n_bands, seed=0,
                    notes=f"graded bands n0={n0}, N={N}, B=0.3(4-x), still level 0.55, hump at (2.3, 0.5)")


def stepped_bed(case: str = "lake", n: int = 8, N: int = 3, seed: int = 13,
                steps: int = 200) -> Workload:
    """A bed that jumps across every face: on a jittered n x n x 2 unit square,
    element k's bed is 0.1 x + 0.04 r_k (r_k ~ U[-1, 1] per element, drawn from
    the seed) plus a step of height ``step`` on the elements whose first
    vertex lies at x > 0.5.  The bathymetry function takes nodal arrays of
    shape (K, Np) in element order (row k = element k), which is how both the
    oracle and the library present their nodes.

    * ``lake``:  still level 1.0 over a step of 0.3, fully wet (the discrete
      steady state that hydrostatic reconstruction, Eq. 5.1-5.2, keeps);
    * ``dam``:   the same bed, surface 1.1 for x < 0.3 and 1.0 beyond, at rest;
    * ``ledge``: a step of 0.6 under still level 0.5 with a hump 0.1
      exp(-50 r^2) at (0.4, 0.5): the elements beyond the step are dry and
      their bed rises above the wet neighbours' surface."""
    rng = np.random.default_rng(seed)
    vx, vy, etov = structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0, jitter=0.2, rng=rng)
    K = etov.shape[0]
    r = rng.uniform(-1.0, 1.0, size=K)
    step = {"lake": 0.3, "dam": 0.3, "ledge": 0.6}[case]
    on_step = vx[etov[:, 0]] > 0.5

    def bath(x, y):
        x = np.asarray(x, dtype=np.float64)
        if x.ndim != 2 or x.shape[0] != K:
            raise ValueError("stepped_bed bathymetry takes (K, Np) nodal arrays in element order")
        return 0.1 * x + (0.04 * r + step * on_step)[:, None]

    def init(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        if case == "lake":
            eta = np.ones_like(x)
        elif case == "dam":
            eta = np.where(x < 0.3, 1.1, 1.0)
        else:
            eta = 0.5 + 0.1 * np.exp(-50.0 * ((x - 0.4) ** 2 + (y - 0.5) ** 2))
        h = np.maximum(0.0, eta - bath(x, y))
        return h, _zeros_like(x), _zeros_like(x)

    return Workload(f"stepped_{case}", N, [Instance(vx, vy, etov, bath, init, f"stepped_{case}")],
                    steps=steps, cfl=0.2, seed=seed,
                    notes=f"stepped bed ({case}) {n}x{n}x2 jittered, N={N}, jump on every face")


def skewed_patch(N: int = 2) -> Workload:
    """Four triangles around a flat central one whose neighbour barycentres do
    not surround its own: two of its edges find no neighbour pair with
    non-negative weights and take the one-neighbour fallback of the TVB
    stencil.  One neighbour is a sliver.  Flat bed, walls all round, a depth
    step at x = 0.6 plus a slope in y (every element is limited)."""
    vx = np.array([0.0, 1.0, 0.5, 3.0, 1.2, -0.2])
    vy = np.array([0.0, 0.0, 0.3, -0.05, 0.5, 0.5])
    etov = np.array([[0, 1, 2], [0, 3, 1], [1, 4, 2], [2, 5, 0]], dtype=np.int64)

    def bath(x, y):
        return _zeros_like(np.asarray(x, dtype=np.float64))

    def init(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        h = 1.0 + 0.3 * (x > 0.6) + 0.2 * y
        return h, _zeros_like(x), _zeros_like(x)

    return Workload("skewed_patch", N, [Instance(vx, vy, etov, bath, init, "skewed_patch")],
                    steps=10, cfl=0.3, notes="TVB stencil fallback case")


def near_dry_front(N: int = 3, n: int = 8, seed: int = 7) -> Workload:
    """A depth front between deep water (h = 1) and a thin film (h ~ 0.002)
    along x + 0.3 y = 0.55 on a jittered n x n x 2 unit square, flat bed,
    momentum (0.3 h sin 3y, 0.1 h): run with M = 0 and h0 = 1e-3, limited
    elements next to the film take the depth modification of Eq. 5.3, and at
    N = 4 some elements with every node wet have a negative mean."""
    rng = np.random.default_rng(seed)
    vx, vy, etov = structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0, jitter=0.2, rng=rng)

    def bath(x, y):
        return _zeros_like(np.asarray(x, dtype=np.float64))

    def init(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        h = np.where(x + 0.3 * y < 0.55, 1.0, 0.002) + 0.001 * x * (0.5 + 0.5 * np.sin(17.0 * x + 5.0 * y))
        return h, 0.3 * h * np.sin(3.0 * y), 0.1 * h

    return Workload("near_dry_front", N, [Instance(vx, vy, etov, bath, init, "near_dry_front")],
                    steps=5, cfl=0.2, seed=seed, notes="deep water against a thin film")


def small_wetdry(n: int = 8, N: int = 3, seed: int = 12, steps: int = 40) -> Workload:
    """A small beach with a hump straddling the shoreline (exercises both limiters)."""
    rng = np.random.default_rng(seed)
    vx, vy, etov = structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0, jitter=0.2, rng=rng)
    bath, _ = beach_bathymetry(rng, n_bumps=2)

    def init(x, y):
        eta = 0.5 + 0.05 * np.exp(-100.0 * ((x - 0.6) ** 2 + (y - 0.5) ** 2))
        return np.maximum(0.0, eta - bath(x, y)), _zeros_like(x), _zeros_like(x)

    return Workload("wetdry", N, [Instance(vx, vy, etov, bath, init, "wetdry")], steps=steps,
                    cfl=0.2, seed=seed, notes="small beach")


def barrier_basin(n: int = 16, N: int = 3, gap: tuple = (0.375, 0.625), steps: int = 60) -> Workload:
    """Unit square with an internal wall along x = 1/2 (tagged faces) that
    leaves an opening for gap[0] < y < gap[1]; flat bed at depth 1 and a
    Gaussian hump cut off at x = 1/2, so the right basin starts at rest.  n
    must be even so that x = 1/2 is a grid line."""
    if n % 2:
        raise ValueError("n must be even")
    vx, vy, etov = structured_mesh(n, n, 0.0, 1.0, 0.0, 1.0)
    a = etov
    b = np.roll(etov, -1, axis=1)
    on_line = (np.abs(vx[a] - 0.5) < 1e-12) & (np.abs(vx[b] - 0.5) < 1e-12)
    ymid = 0.5 * (vy[a] + vy[b])
    bc = (on_line & ((ymid < gap[0]) | (ymid > gap[1]))).astype(np.int8)

    def bath(x, y):
        return _zeros_like(np.asarray(x, dtype=np.float64))

    def init(x, y):
        x = np.asarray(x, dtype=np.float64)
        hump = 0.1 * np.exp(-100.0 * ((x - 0.25) ** 2 + (y - 0.5) ** 2))
        h = 1.0 + np.where(x < 0.5, hump, 0.0)   # the right basin starts exactly at rest
        return h, _zeros_like(x), _zeros_like(x)

    return Workload("barrier", N, [Instance(vx, vy, etov, bath, init, "barrier", bc=bc)], steps=steps,
                    cfl=0.5, notes=f"barrier basin {n}x{n}x2, N={N}, opening {gap}")


def shoreline_lake(n: int = 16, N: int = 2, steps: int = 600) -> Workload:
    """Still water of depth 0.1 in the paraboloid B = 0.1 (x^2 + y^2) on
    [-2, 2]^2: the shoreline r = 1 crosses elements, so partially wet
    elements are not a discrete steady state (a thin-film stress case)."""
    vx, vy, etov = structured_mesh(n, n, -2.0, 2.0, -2.0, 2.0)

    def bath(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return 0.1 * (x * x + y * y)

    def init(x, y):
        h = np.maximum(0.0, 0.1 - bath(x, y))
        return h, _zeros_like(h), _zeros_like(h)

    return Workload("shoreline", N, [Instance(vx, vy, etov, bath, init, "shoreline")], steps=steps,
                    cfl=0.2, notes=f"still water with a shoreline {n}x{n}x2, N={N}")


# ---------------------------------------------------------------------------
# Closed-form wet/dry cases of the paper's numerical section.  Each workload
# carries ``extra["exact"](x, y, t) -> (h, hu, hv)`` (the printed solution),
# ``extra["t0"]`` (the time of the initial state), ``extra["t_end"]`` and
# ``extra["hvel"]``, the depth below which velocities are desingularised
# (the paper says nothing about velocities in thin films; the two curved-bed
# cases need it at a few per cent of their depth scale, see each case).


def parabolic_bowl(n: int = 16, N: int = 2, t_end_periods: float = 0.25) -> Workload:
    """Thacker's periodic flow in a paraboloid bed (Section 6, parabolic
    bowl): B = alpha r^2 on the 8000 m square centred at the origin, alpha =
    1.6e-7, X = 1, Y = -0.41884, omega^2 = 8 g alpha; h is the printed
    quadratic in r inside the moving shoreline and zero outside, u and v are
    linear in x and y.  The water never reaches the walls.  Positivity limiter
    only (the TVB limiter off), as Table 6.1 lists for this case."""
    alpha, X, Y = 1.6e-7, 1.0, -0.41884
    g = G_DEFAULT
    om = math.sqrt(8.0 * g * alpha)
    vx, vy, etov = structured_mesh(n, n, -4000.0, 4000.0, -4000.0, 4000.0)

    def bath(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return alpha * (x * x + y * y)

    def exact(x, y, t):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        den = X + Y * math.cos(om * t)
        r2 = x * x + y * y
        h = np.maximum(0.0, 1.0 / den + alpha * (Y * Y - X * X) * r2 / (den * den))
        f = -Y * om * math.sin(om * t) / den * 0.5
        return h, h * f * x, h * f * y

    period = 2.0 * math.pi / om
    return Workload("bowl", N, [Instance(vx, vy, etov, bath, lambda x, y: exact(x, y, 0.0), "bowl")],
                    steps=0, cfl=0.2, g=g, notes=f"parabolic bowl {n}x{n}x2, N={N}",
                    extra={"exact": exact, "t0": 0.0, "t_end": t_end_periods * period, "period": period,
                           "local_radius": 500.0, "hvel": 0.1, "tvb": False})


def rarefaction(nx: int = 20, N: int = 2, t_end: float = 10.0, cfl: float = 0.1,
                width: float = 2.5) -> Workload:
    """Dam-break rarefaction into a dry bed on a flat bottom (Section 6,
    rarefaction wave): g = 1, h0 = 1, xi = (x - 20)/t; still water h0 for
    xi < -sqrt(g h0), dry for xi > 2 sqrt(g h0), and h = (xi - 2 sqrt(g
    h0))^2 / (9 g), u = 2/3 (xi + sqrt(g h0)) between.  The flow is
    independent of y, so a strip of the given width (cells as close to
    square as its width allows) stands for the 50 x 40 domain; the state at
    t = 2 is the initial condition and the TVB limiter is off, as in the
    paper."""
    g, h0 = 1.0, 1.0
    Lx = 50.0
    ny = max(1, int(round(nx * width / Lx)))
    vx, vy, etov = structured_mesh(nx, ny, 0.0, Lx, 0.0, width)
    c0 = math.sqrt(g * h0)

    def bath(x, y):
        return _zeros_like(np.asarray(x, dtype=np.float64))

    def exact(x, y, t):
        x = np.asarray(x, dtype=np.float64)
        xi = (x - 20.0) / t
        h = np.where(xi < -c0, h0, np.where(xi > 2.0 * c0, 0.0, (xi - 2.0 * c0) ** 2 / (9.0 * g)))
        u = np.where((xi >= -c0) & (xi <= 2.0 * c0), 2.0 / 3.0 * (xi + c0), 0.0)
        return h, h * u, _zeros_like(x)

    return Workload("rarefaction", N, [Instance(vx, vy, etov, bath, lambda x, y: exact(x, y, 2.0), "rare")],
                    steps=0, cfl=cfl, g=g, notes=f"rarefaction strip {nx}x{ny}x2, N={N}",
                    extra={"exact": exact, "t0": 2.0, "t_end": t_end, "local_x": (15.0, 35.0), "tvb": False,
                           "width": width, "hvel": 1e-3})


def oscillating_lake(n: int = 16, N: int = 2, t_end_periods: float = 1.0) -> Workload:
    """Planar free surface rotating in a paraboloid bed (Section 6,
    oscillating lake): [-2,2]^2, B = h0 (x^2 + y^2) / a^2 with a = 1,
    h0 = 0.1, sigma = 0.5, omega = sqrt(2 g h0) / a; h = max(0, sigma h0 /
    a^2 (2x cos wt + 2y sin wt - sigma) + h0 - B), u = -sigma w sin wt,
    v = sigma w cos wt; reflecting walls, both limiters on."""
    a, h0, sg = 1.0, 0.1, 0.5
    g = G_DEFAULT
    om = math.sqrt(2.0 * g * h0) / a
    vx, vy, etov = structured_mesh(n, n, -2.0, 2.0, -2.0, 2.0)

    def bath(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return h0 * (x * x + y * y) / (a * a)

    def exact(x, y, t):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        b = h0 * (x * x + y * y) / (a * a)
        h = np.maximum(0.0, sg * h0 / (a * a) * (2.0 * x * math.cos(om * t) + 2.0 * y * math.sin(om * t) - sg)
                       + h0 - b)
        return h, h * (-sg * om * math.sin(om * t)), h * (sg * om * math.cos(om * t))

    period = 2.0 * math.pi / om
    return Workload("lake", N, [Instance(vx, vy, etov, bath, lambda x, y: exact(x, y, 0.0), "lake")],
                    steps=0, cfl=0.2, g=g, notes=f"oscillating lake {n}x{n}x2, N={N}",
                    extra={"exact": exact, "t0": 0.0, "t_end": t_end_periods * period, "period": period,
                           "hvel": 1e-2})


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


def get(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
