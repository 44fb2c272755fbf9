"""Seeded synthetic inputs for the Jefimenko field evaluation.

This module produces grids and source histories (charge density rho and
current density J sampled on a cell-centred source grid at equally spaced
time steps).  It holds none of the field method's arithmetic: no retarded
time, no interpolation, no 1/R kernels.  Both the oracle and the HIP path
consume what it produces; neither is imported here.

Conventions
-----------
* A grid is ``Grid(n=(nx, ny, nz), origin=(x0, y0, z0), spacing=(dx, dy, dz))``.
  The centre of cell (i, j, k) is ``origin + (i, j, k) * spacing`` and the
  linear cell index is ``i + nx * (j + ny * k)`` (x fastest).
* A history is an FP64 array ``h[step][channel][cell]`` with channel 0 = rho
  and channels 1..3 = Jx, Jy, Jz.  Step ``s`` sits at time ``t0 + s * dt``.
* Workload sizes follow the paper's problem statement (two independent
  uniform grids, a resident history of ``lts`` slices, section "Parameter
  dependence"), with Gaussian charge blobs as sources.  The paper's own two
  analytic source families (constant step sources and the sinusoidal pair,
  section "Comparisons with the theoretical results") are provided too.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "Grid", "Blob", "Problem", "centred_grid", "cell_centres", "blob_history",
    "constant_step_history", "sinusoidal_history", "draw_blobs", "config_tiny",
    "config_medium", "config_large", "batch_instances", "serving_trace",
    "default_screen",
]


@dataclass(frozen=True)
class Grid:
    n: Tuple[int, int, int]
    origin: Tuple[float, float, float]
    spacing: Tuple[float, float, float]

    @property
    def size(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def shifted_cells(self, di: int, dj: int, dk: int) -> "Grid":
        """The same grid moved by a whole number of cells along each axis."""
        o = tuple(self.origin[a] + (di, dj, dk)[a] * self.spacing[a] for a in range(3))
        return Grid(self.n, o, self.spacing)


def centred_grid(n: Sequence[int], dx: float) -> Grid:
    """Cell-centred grid of ``n`` cells with spacing ``dx`` centred on 0."""
    n3 = tuple(int(v) for v in n)
    return Grid(n3, tuple(-(v - 1) / 2.0 * dx for v in n3), (dx, dx, dx))


def cell_centres(g: Grid) -> np.ndarray:
    """FP64 [n_cells, 3] cell centres in linear (x fastest) order."""
    nx, ny, nz = g.n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.empty((g.size, 3), dtype=np.float64)
    out[:, 0] = g.origin[0] + i.reshape(-1).astype(np.float64) * g.spacing[0]
    out[:, 1] = g.origin[1] + j.reshape(-1).astype(np.float64) * g.spacing[1]
    out[:, 2] = g.origin[2] + k.reshape(-1).astype(np.float64) * g.spacing[2]
    return out


def default_screen(src: Grid) -> Tuple[float, float, float]:
    """Screening half-widths: half the source spacing per axis (the paper
    takes the screening length as half the grid length)."""
    return tuple(0.5 * s for s in src.spacing)


@dataclass(frozen=True)
class Blob:
    q: float                       # total charge
    sigma: float                   # Gaussian width
    centre: Tuple[float, float, float]
    velocity: Tuple[float, float, float]


def blob_history(g: Grid, blobs: Sequence[Blob], steps: Sequence[int] | int,
                 dt: float, t0: float = 0.0) -> np.ndarray:
    """Sample rho and J = sum_i rho_i v_i of moving Gaussian blobs.

    rho_i(r, t) = q_i (2 pi sigma_i^2)^(-3/2) exp(-|r - c_i - v_i t|^2 / (2 sigma_i^2)).
    Returns FP64 ``h[len(steps)][4][n_cells]`` for absolute ``steps`` at
    times ``t0 + s * dt`` (an int means steps 0..n-1).  The Gaussian factors
    per axis, so each slice is a sum of outer products of 1-D profiles.
    """
    if isinstance(steps, (int, np.integer)):
        steps = list(range(int(steps)))
    nx, ny, nz = g.n
    ax = [g.origin[a] + np.arange(g.n[a], dtype=np.float64) * g.spacing[a] for a in range(3)]
    q = np.array([b.q for b in blobs], dtype=np.float64)
    sig = np.array([b.sigma for b in blobs], dtype=np.float64)
    cen = np.array([b.centre for b in blobs], dtype=np.float64).reshape(-1, 3)
    vel = np.array([b.velocity for b in blobs], dtype=np.float64).reshape(-1, 3)
    norm = q * (2.0 * math.pi * sig ** 2) ** -1.5
    out = np.zeros((len(steps), 4, g.size), dtype=np.float64)
    if len(blobs) == 0:
        return out
    weights = np.stack([norm, norm * vel[:, 0], norm * vel[:, 1], norm * vel[:, 2]])  # [4][K]
    for si, s in enumerate(steps):
        t = t0 + s * dt
        c = cen + vel * t
        prof = [np.exp(-((ax[a][None, :] - c[:, a:a + 1]) ** 2) / (2.0 * sig[:, None] ** 2))
                for a in range(3)]  # [K][n_a]
        zy = (prof[2][:, :, None] * prof[1][:, None, :]).reshape(len(blobs), nz * ny)  # [K][nz*ny]
        for ch in range(4):
            out[si, ch] = ((zy * weights[ch][:, None]).T @ prof[0]).reshape(-1)
    return out


def constant_step_history(g: Grid, steps: Sequence[int] | int, dt: float,
                          t0: float = 0.0, rho: float = 1.0,
                          J: Tuple[float, float, float] = (1.0, 1.0, 1.0)) -> np.ndarray:
    """The paper's constant sources: rho = 1, J = (1, 1, 1) for t >= 0 and
    zero before (section "Constant sources")."""
    if isinstance(steps, (int, np.integer)):
        steps = list(range(int(steps)))
    out = np.zeros((len(steps), 4, g.size), dtype=np.float64)
    for si, s in enumerate(steps):
        if t0 + s * dt >= 0.0:
            out[si, 0] = rho
            out[si, 1:4] = np.asarray(J, dtype=np.float64)[:, None]
    return out


def sinusoidal_history(g: Grid, steps: Sequence[int] | int, dt: float,
                       t0: float = 0.0) -> np.ndarray:
    """The paper's sinusoidal sources (section "Sinusoidal sources"):
    rho = 3 (cos t - 1) cos(x + y + z) and jx = jy = jz = sin(x + y + z) sin t
    for t >= 0, zero before.  They satisfy div J + d rho / dt = 0."""
    if isinstance(steps, (int, np.integer)):
        steps = list(range(int(steps)))
    r = cell_centres(g)
    phase = r.sum(axis=1)
    out = np.zeros((len(steps), 4, g.size), dtype=np.float64)
    for si, s in enumerate(steps):
        t = t0 + s * dt
        if t >= 0.0:
            out[si, 0] = 3.0 * (math.cos(t) - 1.0) * np.cos(phase)
            j = np.sin(phase) * math.sin(t)
            out[si, 1] = j
            out[si, 2] = j
            out[si, 3] = j
    return out


def paper_source_factors(kind: str, t: float) -> Tuple[float, float]:
    """The paper's analytic sources as (time factor of rho, time factor of
    each J component) times fixed spatial patterns: "constant" -> patterns
    1 and 1; "sinusoidal" -> patterns cos(x + y + z) and sin(x + y + z).
    Zero before t = 0 (sections "Constant sources", "Sinusoidal sources")."""
    if t < 0.0:
        return 0.0, 0.0
    if kind == "constant":
        return 1.0, 1.0
    if kind == "sinusoidal":
        return 3.0 * (math.cos(t) - 1.0), math.sin(t)
    raise ValueError(kind)


def draw_blobs(rng: np.random.Generator, k: int, box: Tuple[float, float]) -> List[Blob]:
    """Blob parameters in a fixed draw order: centres (3k, uniform in the
    box), sigma (k, uniform in [0.05, 0.2]), charge (k, uniform in [-1, 1]),
    velocity (direction from 3k normals, speed 0.8 * U^(1/3): uniform in the
    ball of radius 0.8)."""
    lo, hi = box
    centres = rng.uniform(lo, hi, size=(k, 3))
    sigmas = rng.uniform(0.05, 0.2, size=k)
    charges = rng.uniform(-1.0, 1.0, size=k)
    dirs = rng.normal(size=(k, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    speeds = 0.8 * rng.uniform(0.0, 1.0, size=k) ** (1.0 / 3.0)
    vel = dirs * speeds[:, None]
    return [Blob(float(charges[i]), float(sigmas[i]), tuple(map(float, centres[i])),
                 tuple(map(float, vel[i]))) for i in range(k)]


@dataclass
class Problem:
    """One field evaluation: source grid, history, observation grid, time."""
    name: str
    src: Grid
    obs: Grid
    hist: np.ndarray            # FP64 [nt][4][n_src], oldest slice first
    dt: float
    t: float
    t0: float = 0.0             # time of absolute step 0
    newest: int = 0             # absolute step of hist[-1]
    c: float = 1.0
    screen: Tuple[float, float, float] = field(default=(0.0, 0.0, 0.0))
    blobs: list = field(default_factory=list)   # sources, when generated from blobs

    @property
    def nt(self) -> int:
        return int(self.hist.shape[0])

    @property
    def pairs(self) -> int:
        return self.src.size * self.obs.size


def _problem(name, src, obs, blobs, nt, dt):
    hist = blob_history(src, blobs, nt, dt)
    p = Problem(name, src, obs, hist, dt, t=(nt - 1) * dt, t0=0.0,
                newest=nt - 1, c=1.0, screen=default_screen(src))
    p.blobs = list(blobs)
    return p


def config_tiny() -> Problem:
    """8^3 source (dx 0.1) centred on 0, 16 slices (dt 0.05) of one blob
    (sigma 0.2, charge 1) moving at (0, 0, 0.5); 8^3 observation grid
    (spacing 0.1) shifted +1.0 in x; evaluated at t = 0.75; seed 0."""
    src = centred_grid((8, 8, 8), 0.1)
    obs = src.shifted_cells(10, 0, 0)
    blobs = [Blob(1.0, 0.2, (0.0, 0.0, 0.0), (0.0, 0.0, 0.5))]
    return _problem("tiny-8^3x8^3-nt16", src, obs, blobs, 16, 0.05)


def config_medium() -> Problem:
    """32^3 source (dx 0.05, box [-0.8, 0.8]^3), 64 slices (dt 0.025), 20
    seeded blobs; coincident 32^3 observation grid; t = newest; seed 1."""
    rng = np.random.default_rng(1)
    src = centred_grid((32, 32, 32), 0.05)
    blobs = draw_blobs(rng, 20, (-0.8, 0.8))
    return _problem("medium-32^3x32^3-nt64", src, src, blobs, 64, 0.025)


def config_large(obs_shift_cells: int = 32) -> Problem:
    """64^3 source (dx 0.025, box [-0.8, 0.8]^3), 128 slices (dt 0.0125),
    100 seeded blobs; 64^3 observation grid displaced by half a box
    (32 cells) in x; t = newest; seed 2."""
    rng = np.random.default_rng(2)
    src = centred_grid((64, 64, 64), 0.025)
    blobs = draw_blobs(rng, 100, (-0.8, 0.8))
    return _problem("large-64^3x64^3-nt128", src, src.shifted_cells(obs_shift_cells, 0, 0),
                    blobs, 128, 0.0125)


def batch_instances(count: int = 64, seed: int = 3, with_history: bool = True) -> List[Problem]:
    """Uneven independent problems: source edge from {8, 12, ..., 40},
    observation edge from {8, 12, ..., 48}, history of 2 * e_s + 8 slices,
    1..30 blobs each; box [-0.8, 0.8]^3, dx = 1.6 / e_s, dt = dx / 2;
    the observation grid shares the source spacing and sits centred on the
    source box at a whole-cell offset."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        es = int(rng.choice(np.arange(8, 41, 4)))
        eo = int(rng.choice(np.arange(8, 49, 4)))
        kb = int(rng.integers(1, 31))
        dx = 1.6 / es
        dt = dx / 2.0
        nt = 2 * es + 8
        src = centred_grid((es, es, es), dx)
        m = (es - eo) // 2
        obs = Grid((eo, eo, eo), tuple(src.origin[a] + m * dx for a in range(3)), (dx, dx, dx))
        blobs = draw_blobs(rng, kb, (-0.8, 0.8))
        if with_history:
            p = _problem(f"batch{i}-{es}^3x{eo}^3-nt{nt}", src, obs, blobs, nt, dt)
        else:
            p = Problem(f"batch{i}-{es}^3x{eo}^3-nt{nt}", src, obs,
                        np.zeros((0, 4, 0)), dt, t=(nt - 1) * dt, newest=nt - 1,
                        screen=default_screen(src))
        p.blobs = list(blobs)
        out.append(p)
    return out


def serving_trace(rate: float = 200.0, duration: float = 60.0, sessions: int = 128,
                  seed: int = 5):
    """A Poisson request stream over a pool of sessions.

    Returns (session_specs, requests).  Each session has a source edge
    round(exp U[ln 8, ln 48]), history capacity 2 e_s + 8, box
    [-0.8, 0.8]^3, dx = 1.6 / e_s, dt = dx / 2 and its own 1..30 blobs.  Each
    request names a uniformly drawn session, pushes that session's next
    slice and evaluates on an observation grid of edge
    round(exp U[ln 8, ln 64]) (same spacing, centred) at the newest time.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for s in range(sessions):
        es = int(round(math.exp(rng.uniform(math.log(8), math.log(48)))))
        kb = int(rng.integers(1, 31))
        dx = 1.6 / es
        specs.append(dict(session=s, edge=es, dx=dx, dt=dx / 2.0, capacity=2 * es + 8,
                          blobs=draw_blobs(rng, kb, (-0.8, 0.8))))
    n = int(rng.poisson(rate * duration))
    arrivals = np.sort(rng.uniform(0.0, duration, size=n))
    reqs = []
    for i in range(n):
        s = int(rng.integers(0, sessions))
        eo = int(round(math.exp(rng.uniform(math.log(8), math.log(64)))))
        reqs.append(dict(index=i, arrival=float(arrivals[i]), session=s, obs_edge=eo))
    return specs, reqs
