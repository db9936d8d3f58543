"""Seeded synthetic inputs for the augmented-wavefield (WRI) problems.

This module only *describes* problems: grids, velocity models (squared
slowness m = 1/v^2), source/receiver cell indices, frequencies, the data
weight lambda, per-system tolerances, the true source weights and synthetic
observed data.  It contains none of the method's arithmetic (no Helmholtz
operator, no sponge, no solve).  Both the CPU oracle and the GPU path consume
these objects; neither shares anything else.

Cell layout everywhere: x fastest, linear index (z*ny + y)*nx + x, z pointing
down with z = 0 the top face.

Observed data.  The paper's models are figure-only and its lab dataset is not
available, so the data here are synthetic stand-ins: the free-space Green's
function of a homogeneous medium (the velocity at the source), scaled by the
true source weight and the cell volume, plus 1 % complex Gaussian noise.  The
tiny configuration instead takes its clean data from a true-model solve done by
the caller (the oracle), then adds noise with :func:`add_noise`.

Source weights follow the paper's source tables (Camembert and VSP examples):
the true weight at frequency f is 10*exp(-i*2*pi*f*0.10) and the initial
("wrong") weight 10*exp(-i*2*pi*f*0.11).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Grid", "System", "Problem", "cell_index", "alpha_true", "alpha_initial",
    "add_noise", "layered_model", "make_config", "CONFIG_NAMES", "custom_problem",
]

KNOWN = "known"
ESTIMATE = "estimate"


@dataclass(frozen=True)
class Grid:
    """A regular 3D grid: nx*ny*nz cells of spacing h [m]; sponge of nb cells
    on every face, parameterised by the reference velocity v_ref [m/s]."""
    nx: int
    ny: int
    nz: int
    h: float
    nb: int
    v_ref: float

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        """numpy shape, slowest axis first: (nz, ny, nx)."""
        return (self.nz, self.ny, self.nx)


@dataclass
class System:
    """One (source i, frequency j) right-hand side."""
    grid: int                 # index into Problem.grids
    freq: float               # [Hz]
    lam: float                # data weight (J = ||A u - a e||^2 + lam^2 ||P u - d||^2)
    src: int                  # linear cell index of the point source
    rec: np.ndarray           # int32 linear cell indices of the receivers (distinct)
    d: np.ndarray             # complex128 observed data at the receivers
    alpha: complex            # source weight used in KNOWN mode
    rtol: float               # tolerance on the normal-equation residual

    @property
    def omega(self) -> float:
        return 2.0 * np.pi * self.freq


@dataclass
class Problem:
    name: str
    grids: List[Grid]
    m: List[np.ndarray]          # per grid, float64 (nz, ny, nx): model at which J, g are evaluated
    m_true: List[np.ndarray]     # per grid, model that generated the data
    systems: List[System]
    mode: str = ESTIMATE
    max_iter: int = 20000
    notes: dict = field(default_factory=dict)

    def with_data(self, d_list: Sequence[np.ndarray]) -> "Problem":
        systems = [replace(s, d=np.asarray(d, dtype=np.complex128)) for s, d in zip(self.systems, d_list)]
        return replace(self, systems=systems)

    def with_rtol(self, rtol) -> "Problem":
        if np.isscalar(rtol):
            rtol = [float(rtol)] * len(self.systems)
        systems = [replace(s, rtol=float(r)) for s, r in zip(self.systems, rtol)]
        return replace(self, systems=systems)

    def subset(self, idx: Sequence[int]) -> "Problem":
        return replace(self, systems=[self.systems[i] for i in idx])


def cell_index(grid: Grid, x, y, z):
    """Linear index of cell (x, y, z): x fastest."""
    return (np.asarray(z) * grid.ny + np.asarray(y)) * grid.nx + np.asarray(x)


def alpha_true(freq: float) -> complex:
    """True source weight (matches the paper's Camembert/VSP source tables)."""
    return complex(10.0 * np.exp(-2j * np.pi * freq * 0.10))


def alpha_initial(freq: float) -> complex:
    """Initial (wrong) source weight of the paper's inversions: 0.11 s delay."""
    return complex(10.0 * np.exp(-2j * np.pi * freq * 0.11))


def add_noise(d: np.ndarray, rng: np.random.Generator, level: float = 0.01) -> np.ndarray:
    """1 % complex Gaussian noise: sigma = level*||d||/sqrt(n_r) per entry,
    split equally between the real and imaginary parts."""
    d = np.asarray(d, dtype=np.complex128)
    if d.size == 0:
        return d.copy()
    sigma = level * np.linalg.norm(d) / np.sqrt(d.size)
    noise = (rng.standard_normal(d.size) + 1j * rng.standard_normal(d.size)) * (sigma / np.sqrt(2.0))
    return d + noise


def layered_model(shape, interfaces, velocities, anomaly_center=None, anomaly_sigma=None,
                  anomaly_amp=0.10):
    """Velocity model [m/s] on (nz, ny, nx): horizontal layers with the given
    interface depths (cell units, z of the first cell of each deeper layer) and
    layer velocities; optionally a Gaussian velocity perturbation of relative
    amplitude anomaly_amp at anomaly_center = (x, y, z) cells, width sigma cells.
    Returns (v_layers, v_with_anomaly)."""
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64)
    layer = np.searchsorted(np.asarray(interfaces, dtype=np.float64), z, side="right")
    v1d = np.asarray(velocities, dtype=np.float64)[layer]
    v0 = np.broadcast_to(v1d[:, None, None], shape).copy()
    if anomaly_center is None:
        return v0, v0.copy()
    cx, cy, cz = anomaly_center
    r2 = ((np.arange(nx) - cx) ** 2)[None, None, :] + ((np.arange(ny) - cy) ** 2)[None, :, None] \
        + ((np.arange(nz) - cz) ** 2)[:, None, None]
    v1 = v0 * (1.0 + anomaly_amp * np.exp(-r2 / (2.0 * anomaly_sigma ** 2)))
    return v0, v1


def _random_layers(rng: np.random.Generator, n_depth: int, n_ref: int = 64):
    """Five layers: 4 interfaces uniform in [12, 52] cells of a 64-cell depth
    (scaled to n_depth), velocities 1500, three sorted uniform draws in
    [1500, 4500], 4500 m/s."""
    interfaces = np.sort(rng.uniform(12.0, 52.0, 4)) * (n_depth / n_ref)
    vel = np.concatenate([[1500.0], np.sort(rng.uniform(1500.0, 4500.0, 3)), [4500.0]])
    return interfaces, vel


def _greens_data(grid: Grid, v: np.ndarray, src: int, rec: np.ndarray, freq: float,
                 alpha: complex) -> np.ndarray:
    """Free-space Green's-function data for a point source of weight alpha on
    one cell: alpha*h^3*(-exp(-i k r)/(4 pi r)), k = omega / v(src)."""
    sx = src % grid.nx
    sy = (src // grid.nx) % grid.ny
    sz = src // (grid.nx * grid.ny)
    rx = rec % grid.nx
    ry = (rec // grid.nx) % grid.ny
    rz = rec // (grid.nx * grid.ny)
    r = grid.h * np.sqrt((rx - sx) ** 2.0 + (ry - sy) ** 2.0 + (rz - sz) ** 2.0)
    r = np.maximum(r, 0.5 * grid.h)
    k = 2.0 * np.pi * freq / v.reshape(-1)[src]
    return alpha * grid.h ** 3 * (-np.exp(-1j * k * r) / (4.0 * np.pi * r))


def _finish(name, grids, v0s, v1s, geom, freqs_per_grid, lam_per_grid, rtols, mode, seed,
            data: str, max_iter=20000, notes=None) -> Problem:
    """Assemble a Problem: one System per (frequency, source), frequency-major."""
    rng = np.random.default_rng(seed + 1000)
    systems = []
    k = 0
    for gi, g in enumerate(grids):
        srcs, rec = geom[gi]
        rec = np.asarray(rec, dtype=np.int32)
        for f in freqs_per_grid[gi]:
            for s in srcs:
                if data == "green":
                    d = add_noise(_greens_data(g, v1s[gi], int(s), rec, f, alpha_true(f)), rng)
                else:
                    d = np.zeros(rec.size, dtype=np.complex128)
                systems.append(System(grid=gi, freq=float(f), lam=float(lam_per_grid[gi]),
                                      src=int(s), rec=rec, d=d, alpha=alpha_true(f),
                                      rtol=float(rtols[k])))
                k += 1
    return Problem(name=name, grids=list(grids), m=[1.0 / v ** 2 for v in v0s],
                   m_true=[1.0 / v ** 2 for v in v1s], systems=systems, mode=mode,
                   max_iter=max_iter, notes=dict(notes or {}))


def _n_systems(freqs_per_grid, geom):
    return sum(len(f) * len(g[0]) for f, g in zip(freqs_per_grid, geom))


def make_config(name: str, seed: int = 0, data: str = "green") -> Problem:
    """Build one of the named workloads.

    data: "green" -> synthetic Green's-function data + 1 % noise;
          "none"  -> zero data (the caller fills it, e.g. from a true-model solve).
    Names: tiny, medium, uneven, differentiation, crop32, large.
    """
    if name == "tiny":
        g = Grid(16, 16, 16, 10.0, 4, 2000.0)
        v0, v1 = layered_model(g.shape, [8.0], [2000.0, 3000.0], (7.5, 7.5, 7.5), 2.0)
        src = [int(cell_index(g, 8, 8, 4))]
        rec = cell_index(g, 12, 8, np.arange(16))
        return _finish("tiny", [g], [v0], [v1], [(src, rec)], [[8.0]], [1.0], [1e-10],
                       ESTIMATE, seed, data, notes={"precision": "complex128"})
    if name == "medium":
        rng = np.random.default_rng(seed)
        g = Grid(64, 64, 64, 10.0, 10, 1500.0)
        interfaces, vel = _random_layers(rng, 64)
        c = rng.uniform(16.0, 48.0, 3)
        v0, v1 = layered_model(g.shape, interfaces, vel, tuple(c), 4.0)
        src = [int(cell_index(g, 14 + 5 * k, 32, 10)) for k in range(8)]
        rec = cell_index(g, 20, 32, np.arange(64))
        return _finish("medium", [g], [v0], [v1], [(src, rec)], [[6.0]], [12.0 / g.h ** 2],
                       [1e-4] * 8, ESTIMATE, seed, data)
    if name == "uneven":
        rng = np.random.default_rng(seed)
        interfaces64, vel = _random_layers(rng, 64)
        c64 = rng.uniform(16.0, 48.0, 3)
        freqs = [5.0, 8.0, 12.0]
        grids, v0s, v1s, geom = [], [], [], []
        for f, n in zip(freqs, (48, 64, 96)):
            h = 1500.0 / (8.0 * f)
            g = Grid(n, n, n, h, 8, 1500.0)
            s = n / 64.0
            v0, v1 = layered_model(g.shape, interfaces64 * s, vel, tuple(c64 * s), 4.0 * s)
            xs = np.round(np.linspace(g.nb, n - 1 - g.nb, 32)).astype(int)
            srcs = [int(cell_index(g, x, n // 2, g.nb)) for x in xs]
            zr = np.arange(g.nb, n - g.nb)
            rec = cell_index(g, n // 4, n // 2, zr)
            grids.append(g); v0s.append(v0); v1s.append(v1); geom.append((srcs, rec))
        rtols = 10.0 ** (-2.0 - 3.0 * np.random.default_rng(seed).uniform(size=96))
        return _finish("uneven", grids, v0s, v1s, geom, [[f] for f in freqs],
                       [12.0 / g.h ** 2 for g in grids], rtols, ESTIMATE, seed, data)
    if name in ("differentiation", "crop32"):
        rng = np.random.default_rng(seed)
        n = 128
        interfaces, vel = _random_layers(rng, n)
        c = rng.uniform(16.0, 48.0, 3) * (n / 64.0)
        full = Grid(n, n, n, 10.0, 10, 1500.0)
        v0, v1 = layered_model(full.shape, interfaces, vel, tuple(c), 4.0)
        freqs = [5.0, 7.0, 9.0]
        if name == "differentiation":
            pos = (24, 48, 80, 104)
            srcs = [int(cell_index(full, x, y, 10)) for y in pos for x in pos]
            rec = cell_index(full, 64, 64, np.arange(n))
            return _finish(name, [full], [v0], [v1], [(srcs, rec)], [freqs], [0.12],
                           [1e-4] * 48, ESTIMATE, seed, data)
        g = Grid(32, 32, 32, 10.0, 6, 1500.0)
        sl = slice(48, 80)
        v0c, v1c = v0[sl, sl, sl].copy(), v1[sl, sl, sl].copy()
        pos = (9, 13, 19, 23)
        srcs = [int(cell_index(g, x, y, 7)) for y in pos for x in pos]
        rec = cell_index(g, 16, 16, np.arange(32))
        return _finish(name, [g], [v0c], [v1c], [(srcs, rec)], [freqs], [0.12],
                       [1e-8] * 48, ESTIMATE, seed, data)
    if name == "large":
        rng = np.random.default_rng(seed)
        g = Grid(256, 256, 192, 10.0, 12, 1500.0)
        interfaces, vel = _random_layers(rng, 192)
        c = rng.uniform(0.25, 0.75, 3) * np.array([256, 256, 192])
        v0, v1 = layered_model(g.shape, interfaces, vel, tuple(c), 4.0)
        xs = np.round(np.linspace(g.nb + 16, 255 - g.nb - 16, 8)).astype(int)
        srcs = [int(cell_index(g, x, y, 12)) for y in xs for x in xs]
        rec = np.concatenate([cell_index(g, wx, wy, 12 + 2 * np.arange(64))
                              for wy in (64, 192) for wx in (64, 192)])
        freqs = [4.0, 6.0, 8.0, 10.0, 12.0, 14.0]
        return _finish(name, [g], [v0], [v1], [(srcs, rec)], [freqs], [0.12],
                       [1e-2] * 384, ESTIMATE, seed, data)
    raise ValueError(f"unknown config {name!r}")


CONFIG_NAMES = ("tiny", "medium", "uneven", "differentiation", "crop32", "large")


def custom_problem(shape_xyz, h=10.0, nb=3, freqs=(6.0,), n_src=2, n_rec=8, lam=None,
                   seed=0, rtol=1e-8, mode=ESTIMATE, v=(1800.0, 2600.0), data="green",
                   homogeneous=False) -> Problem:
    """Small seeded problem on an arbitrary (possibly ragged) grid, for parity
    tests: two layers plus a Gaussian anomaly, sources on a line near the top,
    receivers in a vertical well."""
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    g = Grid(nx, ny, nz, float(h), int(nb), float(min(v)))
    if homogeneous:
        v0 = np.full(g.shape, float(v[0])); v1 = v0.copy()
    else:
        v0, v1 = layered_model(g.shape, [nz / 2.0], list(v),
                               (nx / 2.0 + 0.3, ny / 2.0 - 0.2, nz / 2.0 + 0.1),
                               max(1.0, min(nx, ny, nz) / 8.0))
    zsrc = min(nb + 1, nz - 1)
    xs = rng.choice(np.arange(nx), size=min(n_src, nx), replace=False)
    ys = rng.integers(0, ny, size=xs.size)
    srcs = [int(cell_index(g, x, y, zsrc)) for x, y in zip(xs, ys)]
    wx, wy = int(rng.integers(0, nx)), int(rng.integers(0, ny))
    zr = np.sort(rng.choice(np.arange(nz), size=min(n_rec, nz), replace=False))
    rec = cell_index(g, wx, wy, zr)
    if n_rec > nz:   # more receivers than one well holds: add a second well
        wx2 = (wx + nx // 2) % nx
        extra = cell_index(g, wx2, wy, np.arange(min(n_rec - nz, nz)))
        rec = np.unique(np.concatenate([rec, extra]))
    if lam is None:
        lam = 12.0 / h ** 2
    nsys = len(freqs) * len(srcs)
    rtols = [rtol] * nsys if np.isscalar(rtol) else list(rtol)
    return _finish(f"custom{tuple(shape_xyz)}", [g], [v0], [v1], [(srcs, rec)], [list(freqs)],
                   [lam], rtols, mode, seed, data)
