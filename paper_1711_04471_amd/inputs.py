"""Seeded synthetic inputs for the 2-D shallow-water (2DSW) time loop.

This module only draws random numbers and lays out arrays. It holds none of the
model's arithmetic, so both the HIP path and the CPU oracle can be fed from it.

The paper's 2DSW test case (Sect. 6.2) gives the workload shape only: square
grids, a fixed number of time steps, a spatial step and a time step. It prints
no depth field, mask or initial state, so every input here is synthetic:

* bathymetry: 16 random Fourier modes (|k| <= 4) rescaled to 5..50 m depth;
* land: a 1-cell (or wider) land border plus random disks until at least 10 %
  of the interior is land;
* initial surface: a sum of Gaussian bumps (0.1..1 m, sigma 8..32 cells) with
  u = v = 0.

Arrays are row-major ``[ny][nx]``; ``j`` runs north, ``i`` runs east. Every
draw uses ``numpy.random.Generator(PCG64(seed))`` in a fixed order (modes, then
disks, then bumps). Values are generated in float64 and rounded once to
float32; both sides of a comparison read those same float32 values.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

G = 9.81


@dataclass
class Case:
    """One closed-basin 2DSW problem: grid, constants, static fields, state."""

    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    g: float
    dt: float
    eps: float
    H: np.ndarray  # float32 [ny][nx]; the value on land cells is ignored
    mask: np.ndarray  # uint8 [ny][nx]; 1 = water, 0 = land
    eta: np.ndarray  # float32 [ny][nx]
    u: np.ndarray  # float32 [ny][nx]; east face of each cell
    v: np.ndarray  # float32 [ny][nx]; north face of each cell
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def stable_dt(dx: float, dy: float, g: float, h_max: float, courant: float = 0.5) -> float:
    """Time step from the shallow-water wave speed: courant * min(dx, dy) / sqrt(g H_max)."""
    return courant * min(dx, dy) / math.sqrt(g * h_max)


def bathymetry(rng: np.random.Generator, nx: int, ny: int, n_modes: int = 16,
               h_min: float = 5.0, h_max: float = 50.0) -> np.ndarray:
    """Smooth depth from ``n_modes`` random Fourier modes, rescaled to [h_min, h_max] (float64)."""
    kx = np.empty(n_modes, dtype=np.int64)
    ky = np.empty(n_modes, dtype=np.int64)
    amp = np.empty(n_modes)
    phase = np.empty(n_modes)
    for m in range(n_modes):
        while True:
            a = int(rng.integers(-4, 5))
            b = int(rng.integers(0, 5))
            if a != 0 or b != 0:
                break
        kx[m], ky[m] = a, b
        amp[m] = rng.standard_normal() / math.sqrt(a * a + b * b)
        phase[m] = rng.uniform(0.0, 2.0 * math.pi)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    ax = 2.0 * math.pi * np.outer(kx, x) + phase[:, None]  # [m][nx]
    by = 2.0 * math.pi * np.outer(ky, y)  # [m][ny]
    # cos(ax + by) = cos(by) cos(ax) - sin(by) sin(ax), summed over modes as one product
    left = np.concatenate([np.cos(by).T * amp, -np.sin(by).T * amp], axis=1)  # [ny][2m]
    right = np.concatenate([np.cos(ax), np.sin(ax)], axis=0)  # [2m][nx]
    B = left @ right
    lo, hi = B.min(), B.max()
    return h_min + (h_max - h_min) * (B - lo) / (hi - lo)


def land_mask(rng: np.random.Generator, nx: int, ny: int, border: int = 1,
              land_fraction: float = 0.10) -> np.ndarray:
    """Land border of width ``border`` plus random land disks until the interior is >= 10 % land."""
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[border:ny - border, border:nx - border] = 1
    n_int = (nx - 2 * border) * (ny - 2 * border)
    land = 0
    side = min(nx, ny)
    while land < land_fraction * n_int:
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(0.0, ny)
        r = rng.uniform(0.01, 0.04) * side
        i0, i1 = max(border, int(cx - r) - 1), min(nx - border, int(cx + r) + 2)
        j0, j1 = max(border, int(cy - r) - 1), min(ny - border, int(cy + r) + 2)
        if i0 >= i1 or j0 >= j1:
            continue
        ii = np.arange(i0, i1) + 0.5
        jj = np.arange(j0, j1) + 0.5
        inside = (ii[None, :] - cx) ** 2 + (jj[:, None] - cy) ** 2 <= r * r
        box = mask[j0:j1, i0:i1]
        land += int(np.count_nonzero(inside & (box == 1)))
        box[inside] = 0
    return mask


def gaussian_bumps(rng: np.random.Generator, nx: int, ny: int, n_bumps: int,
                   a_range=(0.1, 1.0), sigma_range=(8.0, 32.0)) -> np.ndarray:
    """Sum of ``n_bumps`` Gaussian surface bumps in metres (float64); distances in cells."""
    eta = np.zeros((ny, nx))
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    for _ in range(n_bumps):
        a = rng.uniform(*a_range)
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(0.0, ny)
        s = rng.uniform(*sigma_range)
        gx = np.exp(-((x - cx) ** 2) / (2.0 * s * s))
        gy = np.exp(-((y - cy) ** 2) / (2.0 * s * s))
        eta += a * np.outer(gy, gx)
    return eta


def seeded_basin(name: str, nx: int, ny: int, dx: float, seed: int, n_bumps: int,
                 steps: int, border: int = 1, eps: float = 0.05, g: float = G,
                 bumps_range: tuple | None = None) -> Case:
    """A random closed basin: Fourier bathymetry, disk land mask, Gaussian bumps.

    ``bumps_range`` (lo, hi) draws the bump count uniformly instead of using ``n_bumps``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    H64 = bathymetry(rng, nx, ny)
    mask = land_mask(rng, nx, ny, border=border)
    if bumps_range is not None:
        n_bumps = int(rng.integers(bumps_range[0], bumps_range[1] + 1))
    eta64 = gaussian_bumps(rng, nx, ny, n_bumps)
    H = H64.astype(np.float32)
    eta = eta64.astype(np.float32)
    eta[mask == 0] = 0.0
    h_max = float(H[mask != 0].max())
    dt = stable_dt(dx, dx, g, h_max)
    z = np.zeros((ny, nx), dtype=np.float32)
    return Case(name, nx, ny, dx, dx, g, dt, eps, H, mask, eta, z, z.copy(), steps,
                meta={"seed": seed, "n_bumps": n_bumps, "border": border})


def gaussian_basin_64() -> Case:
    """64 x 64 wet interior plus a 1-cell land border, uniform 10 m depth, dx = 100 m.

    A 1 m Gaussian bump with sigma = 5 cells sits at the basin centre (32 dx, 32 dy from
    the west and south walls), u = v = 0, Shapiro eps = 0.05, dt = 0.5 dx / sqrt(g H),
    200 steps.
    """
    nx = ny = 66
    dx = 100.0
    g = G
    H = np.full((ny, nx), 10.0, dtype=np.float32)
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[1:-1, 1:-1] = 1
    # cell (j, i) has its centre at ((i - 1/2) dx, (j - 1/2) dy) from the walls
    xc = (np.arange(nx) - 0.5) * dx
    yc = (np.arange(ny) - 0.5) * dx
    s = 5.0 * dx
    r2 = (xc[None, :] - 32.0 * dx) ** 2 + (yc[:, None] - 32.0 * dx) ** 2
    eta = np.exp(-r2 / (2.0 * s * s)).astype(np.float32)
    eta[mask == 0] = 0.0
    dt = 0.5 * dx / math.sqrt(g * 10.0)
    z = np.zeros((ny, nx), dtype=np.float32)
    return Case("gaussian_basin_64", nx, ny, dx, dx, g, dt, 0.05, H, mask, eta, z, z.copy(), 200)


def basin_2048() -> Case:
    """2048 x 2048 cells (border included), dx = 500 m, seed 2, 8 bumps, 1000 steps."""
    return seeded_basin("basin_2048", 2048, 2048, 500.0, seed=2, n_bumps=8, steps=1000)


def basin_8192() -> Case:
    """8192 x 8192 cells (border included), dx = 250 m, seed 3, 8 bumps, 500 steps."""
    return seeded_basin("basin_8192", 8192, 8192, 250.0, seed=3, n_bumps=8, steps=500)


def row_strip(case: Case, j_lo: int, j_hi: int, halo: int) -> Case:
    """Rows [j_lo - halo, j_hi + halo) of ``case``: the rows one GPU of a row-strip split
    would hold (its own rows j_lo..j_hi-1 and ``halo`` rows of each neighbour), with the
    outermost row on each side turned to land so that the strip is a closed basin of that
    shape. Same dx, dt and eps as ``case``."""
    a, b = j_lo - halo, j_hi + halo
    if not (0 <= a < b <= case.ny and b - a >= 3):
        raise ValueError("strip rows outside the grid")
    mask = case.mask[a:b].copy()
    mask[0] = 0
    mask[-1] = 0
    eta = np.where(mask != 0, case.eta[a:b], 0.0).astype(np.float32)
    u = np.where(mask != 0, case.u[a:b], 0.0).astype(np.float32)
    v = np.where(mask != 0, case.v[a:b], 0.0).astype(np.float32)
    v[-2] = 0.0  # the north face of the last water row now borders land
    return Case(f"{case.name}_rows{j_lo}-{j_hi}_halo{halo}", case.nx, b - a, case.dx, case.dy, case.g, case.dt,
                case.eps, case.H[a:b].copy(), mask, eta, u, v, case.steps,
                meta={**case.meta, "rows": (j_lo, j_hi), "halo": halo})


def small_basin(nx: int, ny: int, seed: int, steps: int = 50, n_bumps: int = 3,
                dx: float = 500.0, eps: float = 0.05) -> Case:
    """A small seeded basin for parity tests (any shape, including ragged tile tails)."""
    return seeded_basin(f"basin_{nx}x{ny}_s{seed}", nx, ny, dx, seed=seed, n_bumps=n_bumps,
                        steps=steps, eps=eps)


def ensemble_sizes(n: int = 256, seed: int = 4, lo: int = 128, hi: int = 1024) -> list[tuple[int, int]]:
    """(nx, ny) of each ensemble member, uniform on {lo..hi} for both sides."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.integers(lo, hi + 1, size=(n, 2))
    return [(int(a), int(b)) for a, b in sides]


def ensemble_member(k: int, nx: int, ny: int, steps: int = 1000) -> Case:
    """Member ``k`` of the ensemble: seed 40000 + k, 1..4 bumps, dx = 500 m, its own dt."""
    return seeded_basin(f"member_{k}", nx, ny, 500.0, seed=40000 + k, n_bumps=1,
                        steps=steps, bumps_range=(1, 4))


def ensemble(n: int = 256, seed: int = 4, steps: int = 1000, sizes=None) -> list[Case]:
    """The ensemble of uneven basins (sides 128..1024 by default)."""
    sizes = sizes if sizes is not None else ensemble_sizes(n, seed)
    return [ensemble_member(k, nx, ny, steps) for k, (nx, ny) in enumerate(sizes)]


def shore_basin(nx: int, ny: int, seed: int, steps: int = 60, dx: float = 500.0, level: float = -1.0,
                n_bumps: int = 3, eps: float = 0.05) -> Case:
    """A basin with a beach, for wetting and drying: the seeded basin's depth (5..50 m below
    the datum) ramps down east of x = 0.6 nx to 0.2 m at x = 0.95 nx and stays there; the
    still water stands at ``level`` (below the datum), so ground shallower than -level is
    dry at rest with its surface on the ground (eta = -H). Bumps of 0.5..2 m are added on
    the cells that are under water at rest."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H64 = bathymetry(rng, nx, ny)
    mask = land_mask(rng, nx, ny)
    bumps = gaussian_bumps(rng, nx, ny, n_bumps, a_range=(0.5, 2.0))
    x = (np.arange(nx) + 0.5) / nx
    ramp = np.clip((0.95 - x) / 0.35, 0.0, 1.0)[None, :]
    H64 = 0.2 + (H64 - 0.2) * ramp
    under = (mask != 0) & (H64 + level > 0.0)
    eta64 = np.where(under, level + bumps, -H64)
    H = H64.astype(np.float32)
    eta = np.where(mask != 0, eta64, 0.0).astype(np.float32)
    h_max = float(H[mask != 0].max())
    dt = stable_dt(dx, dx, G, h_max)
    z = np.zeros((ny, nx), dtype=np.float32)
    return Case(f"shore_{nx}x{ny}_s{seed}", nx, ny, dx, dx, G, dt, eps, H, mask, eta, z, z.copy(), steps,
                meta={"seed": seed, "n_bumps": n_bumps, "level": level})


def lake_at_rest(nx: int, ny: int, seed: int, level: float = 0.25) -> Case:
    """Random depth and mask with a flat surface at ``level`` on wet cells and no flow."""
    c = seeded_basin(f"rest_{nx}x{ny}_s{seed}", nx, ny, 500.0, seed=seed, n_bumps=0, steps=20)
    c.eta = np.where(c.mask != 0, np.float32(level), np.float32(0.0)).astype(np.float32)
    return c


# --------------------------------------------------------------------------- pressure Poisson
@dataclass
class PoissonCase:
    """A pressure Poisson problem for red-black SOR: arrays [nz][ny][nx] (float32), the
    outermost layer of ``p0`` holds the fixed boundary values."""
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    omega: float
    iters: int
    p0: np.ndarray = field(repr=False)
    f: np.ndarray = field(repr=False)


def poisson_source(rng: np.random.Generator, nx: int, ny: int, nz: int, n_blobs: int = 8,
                   noise: float = 1e-3) -> np.ndarray:
    """Right-hand side: Gaussian blobs (amplitude U(-1, 1), sigma U(5, 20) cells in x and y,
    U(3, 12) cells in z, centre uniform) plus uniform noise of amplitude ``noise``; zero on
    the boundary layer."""
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    f = np.zeros((nz, ny, nx))
    for _ in range(n_blobs):
        a = rng.uniform(-1.0, 1.0)
        sx, sy, sz = rng.uniform(5.0, 20.0), rng.uniform(5.0, 20.0), rng.uniform(3.0, 12.0)
        cx, cy, cz = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)
        f += a * (np.exp(-0.5 * ((x - cx) / sx) ** 2) * np.exp(-0.5 * ((y - cy) / sy) ** 2)
                  * np.exp(-0.5 * ((z - cz) / sz) ** 2))
    f += noise * rng.uniform(-1.0, 1.0, size=f.shape)
    f[0], f[-1], f[:, 0], f[:, -1], f[:, :, 0], f[:, :, -1] = 0, 0, 0, 0, 0, 0
    return f.astype(np.float32)


def poisson_case(nx: int, ny: int, nz: int, seed: int, iters: int = 50, omega: float = 1.7,
                 dx: float = 4.0, dy: float = 4.0, dz: float = 2.0, boundary: float = 0.0,
                 name: str | None = None) -> PoissonCase:
    """p0 = 0 inside; the boundary layer holds uniform noise of amplitude ``boundary``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = poisson_source(rng, nx, ny, nz)
    p0 = np.zeros((nz, ny, nx), dtype=np.float64)
    if boundary > 0.0:
        b = boundary * rng.uniform(-1.0, 1.0, size=p0.shape)
        inner = (slice(1, -1),) * 3
        b[inner] = 0.0
        p0 = b
    return PoissonCase(name or f"poisson_{nx}x{ny}x{nz}", nx, ny, nz, dx, dy, dz, omega, iters,
                       p0.astype(np.float32), f)


def poisson_300() -> PoissonCase:
    """The large-eddy simulator's pressure grid: 300 x 300 x 90 cells (1.2 km x 1.2 km at
    4 m, 2 m vertical), 50 SOR iterations."""
    return poisson_case(300, 300, 90, seed=60, iters=50, name="poisson_300x300x90")
