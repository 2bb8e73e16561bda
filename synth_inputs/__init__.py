"""Seeded synthetic inputs for the mEVP momentum subcycle.

This module only draws and lays out inputs: mesh vertices, ice height H and
concentration A as DG coefficients, and wind / ocean velocities at the CG2
nodes. It holds none of the method's arithmetic (no basis functions, no
quadrature, no stress or velocity update), so both the FP64 CPU oracle and the
HIP path can consume the same arrays without sharing any method code.

The paper evaluates on a moving-cyclone benchmark whose definition (forcing,
initial ice) is not part of the paper text (Sec. 4); the recipe below is a
synthetic stand-in with the same structure: a structured quad mesh on a
512 km square (the resolution study of Sec. 4 / Fig. 3), H ~ U[0.5, 2] m,
A ~ U[0.8, 1] per element, a rotating wind gyre of 10 m/s peak and a weak
0.1 m/s ocean current.

Layouts (all float64, C order):
  vertices  [2][(ny+1)*(nx+1)]   vertex (ix, iy) at index iy*(nx+1)+ix, metres
  nodes     [2][(2nx+1)*(2ny+1)] CG2 node positions of a curved mesh, or None
  H, A      [n_a][nx*ny]         element e = ey*nx+ex, DG coefficients
  wind      [2][(2nx+1)*(2ny+1)] CG2 node (ix, iy) at index iy*(2nx+1)+ix, m/s
  ocean     [2][(2nx+1)*(2ny+1)] same
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "DomainInputs",
    "uniform_vertices",
    "perturbed_vertices",
    "curved_nodes",
    "ice_fields",
    "wind_field",
    "ocean_field",
    "make_domain",
    "batched_sizes",
    "WORKLOAD_SEEDS",
    "named_workload",
    "random_state",
]

#: seeds of the named workloads; the batched one derives per-domain seeds from 466
WORKLOAD_SEEDS = {"32x32-dg1": 1001, "256x256-dg2": 1002, "1024x1024-dg2": 1003,
                  "2048x2048-dg2": 1005, "batch64-dg2": 466,
                  "1024x1024-ns8": 1008, "1024x1024-dg2-bilinear": 1009,
                  "2048x2048-dg2-bilinear": 1010, "256x256-dg2-iso": 1011,
                  "1024x1024-dg2-iso": 1012}

#: wind gyre peak speed [m/s], angular rotation rate [1/s], ocean peak [m/s]
WIND_PEAK = 10.0
WIND_OMEGA = 2.0 * math.pi / 86400.0
OCEAN_PEAK = 0.1


@dataclass
class DomainInputs:
    nx: int
    ny: int
    n_s: int
    n_a: int
    vertices: np.ndarray
    H: np.ndarray
    A: np.ndarray
    wind: np.ndarray
    ocean: np.ndarray
    meta: dict = field(default_factory=dict)
    nodes: np.ndarray | None = None  # CG2 node positions of a curved (isoparametric) mesh

    @property
    def n_elements(self) -> int:
        return self.nx * self.ny

    @property
    def n_nodes(self) -> int:
        return (2 * self.nx + 1) * (2 * self.ny + 1)


def uniform_vertices(nx: int, ny: int, hx: float, hy: float | None = None) -> np.ndarray:
    """Vertices of an nx x ny grid of hx x hy rectangles with origin (0, 0)."""
    hy = hx if hy is None else hy
    ix = np.arange(nx + 1, dtype=np.float64)
    iy = np.arange(ny + 1, dtype=np.float64)
    X, Y = np.meshgrid(ix * hx, iy * hy)  # [ny+1][nx+1]
    return np.stack([X.ravel(), Y.ravel()]).astype(np.float64)


def perturbed_vertices(nx: int, ny: int, hx: float, hy: float | None = None,
                       amp: float = 0.1, seed: int = 0) -> np.ndarray:
    """Uniform grid with interior vertices moved by at most ``amp`` cell widths.

    A smooth sinusoidal displacement plus a small seeded jitter; boundary
    vertices stay on the box so the domain remains a rectangle. Elements become
    general (non-parallelogram) quadrilaterals, which exercises a varying
    Jacobian inside each element.
    """
    hy = hx if hy is None else hy
    V = uniform_vertices(nx, ny, hx, hy).reshape(2, ny + 1, nx + 1)
    rng = np.random.default_rng(seed)
    iy, ix = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    s = np.sin(math.pi * ix / nx) * np.sin(math.pi * iy / ny)
    jx = rng.uniform(-1.0, 1.0, size=s.shape)
    jy = rng.uniform(-1.0, 1.0, size=s.shape)
    interior = (ix > 0) & (ix < nx) & (iy > 0) & (iy < ny)
    dx = amp * hx * (0.6 * s * np.sin(2.0 * math.pi * iy / ny) + 0.4 * jx) * interior
    dy = amp * hy * (0.6 * s * np.cos(2.0 * math.pi * ix / nx) + 0.4 * jy) * interior
    V[0] += dx
    V[1] += dy
    return V.reshape(2, -1).copy()


def curved_nodes(nx: int, ny: int, hx: float, hy: float | None = None,
                 amp: float = 0.1, seed: int = 0) -> np.ndarray:
    """CG2 node positions [2][(2nx+1)(2ny+1)] of a curved mesh: the uniform
    grid's nodes (cell corners, edge midpoints, centres) moved by a smooth
    displacement of at most ``amp`` cell widths that also bends the outer
    boundary, plus a seeded jitter of the interior nodes (0.3 of the smooth
    amplitude). Cell edges become quadratic curves, so the cells are neither
    parallelograms nor bilinear images of the square."""
    hy = hx if hy is None else hy
    NX, NY = 2 * nx + 1, 2 * ny + 1
    iy, ix = np.meshgrid(np.arange(NY), np.arange(NX), indexing="ij")
    xh, yh = ix / (NX - 1), iy / (NY - 1)
    rng = np.random.default_rng(seed)
    jx = rng.uniform(-1.0, 1.0, size=xh.shape)
    jy = rng.uniform(-1.0, 1.0, size=xh.shape)
    interior = (ix > 0) & (ix < NX - 1) & (iy > 0) & (iy < NY - 1)
    dx = amp * hx * (0.7 * np.sin(2.0 * math.pi * yh) * np.sin(math.pi * xh + 0.3)
                     + 0.3 * jx * interior)
    dy = amp * hy * (0.7 * np.sin(2.0 * math.pi * xh) * np.sin(math.pi * yh + 0.3)
                     + 0.3 * jy * interior)
    X = ix * (0.5 * hx) + dx
    Y = iy * (0.5 * hy) + dy
    return np.stack([X.ravel(), Y.ravel()]).astype(np.float64)


def ice_fields(n_elements: int, n_a: int, seed: int, ho_amp: float = 0.0):
    """H ~ U[0.5, 2] m and A ~ U[0.8, 1] as DG coefficient 0 (draw order: H, then A).

    With ``ho_amp`` > 0 the higher DG coefficients are drawn too (U[-ho_amp,
    ho_amp] scaled by the mean), so that pointwise values leave [0, inf) and
    [0, 1] and the clamps of the stress update become active. The named
    workloads use ho_amp = 0.
    """
    rng = np.random.default_rng(seed)
    H = np.zeros((n_a, n_elements), dtype=np.float64)
    A = np.zeros((n_a, n_elements), dtype=np.float64)
    H[0] = rng.uniform(0.5, 2.0, n_elements)
    A[0] = rng.uniform(0.8, 1.0, n_elements)
    if ho_amp > 0.0 and n_a > 1:
        H[1:] = rng.uniform(-ho_amp, ho_amp, (n_a - 1, n_elements)) * 1.25
        A[1:] = rng.uniform(-ho_amp, ho_amp, (n_a - 1, n_elements)) * 0.9
    return H, A


def _node_logical(nx: int, ny: int):
    """Logical coordinates (xh, yh) in [0,1]^2 of the CG2 nodes, node-index order."""
    ix = np.arange(2 * nx + 1, dtype=np.float64) / (2 * nx)
    iy = np.arange(2 * ny + 1, dtype=np.float64) / (2 * ny)
    XH, YH = np.meshgrid(ix, iy)
    return XH.ravel(), YH.ravel()


def wind_field(nx: int, ny: int, t: float = 0.0, phase: float = 0.0) -> np.ndarray:
    """Rotating gyre, 10 m/s peak: R(w t + phase) (sin(pi x) cos(pi y), -cos(pi x) sin(pi y))."""
    xh, yh = _node_logical(nx, ny)
    ux = WIND_PEAK * np.sin(math.pi * xh) * np.cos(math.pi * yh)
    uy = -WIND_PEAK * np.cos(math.pi * xh) * np.sin(math.pi * yh)
    th = WIND_OMEGA * t + phase
    c, s = math.cos(th), math.sin(th)
    return np.stack([c * ux - s * uy, s * ux + c * uy]).astype(np.float64)


def ocean_field(nx: int, ny: int) -> np.ndarray:
    """Weak cross-domain current, 0.1 m/s at the corners: (0.1/sqrt2)(2y-1, 1-2x)."""
    xh, yh = _node_logical(nx, ny)
    s = OCEAN_PEAK / math.sqrt(2.0)
    return np.stack([s * (2.0 * yh - 1.0), s * (1.0 - 2.0 * xh)]).astype(np.float64)


def make_domain(nx: int, ny: int, n_s: int, n_a: int = 1, seed: int = 0, *,
                length: float | None = None, h: float | None = None,
                perturb: float = 0.0, ho_amp: float = 0.0,
                wind_phase: float = 0.0, curved: float = 0.0) -> DomainInputs:
    """One seeded domain. Give either the cell size ``h`` or the domain ``length``
    (of the x side; cells are square). Default: 512 km domain. ``perturb``
    moves the vertices (bilinear cells); ``curved`` instead gives CG2 node
    positions of a curved mesh (``nodes``; the vertices are its corner nodes)."""
    if h is None:
        length = 512e3 if length is None else length
        h = length / nx
    nodes = None
    if curved > 0.0:
        nodes = curved_nodes(nx, ny, h, h, amp=curved, seed=seed + 7919)
        NX = 2 * nx + 1
        corner = (np.arange(ny + 1)[:, None] * 2 * NX + np.arange(nx + 1)[None, :] * 2).ravel()
        V = nodes[:, corner].copy()
    elif perturb > 0.0:
        V = perturbed_vertices(nx, ny, h, h, amp=perturb, seed=seed + 7919)
    else:
        V = uniform_vertices(nx, ny, h, h)
    H, A = ice_fields(nx * ny, n_a, seed, ho_amp=ho_amp)
    return DomainInputs(nx, ny, n_s, n_a, V, H, A,
                        wind_field(nx, ny, phase=wind_phase), ocean_field(nx, ny),
                        meta={"seed": seed, "h": h, "perturb": perturb, "curved": curved,
                              "ho_amp": ho_amp, "wind_phase": wind_phase},
                        nodes=nodes)


def batched_sizes(seed: int = 466, n_domains: int = 64, lo: int = 64, hi: int = 512):
    """Side lengths N_d of the batched workload and a wind phase per domain.

    N_d = integers(lo, hi+1) per domain, with the first forced to ``lo`` and
    the last to ``hi`` so the smallest and largest sizes are always present.
    Domain d then draws its own fields with seed 1000*seed + d.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, n_domains)
    sizes[0] = lo
    sizes[-1] = hi
    phases = 2.0 * math.pi * rng.uniform(0.0, 1.0, n_domains)
    return [int(s) for s in sizes], [float(p) for p in phases]


def named_workload(name: str) -> list[DomainInputs]:
    """A named workload as a list of domains (one entry unless batched):
      32x32-dg1       32 x 32 cells of 10 km, 3 stress dofs (2x2 Gauss)
      256x256-dg2     256 x 256 cells on a 512 km square (2 km), 6 stress dofs
      1024x1024-dg2   1024 x 1024 cells on 512 km (0.5 km)
      2048x2048-dg2   2048 x 2048 cells on 512 km (0.25 km)
      batch64-dg2     64 square domains of 512 km, sides 64..512 cells (seeded)
      1024x1024-ns8   1024 x 1024 on 512 km, 8 stress dofs (the Q2-gradient space)
      *-bilinear      the same meshes with interior vertices moved by <= 0.15 h,
                      so every cell is a general quadrilateral
      *-iso           the same meshes with curved cells: CG2 node positions
                      moved by <= 0.15 h (isoparametric map)
    """
    seed = WORKLOAD_SEEDS[name]
    if name == "32x32-dg1":
        return [make_domain(32, 32, 3, 1, seed, h=10e3)]
    if name == "batch64-dg2":
        sizes, phases = batched_sizes(seed)
        return [make_domain(n, n, 6, 1, 1000 * seed + d, wind_phase=phases[d])
                for d, n in enumerate(sizes)]
    n = int(name.split("x")[0])
    if name.endswith("-ns8"):
        return [make_domain(n, n, 8, 1, seed)]
    if name.endswith("-bilinear"):
        return [make_domain(n, n, 6, 1, seed, perturb=0.15)]
    if name.endswith("-iso"):
        return [make_domain(n, n, 6, 1, seed, curved=0.15)]
    return [make_domain(n, n, 6, 1, seed)]


def random_state(nx: int, ny: int, n_s: int, seed: int, v_scale: float = 0.01,
                 s_scale: float = 5000.0):
    """A seeded mid-iteration state (v, S) for tests that start from a state
    other than rest: a smooth velocity gyre of ``v_scale`` m/s plus 1% noise,
    zero on the outer boundary, and DG stress coefficients of magnitude
    ``s_scale`` N/m (higher-order coefficients smaller)."""
    rng = np.random.default_rng(seed)
    xh, yh = _node_logical(nx, ny)
    bump = np.sin(math.pi * xh) * np.sin(math.pi * yh)
    vx = v_scale * (bump * np.cos(3.0 * yh) + 0.01 * rng.standard_normal(xh.shape))
    vy = v_scale * (-bump * np.sin(2.0 * xh) + 0.01 * rng.standard_normal(xh.shape))
    NX, NY = 2 * nx + 1, 2 * ny + 1
    ix, iy = np.arange(NX * NY) % NX, np.arange(NX * NY) // NX
    edge = (ix == 0) | (iy == 0) | (ix == NX - 1) | (iy == NY - 1)
    vx[edge] = 0.0
    vy[edge] = 0.0
    decay = np.array([1.0, 0.3, 0.3, 0.1, 0.1, 0.1, 0.03, 0.03])[:n_s]
    S = s_scale * rng.standard_normal((3, n_s, nx * ny)) * decay[None, :, None]
    S[0, 0] -= s_scale
    S[2, 0] -= s_scale
    return np.stack([vx, vy]).astype(np.float64), S
