"""Seeded synthetic scattered-node sets.

This module only produces inputs: node coordinates, boundary masks, per-node
orders and the manufactured Poisson data.  It holds none of the RBF-FD
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

The paper's node sets come from an automated node-positioning algorithm that
is not reproduced here (paper section II).  A jittered lattice stands in for
it: every interior lattice point is moved by an independent uniform offset in
[-0.25 h, 0.25 h] per coordinate, which keeps the minimum spacing at or above
0.5 h, like a Poisson-disk fill.  Interior nodes are listed in lattice
row-major order (y outer, x inner, so neighbours in memory are neighbours in
space), followed by the unjittered boundary nodes.

Random numbers come from numpy's PCG64 generator with the stated seeds.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class NodeSet:
    """A scattered node set: SoA float64 coordinates plus a boundary mask."""

    name: str
    x: np.ndarray
    y: np.ndarray
    is_boundary: np.ndarray  # uint8, 1 on the Dirichlet boundary
    h: float                 # nominal spacing
    order: np.ndarray | None = None  # int8 per-node m in {2,4,6}, or None
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_interior(self) -> int:
        return int(self.n_nodes - int(self.is_boundary.sum()))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _jitter(rng: np.random.Generator, px: np.ndarray, py: np.ndarray, h: float,
            amount: float = 0.25) -> tuple[np.ndarray, np.ndarray]:
    jx = rng.uniform(-amount * h, amount * h, size=px.shape[0])
    jy = rng.uniform(-amount * h, amount * h, size=py.shape[0])
    return px + jx, py + jy


def _pack(name, xi, yi, xb, yb, h, order=None, **meta) -> NodeSet:
    x = np.ascontiguousarray(np.concatenate([xi, xb]), dtype=np.float64)
    y = np.ascontiguousarray(np.concatenate([yi, yb]), dtype=np.float64)
    bnd = np.zeros(x.shape[0], dtype=np.uint8)
    bnd[xi.shape[0]:] = 1
    return NodeSet(name=name, x=x, y=y, is_boundary=bnd, h=h, order=order,
                   meta=dict(meta))


def unit_square(cells: int = 45, seed: int = 1, jitter: float = 0.25) -> NodeSet:
    """[0,1]^2 with spacing h = 1/cells.

    Interior: lattice points (i h, j h), i, j = 1..cells-1, jittered.
    Boundary: 4*cells unjittered nodes walking the edges at spacing h
    (corners appear once).  cells=45 gives 1936 + 180 = 2116 nodes.
    """
    h = 1.0 / cells
    t = np.arange(1, cells, dtype=np.float64) * h
    gx, gy = np.meshgrid(t, t, indexing="xy")
    xi, yi = _jitter(_rng(seed), gx.ravel(), gy.ravel(), h, jitter)
    k = np.arange(cells, dtype=np.float64) * h
    one = np.ones(cells)
    zero = np.zeros(cells)
    xb = np.concatenate([k, one, 1.0 - k, zero])
    yb = np.concatenate([zero, k, one, 1.0 - k])
    return _pack(f"unit_square_h1/{cells}", xi, yi, xb, yb, h, seed=seed)


def unit_disk(n_target: int = 100_000, n_boundary: int = 1000, seed: int = 2,
              jitter: float = 0.25) -> NodeSet:
    """Unit disk: square lattice with h = 1/(sqrt(n_target/pi) + 1), points
    with r <= 1 - h/2 kept and jittered, plus n_boundary unjittered nodes at
    angles 2 pi k / n_boundary on the circle."""
    h = 1.0 / (math.sqrt(n_target / math.pi) + 1.0)
    L = int(math.ceil(1.0 / h)) + 1
    t = np.arange(-L, L + 1, dtype=np.float64) * h
    gx, gy = np.meshgrid(t, t, indexing="xy")
    gx = gx.ravel()
    gy = gy.ravel()
    keep = np.hypot(gx, gy) <= 1.0 - 0.5 * h
    xi, yi = _jitter(_rng(seed), gx[keep], gy[keep], h, jitter)
    th = 2.0 * math.pi * np.arange(n_boundary, dtype=np.float64) / n_boundary
    return _pack(f"unit_disk_{n_target}", xi, yi, np.cos(th), np.sin(th), h,
                 seed=seed)


def cell_centred_square(cells: int = 1000, seed: int = 3, jitter: float = 0.25,
                        order_seed: int | None = None) -> NodeSet:
    """[0,1]^2 cell-centred lattice ((i+1/2) h, (j+1/2) h), h = 1/cells,
    jittered; cells^2 nodes, no boundary nodes.  With order_seed set, each node
    also gets an order m drawn uniformly from {2, 4, 6}."""
    h = 1.0 / cells
    t = (np.arange(cells, dtype=np.float64) + 0.5) * h
    gx, gy = np.meshgrid(t, t, indexing="xy")
    xi, yi = _jitter(_rng(seed), gx.ravel(), gy.ravel(), h, jitter)
    order = None
    if order_seed is not None:
        pick = _rng(order_seed).integers(0, 3, size=xi.shape[0])
        order = (2 * (pick + 1)).astype(np.int8)
    empty = np.zeros(0)
    return _pack(f"square_cc_{cells}x{cells}", xi, yi, empty, empty, h,
                 order=order, seed=seed, order_seed=order_seed)


def annulus(n_target: int = 200_000, r_in: float = 0.3, r_out: float = 1.0,
            seed: int = 5, jitter: float = 0.25) -> NodeSet:
    """Annulus r_in <= r <= r_out: square lattice with h chosen so the area
    holds about n_target nodes, points with r_in + h/2 <= r <= r_out - h/2
    kept and jittered, plus unjittered rings on both circles at spacing ~h."""
    area = math.pi * (r_out ** 2 - r_in ** 2)
    h = math.sqrt(area / n_target)
    L = int(math.ceil(r_out / h)) + 1
    t = np.arange(-L, L + 1, dtype=np.float64) * h
    gx, gy = np.meshgrid(t, t, indexing="xy")
    gx = gx.ravel()
    gy = gy.ravel()
    r = np.hypot(gx, gy)
    keep = (r >= r_in + 0.5 * h) & (r <= r_out - 0.5 * h)
    xi, yi = _jitter(_rng(seed), gx[keep], gy[keep], h, jitter)
    n_o = int(round(2.0 * math.pi * r_out / h))
    n_i = int(round(2.0 * math.pi * r_in / h))
    to = 2.0 * math.pi * np.arange(n_o) / n_o
    ti = 2.0 * math.pi * np.arange(n_i) / n_i
    xb = np.concatenate([r_out * np.cos(to), r_in * np.cos(ti)])
    yb = np.concatenate([r_out * np.sin(to), r_in * np.sin(ti)])
    return _pack(f"annulus_{n_target}", xi, yi, xb, yb, h, seed=seed)


def jittered_cube(cells: int = 100, seed: int = 6, jitter: float = 0.25):
    """Three-dimensional nodes: the cell-centred cells^3 lattice of [0,1]^3
    (spacing h = 1/cells), each coordinate jittered by U(-jitter h, jitter h),
    in lattice order (x fastest).  Returns (x, y, z) float64 arrays."""
    rng = _rng(seed)
    h = 1.0 / cells
    g = (np.arange(cells) + 0.5) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    pts += rng.uniform(-jitter * h, jitter * h, pts.shape)
    return (np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
            np.ascontiguousarray(pts[:, 2]))


def manufactured(x: np.ndarray, y: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Manufactured Poisson data: u = sin(pi x) sin(pi y) and
    f = lap u = -2 pi^2 sin(pi x) sin(pi y)."""
    u = np.sin(np.pi * x) * np.sin(np.pi * y)
    return u, -2.0 * np.pi ** 2 * u


def gaussian_cotangent(n_nodes: int, k: int, seed: int = 55) -> np.ndarray:
    """Seeded N(0,1) cotangent g[n_nodes][k] for the loss L = sum g_ij w_ij."""
    return _rng(seed).standard_normal((n_nodes, k))


# The five workloads, by what they are.
def workload(name: str) -> NodeSet:
    if name == "square_h45_m2":
        return unit_square(45, seed=1)
    if name == "disk_100k_m4":
        return unit_disk(100_000, 1000, seed=2)
    if name == "square_1m_mixed":
        return cell_centred_square(1000, seed=3, order_seed=33)
    if name == "square_1m_m6":
        return cell_centred_square(1000, seed=4)
    if name == "square_10k_m6":
        return cell_centred_square(100, seed=4)
    if name == "annulus_200k_m4":
        return annulus(200_000, seed=5)
    raise KeyError(name)
