"""Seeded, synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds geometry and draws random numbers: time partitions,
triangulations with their interior-node numbering, and the random coefficients
of the smooth right-hand sides.  It holds none of the solver's arithmetic
(no matrices, no quadrature, no transforms), so both the oracle and the GPU
library can take their inputs from here without sharing any computation.

Workloads (Sec. 5 of the paper describes the L-shape experiment; the other
shapes are the unit-square problems the GPU benchmark is quoted on):

* ``square_mesh(nc)``: unit square, ``nc`` cells per side, each cell cut along
  its SW-NE diagonal.  Interior nodes are numbered row by row, x fastest.
* ``lshape_mesh(nc, diagonal)``: (-1,1)^2 minus [0,1]x[-1,0] on the same kind of grid
  with ``nc`` cells per side of the big square (mesh size 2/nc).
* ``uniform_times``, ``graded_times``, ``paper_times``: time partitions.
* ``random_modes``: the eight separable sine/cosine modes of the random
  right-hand sides, drawn from a seeded PCG64 stream.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Mesh:
    """A P1 triangulation.

    xy   : (nv, 2) float64 vertex coordinates
    tri  : (ntri, 3) int32 vertex indices, counter-clockwise
    dof  : (nv,) int32 interior-node number of each vertex, -1 on the
           Dirichlet boundary
    h    : cell size of the underlying grid
    rows : number of interior nodes in each grid row, bottom to top (the
           block sizes of the lexicographic ordering)
    box  : (xmin, xmax, ymin, ymax) bounding box, used to map the random
           right-hand sides onto the unit square
    """

    xy: np.ndarray
    tri: np.ndarray
    dof: np.ndarray
    h: float
    rows: tuple
    box: tuple

    @property
    def n_dof(self) -> int:
        return int((self.dof >= 0).sum())


def _grid_mesh(nc: int, lo: float, hi: float, keep_cell, diagonal: str = "sw-ne") -> Mesh:
    if diagonal not in ("sw-ne", "nw-se"):
        raise ValueError("diagonal must be 'sw-ne' or 'nw-se'")
    h = (hi - lo) / nc
    n1 = nc + 1
    ii, jj = np.meshgrid(np.arange(n1), np.arange(n1), indexing="xy")
    xy_all = np.stack([lo + ii.ravel() * h, lo + jj.ravel() * h], axis=1)

    tris = []
    used = np.zeros(n1 * n1, dtype=bool)
    for j in range(nc):
        for i in range(nc):
            if not keep_cell(i, j):
                continue
            v00 = j * n1 + i
            v10 = v00 + 1
            v01 = v00 + n1
            v11 = v01 + 1
            if diagonal == "sw-ne":
                # lower-right and upper-left triangles
                tris.append((v00, v10, v11))
                tris.append((v00, v11, v01))
            else:
                # NW-SE diagonal: lower-left and upper-right triangles
                tris.append((v00, v10, v01))
                tris.append((v10, v11, v01))
            used[[v00, v10, v01, v11]] = True
    tri_all = np.asarray(tris, dtype=np.int64)

    # boundary = vertices on an edge that belongs to exactly one triangle
    edges = np.concatenate([tri_all[:, [0, 1]], tri_all[:, [1, 2]], tri_all[:, [2, 0]]])
    edges = np.sort(edges, axis=1)
    uniq, counts = np.unique(edges, axis=0, return_counts=True)
    bnd = np.zeros(n1 * n1, dtype=bool)
    bnd[uniq[counts == 1].ravel()] = True

    # compact vertex numbering (drop vertices of removed cells)
    new_id = -np.ones(n1 * n1, dtype=np.int64)
    new_id[used] = np.arange(used.sum())
    xy = xy_all[used]
    tri = new_id[tri_all].astype(np.int32)

    # interior numbering: row by row (y), x fastest; vertices are already in
    # that order because the grid is enumerated with x fastest
    interior = used & ~bnd
    dof_all = -np.ones(n1 * n1, dtype=np.int64)
    dof_all[interior] = np.arange(interior.sum())
    dof = dof_all[used].astype(np.int32)

    rows = []
    for j in range(n1):
        c = int(interior[j * n1:(j + 1) * n1].sum())
        if c:
            rows.append(c)
    return Mesh(xy=xy, tri=tri, dof=dof, h=h, rows=tuple(rows),
                box=(lo, hi, lo, hi))


def square_mesh(nc: int) -> Mesh:
    """Unit square (0,1)^2 with nc x nc cells, h = 1/nc, (nc-1)^2 interior nodes."""
    if nc < 2:
        raise ValueError("need at least 2 cells per side")
    return _grid_mesh(nc, 0.0, 1.0, lambda i, j: True)


def rect_mesh(ncx: int, ncy: int) -> Mesh:
    """Rectangle (0, ncx/ncy) x (0, 1) with ncx x ncy square cells: a wide
    band (ncx interior nodes per row) at a small number of unknowns."""
    if ncx < 2 or ncy < 2:
        raise ValueError("need at least 2 cells per side")
    h = 1.0 / ncy
    m = _grid_mesh(max(ncx, ncy), 0.0, max(ncx, ncy) * h, lambda i, j: i < ncx and j < ncy)
    return Mesh(xy=m.xy, tri=m.tri, dof=m.dof, h=h, rows=m.rows, box=(0.0, ncx * h, 0.0, 1.0))


def lshape_mesh(nc: int, diagonal: str = "sw-ne") -> Mesh:
    """L-shape (-1,1)^2 minus [0,1]x[-1,0]; nc even cells per side, h = 2/nc.

    This is the spatial domain of the paper's numerical example (Sec. 5).
    ``diagonal`` picks the cut of every square cell: "sw-ne" (default) or
    "nw-se".
    """
    if nc < 2 or nc % 2:
        raise ValueError("nc must be even and >= 2")
    half = nc // 2
    return _grid_mesh(nc, -1.0, 1.0, lambda i, j: not (i >= half and j < half), diagonal)


def uniform_times(nt: int, T: float = 1.0) -> np.ndarray:
    """t_i = i T / N_t."""
    return T * np.arange(nt + 1, dtype=np.float64) / nt


def graded_times(nt: int, T: float = 1.0) -> np.ndarray:
    """t_i = T (i/N_t)^2, refined towards t = 0."""
    return T * (np.arange(nt + 1, dtype=np.float64) / nt) ** 2


def paper_times(level: int) -> np.ndarray:
    """The nonuniform partition of (0, 1/2) of Sec. 5, bisected ``level`` times.

    Level 0 has the nodes 0, 1/32, 1/16, 1/8, 1/2 (N_t = 4); every level
    halves every element, so N_t = 4 * 2**level.
    """
    t = np.array([0.0, 1.0 / 32, 1.0 / 16, 1.0 / 8, 0.5])
    for _ in range(level):
        mid = 0.5 * (t[:-1] + t[1:])
        out = np.empty(2 * len(t) - 1)
        out[0::2] = t
        out[1::2] = mid
        t = out
    return t


@dataclasses.dataclass(frozen=True)
class Modes:
    """f(x,t) = sum_q c_q sin(a_q pi xi_1) sin(b_q pi xi_2) cos(d_q pi t / T),
    xi = bounding-box map of x onto [0,1]^2."""

    a: np.ndarray
    b: np.ndarray
    d: np.ndarray
    c: np.ndarray


def random_modes(seed: int, nmodes: int = 8) -> Modes:
    """Smooth random right-hand side: 8 separable modes with N(0,1) weights.

    Draw order per mode q: a_q in [1,4], b_q in [1,4], d_q in [0,3], c_q ~ N(0,1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    a = np.empty(nmodes, dtype=np.int64)
    b = np.empty(nmodes, dtype=np.int64)
    d = np.empty(nmodes, dtype=np.int64)
    c = np.empty(nmodes, dtype=np.float64)
    for q in range(nmodes):
        a[q] = rng.integers(1, 5)
        b[q] = rng.integers(1, 5)
        d[q] = rng.integers(0, 4)
        c[q] = rng.standard_normal()
    return Modes(a=a, b=b, d=d, c=c)


def manufactured_modes() -> Modes:
    """The spatial/temporal pattern of u = sin(pi x1) sin(pi x2) t^2 on the unit
    square (its load is not a finite mode sum in t, so the oracle and the
    library each treat it through ``MANUFACTURED`` below)."""
    return Modes(a=np.array([1]), b=np.array([1]), d=np.array([0]), c=np.array([1.0]))


# Manufactured solution of the unit-square configurations:
#   u = sin(pi x1) sin(pi x2) t^2,  f = du/dt - Laplace u
#     = (2 t + 2 pi^2 t^2) sin(pi x1) sin(pi x2).
MANUFACTURED = "sin(pi x1) sin(pi x2) t^2"


def rhs_seeds(config: str, nrhs: int, problem: int = 0) -> list[int]:
    """Seeds of the random right-hand sides of each configuration."""
    base = {"square256_nt512": 3000, "batch": 4000, "lshape_nt1024": 5000, "lshape_paper": 6000}[config]
    if config == "batch":
        return [base + 8 * problem + r for r in range(nrhs)]
    return [base + r for r in range(nrhs)]


def batch_classes() -> list[tuple[int, int]]:
    """The nine (cells per side, N_t) classes of the batched workload, h-major."""
    return [(nc, nt) for nc in (32, 64, 128) for nt in (32, 128, 512)]


def batch_problem_class(p: int) -> tuple[int, int]:
    """Problem p of the 96-problem batch uses class p mod 9."""
    return batch_classes()[p % 9]
