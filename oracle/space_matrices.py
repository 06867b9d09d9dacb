"""P1 spatial matrices (oracle, FP64).

Definitions (Sec. 2):
    M_x[i, j]    = < psi_j , psi_i >_{L2(Omega)}            (mass)
    A_x[i, j]    = < grad psi_j , grad psi_i >_{L2(Omega)}  (stiffness)
    M10[i, j]    = < psi^0_j , psi_i >_{L2(Omega)}          (M_{h_x}^{1,0})
for the interior P1 hats psi_i and the triangle indicators psi^0_j.

Element by element: on a triangle T with area |T| and barycentric
gradients grad lambda_a,
    mass      |T|/12 (1 + delta_ab),
    stiffness |T| grad lambda_a . grad lambda_b,
    M10       int_T lambda_a = |T|/3.
Written as plain loops over triangles; slow but obviously the definition.

Parity status: pinned by tests (closed-form spectra of the 5-point
Laplacian, row sums of the mass matrix, symmetry, a brute-force quadrature
of the hat products on a small mesh).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


def triangle_geometry(xy, tri):
    """Areas (ntri,) and barycentric gradients (ntri, 3, 2)."""
    p0 = xy[tri[:, 0]]
    p1 = xy[tri[:, 1]]
    p2 = xy[tri[:, 2]]
    d1 = p1 - p0
    d2 = p2 - p0
    det = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    area = 0.5 * det
    if np.any(area <= 0):
        raise ValueError("triangles must be counter-clockwise and non-degenerate")
    # grad lambda_a = rot90(opposite edge) / (2|T|)
    e0 = p2 - p1      # opposite vertex 0
    e1 = p0 - p2      # opposite vertex 1
    e2 = p1 - p0      # opposite vertex 2
    g = np.empty((len(tri), 3, 2))
    for a, e in enumerate((e0, e1, e2)):
        g[:, a, 0] = -e[:, 1] / det
        g[:, a, 1] = e[:, 0] / det
    return area, g


def assemble(mesh):
    """Return (Mx, Ax, M10) as scipy CSR matrices.

    Mx, Ax: (M_x, M_x);  M10: (M_x, N_x) with N_x = number of triangles.
    """
    xy = np.asarray(mesh.xy, dtype=np.float64)
    tri = np.asarray(mesh.tri, dtype=np.int64)
    dof = np.asarray(mesh.dof, dtype=np.int64)
    n = int((dof >= 0).sum())
    area, g = triangle_geometry(xy, tri)
    rows, cols, mv, av = [], [], [], []
    r10, c10, v10 = [], [], []
    for e in range(len(tri)):
        for a in range(3):
            i = dof[tri[e, a]]
            if i < 0:
                continue
            r10.append(i)
            c10.append(e)
            v10.append(area[e] / 3.0)
            for b in range(3):
                j = dof[tri[e, b]]
                if j < 0:
                    continue
                rows.append(i)
                cols.append(j)
                mv.append(area[e] / 12.0 * (2.0 if a == b else 1.0))
                av.append(area[e] * float(g[e, a] @ g[e, b]))
    Mx = sp.csr_matrix((mv, (rows, cols)), shape=(n, n))
    Ax = sp.csr_matrix((av, (rows, cols)), shape=(n, n))
    M10 = sp.csr_matrix((v10, (r10, c10)), shape=(n, len(tri)))
    Mx.sum_duplicates()
    Ax.sum_duplicates()
    M10.sum_duplicates()
    return Mx, Ax, M10


def boundary_coupling(mesh):
    """(MB, AB): the entries M_x[i, v], A_x[i, v] of interior rows i against
    Dirichlet vertices v, as (M_x, nv) CSR matrices indexed by vertex number
    (columns of interior vertices are zero).  Same element matrices as
    ``assemble``, with every vertex taken as a node."""
    dof = np.asarray(mesh.dof, dtype=np.int64)
    nv = len(dof)
    every = dataclasses.replace(mesh, dof=np.arange(nv, dtype=np.int32))
    Mf, Af, _ = assemble(every)
    inner = np.where(dof >= 0)[0]
    rows = inner[np.argsort(dof[inner])]                        # vertex of row i
    keep = sp.diags((dof < 0).astype(np.float64))
    return (Mf[rows] @ keep).tocsr(), (Af[rows] @ keep).tocsr()
