"""Right-hand side of the global system (oracle, FP64).

Sec. 2: f is replaced by its L2(Q) projection Q_h^0 f onto functions that
are constant on every prism omega_j x (t_{l-1}, t_l); the coefficient f_{j,l}
is the mean of f over that prism.  The load is then
    F~ = M10 F C_t^T  in R^{M_x x N_t},   F[j, l] = f_{j,l},
with M10 the M_{h_x}^{1,0} matrix and C_t the time matrix of H_T.

Space means use a collapsed (Duffy) tensor Gauss rule on each triangle,
exact for polynomials of total degree 2n-2 (n = points per direction);
time means are exact antiderivatives.

Parity status: pinned by tests (rule exactness on monomials, doubling of
the rule, the exact mean of a linear function; for prism_means, the exact
mean of a polynomial in x and t).
"""
from __future__ import annotations

import math

import numpy as np


def triangle_rule(n: int):
    """Nodes (bary coords l1, l2 with l0 = 1-l1-l2) and weights (sum 1) of the
    collapsed Gauss rule on the reference triangle, n x n points."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    # (u, v) in [0,1]^2 -> (u, u v) in {0 <= y <= x <= 1}, Jacobian u; that
    # triangle has area 1/2, so weights are normalised to sum to one
    l1 = (U * (1 - V)).ravel()      # weight of vertex 1
    l2 = (U * V).ravel()            # weight of vertex 2
    wt = (2 * WU * WV * U).ravel()
    return l1, l2, wt


def _quadrature_points(mesh, n: int):
    """Points (ntri, n*n) x1, x2 and weights (n*n,) of the collapsed rule
    mapped onto every triangle of the mesh."""
    xy = np.asarray(mesh.xy, dtype=np.float64)
    tri = np.asarray(mesh.tri, dtype=np.int64)
    l1, l2, wt = triangle_rule(n)
    p0 = xy[tri[:, 0]][:, None, :]
    p1 = xy[tri[:, 1]][:, None, :]
    p2 = xy[tri[:, 2]][:, None, :]
    P = p0 + l1[None, :, None] * (p1 - p0) + l2[None, :, None] * (p2 - p0)
    return P[..., 0], P[..., 1], wt


def space_means(mesh, fx, n: int = 8, points=None):
    """Mean over every triangle of fx(x1, x2) (vectorised callable).

    Returns (ntri,) array.  ``points``: the result of _quadrature_points for
    this mesh and n, when the caller evaluates several functions."""
    x1, x2, wt = _quadrature_points(mesh, n) if points is None else points
    vals = fx(x1, x2)
    return (vals * wt[None, :]).sum(axis=1)


def modes_cell_means(mesh, t, modes, n: int = 8):
    """F[j, l] = mean of f over omega_j x (t_{l-1}, t_l) for
    f = sum_q c_q sin(a_q pi xi1) sin(b_q pi xi2) cos(d_q pi t / T),
    xi the bounding-box map of x onto [0,1]^2.

    Each mode is separable, so its prism mean is (space mean of the x part)
    times (time mean of the t part); the sum over the modes is written as
    the product Sx diag(c) St^T, Sx[j, q] the space means and St[l, q] the
    time means."""
    t = np.asarray(t, dtype=np.float64)
    T = t[-1]
    h = np.diff(t)
    xmin, xmax, ymin, ymax = mesh.box
    Sx = np.zeros((len(mesh.tri), len(modes.c)))
    St = np.zeros((len(h), len(modes.c)))
    pts = _quadrature_points(mesh, n)
    for q, (a, b, d) in enumerate(zip(modes.a, modes.b, modes.d)):
        def fx(x1, x2, a=a, b=b):
            xi1 = (x1 - xmin) / (xmax - xmin)
            xi2 = (x2 - ymin) / (ymax - ymin)
            return np.sin(a * math.pi * xi1) * np.sin(b * math.pi * xi2)
        Sx[:, q] = space_means(mesh, fx, n, pts)
        if d == 0:
            St[:, q] = 1.0
        else:
            w = d * math.pi / T
            St[:, q] = (np.sin(w * t[1:]) - np.sin(w * t[:-1])) / (w * h)
    return Sx @ (np.asarray(modes.c, dtype=np.float64)[:, None] * St.T)


def manufactured_cell_means(mesh, t, n: int = 8):
    """Cell means of f = (2t + 2 pi^2 t^2) sin(pi x1) sin(pi x2), the load of
    u = sin(pi x1) sin(pi x2) t^2 (du/dt - Laplace u = f)."""
    t = np.asarray(t, dtype=np.float64)
    h = np.diff(t)
    sx = space_means(mesh, lambda x1, x2: np.sin(math.pi * x1) * np.sin(math.pi * x2), n)
    # int (2t + 2 pi^2 t^2) dt = t^2 + 2 pi^2 t^3 / 3
    G = lambda s: s ** 2 + 2 * math.pi ** 2 * s ** 3 / 3
    st = (G(t[1:]) - G(t[:-1])) / h
    return np.outer(sx, st)


def prism_means(mesh, t, f, n_space: int = 10, n_time: int = 12):
    """F[j, l] = mean of f(x1, x2, t) over omega_j x (t_{l-1}, t_l) for a
    general (not separable) f: the collapsed n_space x n_space rule on every
    triangle times n_time-point Gauss-Legendre on every time element."""
    xy = np.asarray(mesh.xy, dtype=np.float64)
    tri = np.asarray(mesh.tri, dtype=np.int64)
    t = np.asarray(t, dtype=np.float64)
    l1, l2, wq = triangle_rule(n_space)
    lam = np.stack([1 - l1 - l2, l1, l2], axis=1)              # (q, 3)
    P = np.einsum("qa,jad->jqd", lam, xy[tri])                 # (ntri, q, 2)
    tg, wg = np.polynomial.legendre.leggauss(n_time)
    tg = 0.5 * (tg + 1)
    wg = 0.5 * wg
    F = np.zeros((len(tri), len(t) - 1))
    for l in range(len(t) - 1):
        h = t[l + 1] - t[l]
        for tau, w in zip(tg, wg):
            F[:, l] += w * (f(P[..., 0], P[..., 1], t[l] + tau * h) * wq[None, :]).sum(axis=1)
    return F


def assemble_load(M10, F, Ct):
    """F~ = M10 F C_t^T  (M_x x N_t)."""
    return np.asarray(M10 @ F) @ np.asarray(Ct).T
