"""Space-time errors of a discrete solution (oracle, FP64).

u_h(x, t) = sum_{i,k} U[i,k] psi_i(x) phi_k(t) (Sec. 2, tensor-product P1).
On each prism omega_j x (t_{l-1}, t_l), u_h is linear in x and linear in t;
its space gradient is the P1 gradient of the nodal values at that time and
its time derivative is the difference quotient of the two time slices.

    ||u - u_h||_{L2(Q)}^2 = sum over prisms of int (u - u_h)^2
    |u - u_h|_{H1(Q)}^2   = sum over prisms of int |grad_x (u-u_h)|^2 + (d_t (u-u_h))^2

Quadrature: the collapsed Gauss rule on triangles times Gauss-Legendre in t.
Parity status: pinned by tests (zero error for a u in the discrete space,
the closed-form norm of a polynomial).
"""
from __future__ import annotations

import numpy as np

from .load import triangle_rule
from .space_matrices import triangle_geometry


def space_time_errors(mesh, t, U, u, grad_u, dt_u, n_space: int = 5, n_time: int = 4,
                      boundary=None):
    """Return (L2(Q) error, H1(Q) seminorm error).

    u, dt_u: callables (x1, x2, t) -> value; grad_u: -> (g1, g2).
    U: (M_x, N_t) coefficients; node values at t_0 = 0 are zero.
    boundary: None (zero Dirichlet data) or (nv, N_t) values at t_1..t_Nt of
    the Dirichlet extension; only its rows for Dirichlet vertices are used.
    """
    xy = np.asarray(mesh.xy, dtype=np.float64)
    tri = np.asarray(mesh.tri, dtype=np.int64)
    dof = np.asarray(mesh.dof, dtype=np.int64)
    t = np.asarray(t, dtype=np.float64)
    nt = len(t) - 1
    area, g = triangle_geometry(xy, tri)
    l1, l2, wq = triangle_rule(n_space)
    lam = np.stack([1 - l1 - l2, l1, l2], axis=1)              # (q, 3)
    P = np.einsum("qa,jad->jqd", lam, xy[tri])                 # (ntri, q, 2)
    tg, wg = np.polynomial.legendre.leggauss(n_time)
    tg = 0.5 * (tg + 1)
    wg = 0.5 * wg

    # nodal values per triangle vertex at every time node (zero at t = 0;
    # on the boundary zero or the given Dirichlet extension)
    Vfull = np.zeros((len(xy), nt + 1))
    inner = dof >= 0
    Vfull[inner, 1:] = U[dof[inner], :]
    if boundary is not None:
        Vfull[~inner, 1:] = np.asarray(boundary, dtype=np.float64)[~inner, :]
    err_l2 = 0.0
    err_h1 = 0.0
    for l in range(nt):
        h = t[l + 1] - t[l]
        v0 = Vfull[tri, l]            # (ntri, 3)
        v1 = Vfull[tri, l + 1]
        for tau, w in zip(tg, wg):
            tt = t[l] + tau * h
            vt = (1 - tau) * v0 + tau * v1
            uh = vt @ lam.T                                          # (ntri, q)
            guh = np.einsum("ja,jad->jd", vt, g)                     # (ntri, 2)
            dtuh = ((v1 - v0) / h) @ lam.T                           # (ntri, q)
            ue = u(P[..., 0], P[..., 1], tt)
            g1, g2 = grad_u(P[..., 0], P[..., 1], tt)
            due = dt_u(P[..., 0], P[..., 1], tt)
            wgt = (area[:, None] * wq[None, :]) * (w * h)
            err_l2 += float((wgt * (ue - uh) ** 2).sum())
            err_h1 += float((wgt * ((g1 - guh[:, None, 0]) ** 2 + (g2 - guh[:, None, 1]) ** 2
                                    + (due - dtuh) ** 2)).sum())
    return np.sqrt(err_l2), np.sqrt(err_h1)
