"""The L-shape example of Sec. 5 (oracle, FP64; test infrastructure only).

Problem (Sec. 5): the heat equation on Omega = (-1,1)^2 minus [0,1]x[-1,0],
T = 1/2, with the manufactured solution
    u(x, t) = 5/(2 pi t) exp(-|x - c|^2 / (4t)) sin(pi x1 x2),  c = (1/4, -1/4),
which fixes the source f = du/dt - Laplace u and the Dirichlet data g = u on
the lateral boundary; u tends to 0 as t -> 0 on the closure of Omega
because c lies outside it.

Closed forms: G = 5/(2 pi t) exp(-|x-c|^2/(4t)) is ten times the heat
kernel centred at c, so dG/dt = Laplace G and grad G = -G (x - c)/(2t).
With s = sin(pi x1 x2), grad s = pi cos(pi x1 x2) (x2, x1) and
Laplace s = -pi^2 (x1^2 + x2^2) s:
    f = -2 grad G . grad s - G Laplace s
      = G [ pi cos(pi x1 x2) ((x1 - c1) x2 + (x2 - c2) x1) / t
            + pi^2 (x1^2 + x2^2) s ],
    grad u = G [ -(x - c) s / (2t) + grad s ],
    du/dt  = G (-1/t + |x - c|^2 / (4 t^2)) s.

Discretisation (Sec. 2 with the homogenisation that Sec. 5 names): the
Dirichlet extension g_h is the nodal interpolant of g on the boundary
vertices at t_1..t_Nt (g(., 0) = 0), extended by zero to interior vertices;
its coupling is moved to the right-hand side,
    F~ = M10 F C_t^T - (M_B G A_t^T + A_B G M_t^T),
K_h u_0 = F~ is solved, and the error is measured for u_0 + g_h.  The load
F holds the prism means of f (the projection Q_h^0 of Sec. 2) by tensor
Gauss quadrature.  Meshes: the uniform grid triangulations of
``workloads.lshape_mesh`` (level L has cell size 2^-(L+1)) with the time
nodes ``workloads.paper_times(L)``.

Parity status: pinned by tests (f against central differences of u, the
exact reproduction of u = t with its inhomogeneous Dirichlet data, the
convergence rates L2 ~ h^2 and H1 ~ h of the error estimates of Sec. 2, the
dof and mesh-size columns of the Sec. 5 tables).  The error values of those
tables are not pinned: the level-0 triangulation is given only as a figure,
and with either grid diagonal the values differ from the printed ones by
up to 20%; both are reported beside the paper's.
"""
from __future__ import annotations

import math

import numpy as np

from . import load, solvers, space_matrices, time_matrices
from .errors import space_time_errors

C1, C2 = 0.25, -0.25
T_END = 0.5


def _g(x1, x2, t):
    return 5.0 / (2.0 * math.pi * t) * np.exp(-((x1 - C1) ** 2 + (x2 - C2) ** 2) / (4.0 * t))


def u(x1, x2, t):
    """The manufactured solution of Sec. 5."""
    return _g(x1, x2, t) * np.sin(math.pi * x1 * x2)


def grad_u(x1, x2, t):
    G = _g(x1, x2, t)
    s = np.sin(math.pi * x1 * x2)
    c = np.cos(math.pi * x1 * x2)
    return (G * (-(x1 - C1) * s / (2.0 * t) + math.pi * x2 * c),
            G * (-(x2 - C2) * s / (2.0 * t) + math.pi * x1 * c))


def dt_u(x1, x2, t):
    r2 = (x1 - C1) ** 2 + (x2 - C2) ** 2
    return _g(x1, x2, t) * (-1.0 / t + r2 / (4.0 * t * t)) * np.sin(math.pi * x1 * x2)


def f(x1, x2, t):
    """Source du/dt - Laplace u of the manufactured solution."""
    G = _g(x1, x2, t)
    s = np.sin(math.pi * x1 * x2)
    c = np.cos(math.pi * x1 * x2)
    return G * (math.pi * c * ((x1 - C1) * x2 + (x2 - C2) * x1) / t
                + math.pi ** 2 * (x1 * x1 + x2 * x2) * s)


def dirichlet_values(mesh, t, g=u):
    """(nv, N_t) values g(x_v, t_k), k = 1..N_t, at every vertex (the solver
    reads only the Dirichlet ones)."""
    xy = np.asarray(mesh.xy, dtype=np.float64)
    return np.stack([g(xy[:, 0], xy[:, 1], tk) for tk in np.asarray(t)[1:]], axis=1)


def lift(MB, AB, At, Mt, G):
    """Coupling of the Dirichlet extension with nodal values G (nv, N_t):
    M_B G A_t^T + A_B G M_t^T  (M_x x N_t)."""
    return np.asarray(MB @ G) @ np.asarray(At).T + np.asarray(AB @ G) @ np.asarray(Mt).T


def quadrature_orders(level: int):
    """(space points per direction, time points) for the load and the error
    norms; coarse levels need more points for the sharp Gaussian near t = 0."""
    return max(5, 12 - 2 * level), max(5, 16 - 3 * level)


def setup(level: int, diagonal: str = "sw-ne", u_exact=u, f_exact=f, orders=None):
    """Assemble one level of the example: returns a dict with the mesh, t,
    the matrices (At, Mt, Ct, Mx, Ax, M10, MB, AB), the Dirichlet values G
    and the lifted right-hand side Ft."""
    import workloads

    mesh = workloads.lshape_mesh(4 * 2 ** level, diagonal=diagonal)
    t = workloads.paper_times(level)
    ns, nt = orders or quadrature_orders(level)
    At, Mt, Ct = time_matrices.time_matrices(t)
    Mx, Ax, M10 = space_matrices.assemble(mesh)
    MB, AB = space_matrices.boundary_coupling(mesh)
    G = dirichlet_values(mesh, t, u_exact)
    F = load.prism_means(mesh, t, f_exact, ns, nt)
    Ft = load.assemble_load(M10, F, Ct) - lift(MB, AB, At, Mt, G)
    return dict(mesh=mesh, t=t, At=At, Mt=Mt, Ct=Ct, Mx=Mx, Ax=Ax, M10=M10, MB=MB, AB=AB,
                G=G, F=F, Ft=Ft, level=level, diagonal=diagonal)


def errors(case, U, orders=None):
    """(L2(Q), H1(Q)-seminorm) errors of u_0 + g_h for interior values U."""
    ns, nt = orders or quadrature_orders(case["level"])
    return space_time_errors(case["mesh"], case["t"], U, u, grad_u, dt_u,
                             n_space=ns, n_time=nt, boundary=case["G"])


def mesh_sizes(case):
    """(h_x, h_t,max, h_t,min) as the Sec. 5 tables list them; h_x is the
    square root of the largest triangle area."""
    area, _ = space_matrices.triangle_geometry(np.asarray(case["mesh"].xy, dtype=np.float64),
                                               np.asarray(case["mesh"].tri, dtype=np.int64))
    ht = np.diff(case["t"])
    return math.sqrt(float(area.max())), float(ht.max()), float(ht.min())


def run_level(level: int, diagonal: str = "sw-ne"):
    """One row of the Sec. 5 tables: dof, mesh sizes and errors, solved
    with the written-out K_h."""
    case = setup(level, diagonal)
    U = solvers.direct(case["At"], case["Mt"], case["Mx"], case["Ax"], case["Ft"])
    l2, h1 = errors(case, U)
    hx, htmax, htmin = mesh_sizes(case)
    return dict(dof=U.size, hx=hx, ht_max=htmax, ht_min=htmin, l2=l2, h1=h1, U=U, case=case)
