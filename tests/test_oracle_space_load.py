"""Pins of the oracle's spatial matrices, load assembly and error norms."""
import math

import numpy as np
import pytest

import workloads as w
from oracle import errors as er
from oracle import load
from oracle import space_matrices as sm
from oracle import time_matrices as tm


@pytest.mark.parametrize("nc", [4, 7, 16])
def test_stiffness_spectrum_is_five_point_laplacian(nc):
    """On the SW-NE triangulation the P1 stiffness matrix is the 5-point
    Laplacian, whose eigenvalues are 4 - 2cos(p pi h) - 2cos(q pi h)."""
    mesh = w.square_mesh(nc)
    _, Ax, _ = sm.assemble(mesh)
    h = 1.0 / nc
    p = np.arange(1, nc)
    want = np.sort((4 - 2 * np.cos(p[:, None] * math.pi * h) - 2 * np.cos(p[None, :] * math.pi * h)).ravel())
    got = np.sort(np.linalg.eigvalsh(Ax.toarray()))
    assert np.abs(got - want).max() < 1e-12


def test_mass_stencil_and_row_sums():
    """Interior mass rows: h^2/2 on the diagonal, h^2/12 for the E, W, N, S,
    NE and SW neighbours, zero for NW and SE; row sum = int psi_i = h^2."""
    nc = 8
    h = 1.0 / nc
    mesh = w.square_mesh(nc)
    Mx, Ax, M10 = sm.assemble(mesh)
    n = nc - 1
    M = Mx.toarray()
    i = 3 * n + 3                # an interior node with interior neighbours
    assert abs(M[i, i] - h * h / 2) < 1e-15
    for d in (1, -1, n, -n, n + 1, -(n + 1)):
        assert abs(M[i, i + d] - h * h / 12) < 1e-15
    for d in (n - 1, -(n - 1)):
        assert M[i, i + d] == 0.0
    assert abs(M[i].sum() - h * h) < 1e-15
    assert np.abs(M - M.T).max() == 0.0
    # M10 rows: int psi_i = h^2 for every interior node
    assert np.allclose(np.asarray(M10.sum(axis=1)).ravel(), h * h, rtol=0, atol=1e-15)


def test_mass_matrix_brute_force():
    """M_x[i,j] = int psi_i psi_j by Monte Carlo-free midpoint refinement:
    evaluate the hats on a fine uniform point lattice of each triangle."""
    mesh = w.square_mesh(3)
    Mx, _, _ = sm.assemble(mesh)
    xy = mesh.xy
    tri = mesh.tri
    n = mesh.n_dof
    B = np.zeros((n, n))
    k = 60   # sub-triangle lattice: midpoint rule on k^2 sub-triangles
    for e in range(len(tri)):
        p = xy[tri[e]]
        area = 0.5 * abs((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[1, 1] - p[0, 1]) * (p[2, 0] - p[0, 0]))
        pts = []
        for a in range(k):
            for b in range(k - a):
                pts.append(((a + 1 / 3) / k, (b + 1 / 3) / k))
                if a + b < k - 1:
                    pts.append(((a + 2 / 3) / k, (b + 2 / 3) / k))
        pts = np.array(pts)
        lam = np.stack([1 - pts.sum(1), pts[:, 0], pts[:, 1]], 1)
        wgt = area / (k * k)
        for a in range(3):
            ia = mesh.dof[tri[e, a]]
            if ia < 0:
                continue
            for b in range(3):
                ib = mesh.dof[tri[e, b]]
                if ib < 0:
                    continue
                B[ia, ib] += wgt * (lam[:, a] * lam[:, b]).sum()
    assert np.abs(B - Mx.toarray()).max() < 1e-4 * np.abs(B).max()


def test_lshape_dof_counts():
    """The paper's L-shape levels: dof = M_x N_t = 20, 264, 2576 for levels
    0-2 (Sec. 5 tables), and M_x = 48641 at h = 1/128."""
    for level, dof in ((0, 20), (1, 264), (2, 2576)):
        mesh = w.lshape_mesh(4 * 2 ** level)
        nt = len(w.paper_times(level)) - 1
        assert mesh.n_dof * nt == dof
    assert w.lshape_mesh(256).n_dof == 48641


@pytest.mark.parametrize("n", [2, 4, 8])
def test_triangle_rule_exact_on_monomials(n):
    """Mean of x^a y^b over the triangle (0,0),(1,0),(0,1) is
    2 a! b! / (a+b+2)!, exact for a + b <= 2n - 2."""
    l1, l2, wt = load.triangle_rule(n)
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            exact = 2 * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs((wt * l1 ** a * l2 ** b).sum() - exact) < 1e-14


def test_cell_means_converged_and_linear():
    mesh = w.square_mesh(8)
    t = w.uniform_times(4)
    modes = w.random_modes(3000)
    F8 = load.modes_cell_means(mesh, t, modes, n=8)
    F16 = load.modes_cell_means(mesh, t, modes, n=16)
    assert np.abs(F8 - F16).max() < 1e-13
    # linear function: mean = value at the centroid
    c = mesh.xy[mesh.tri].mean(axis=1)
    got = load.space_means(mesh, lambda x, y: 2 * x - 3 * y + 1, n=2)
    assert np.allclose(got, 2 * c[:, 0] - 3 * c[:, 1] + 1, atol=1e-14)


def test_load_of_constant_f():
    """f = 1: F~[i,k] = int psi_i * int H_T phi_k ... = rowsum(M10)_i * rowsum(C_t)_k."""
    mesh = w.square_mesh(6)
    t = w.paper_times(1)
    _, _, M10 = sm.assemble(mesh)
    _, _, Ct = tm.kernel(t)
    F = np.ones((len(mesh.tri), len(t) - 1))
    Ft = load.assemble_load(M10, F, Ct)
    want = np.outer(np.asarray(M10.sum(axis=1)).ravel(), Ct.sum(axis=1))
    assert np.abs(Ft - want).max() < 1e-15


def test_error_norms_of_zero_solution():
    """With U = 0 the errors are the norms of u = sin(pi x) sin(pi y) t^2 on
    (0,1)^2 x (0,1): ||u||^2 = 1/20,  |u|_H1^2 = pi^2/10 + 1/3."""
    mesh = w.square_mesh(16)
    t = w.uniform_times(4)
    S = lambda x, y: np.sin(math.pi * x) * np.sin(math.pi * y)
    u = lambda x, y, tt: S(x, y) * tt ** 2
    gu = lambda x, y, tt: (math.pi * np.cos(math.pi * x) * np.sin(math.pi * y) * tt ** 2,
                           math.pi * np.sin(math.pi * x) * np.cos(math.pi * y) * tt ** 2)
    du = lambda x, y, tt: 2 * tt * S(x, y)
    l2, h1 = er.space_time_errors(mesh, t, np.zeros((mesh.n_dof, 4)), u, gu, du, n_space=8, n_time=4)
    assert abs(l2 - math.sqrt(1 / 20)) < 1e-10
    assert abs(h1 - math.sqrt(math.pi ** 2 / 10 + 1 / 3)) < 1e-10
