"""Pins of the oracle's solvers: Algorithm FD and FP64 refinement against the
written-out Kronecker system, the N_t = 1 special case, and the
manufactured solution's convergence rates (Sec. 2 error estimates)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spl

import workloads as w
from oracle import errors as er
from oracle import load
from oracle import solvers as so
from oracle import space_matrices as sm
from oracle import time_matrices as tm


def _problem(nc, t, rhs="manufactured", seed=3000):
    mesh = w.square_mesh(nc)
    At, Mt, Ct = tm.kernel(t)
    Mx, Ax, M10 = sm.assemble(mesh)
    if rhs == "manufactured":
        F = load.manufactured_cell_means(mesh, t)
    else:
        F = load.modes_cell_means(mesh, t, w.random_modes(seed))
    return mesh, At, Mt, Mx, Ax, load.assemble_load(M10, F, Ct)


def test_kronecker_identity():
    """K_h vec(U) = vec(M_x U A_t^T + A_x U M_t^T) (Sec. 3.1)."""
    _, At, Mt, Mx, Ax, _ = _problem(5, w.paper_times(1))
    U = np.random.default_rng(0).standard_normal((Mx.shape[0], At.shape[0]))
    K = so.kh_matrix(At, Mt, Mx, Ax)
    lhs = (K @ U.reshape(-1, order="F")).reshape(U.shape, order="F")
    assert np.abs(lhs - so.kh_apply(At, Mt, Mx, Ax, U)).max() < 1e-14 * np.abs(lhs).max()


@pytest.mark.parametrize("nc,t", [(16, w.uniform_times(16)), (8, w.paper_times(1)),
                                  (6, w.graded_times(8))], ids=["C1", "paper1", "graded8"])
def test_fd_matches_full_system(nc, t):
    """Algorithm FD + one FP64 refinement step equals the sparse LU solution
    of the written-out K_h to 1e-12; plain FD is reported and must be
    within 1e-10 on these small meshes."""
    _, At, Mt, Mx, Ax, F = _problem(nc, t)
    Ud = so.direct(At, Mt, Mx, Ax, F)
    U0 = so.fd(At, Mt, Mx, Ax, F)
    U, hist = so.refine(At, Mt, Mx, Ax, F, max_iter=3)
    nd = np.linalg.norm(Ud)
    assert np.linalg.norm(U0 - Ud) / nd < 1e-10
    assert np.linalg.norm(U - Ud) / nd < 1e-12
    assert hist[-1] < 1e-13


@pytest.mark.parametrize("nc,t", [(16, w.uniform_times(16)), (8, w.paper_times(1)),
                                  (6, w.graded_times(7))], ids=["C1", "paper1", "graded7"])
def test_bartels_stewart_matches_full_system(nc, t):
    """Algorithm BSc (unitary transforms, no refinement) equals the sparse LU
    solution of the written-out K_h to 1e-12: with W unitary the transforms
    amplify nothing, so plain BSc is accurate to rounding."""
    _, At, Mt, Mx, Ax, F = _problem(nc, t)
    Ud = so.direct(At, Mt, Mx, Ax, F)
    Ub = so.bartels_stewart(At, Mt, Mx, Ax, F)
    assert np.linalg.norm(Ub - Ud) / np.linalg.norm(Ud) < 1e-12
    assert so.rel_residual(At, Mt, Mx, Ax, F, Ub) < 1e-13


def test_single_time_element_is_one_spatial_solve():
    """N_t = 1: FD reduces to (A_t M_x + M_t A_x) u = F~ with lambda = M_t/A_t."""
    t = np.array([0.0, 0.6])
    _, At, Mt, Mx, Ax, F = _problem(6, t)
    dec = so.decompose(At, Mt)
    assert abs(dec.lam[0] - Mt[0, 0] / At[0, 0]) < 1e-15
    u = spl.spsolve((At[0, 0] * Mx + Mt[0, 0] * Ax).tocsc(), F[:, 0])
    assert np.abs(so.fd(At, Mt, Mx, Ax, F)[:, 0] - u).max() < 1e-13 * np.abs(u).max()


def test_conjugate_modes_give_conjugate_solves():
    """For real F~, g and z of conjugate eigenvalues are complex conjugates
    (Sec. 4.1: eigenvalues come in conjugate pairs)."""
    _, At, Mt, Mx, Ax, F = _problem(6, w.uniform_times(8), rhs="random")
    dec = so.decompose(At, Mt)
    W = np.linalg.solve(At, dec.Ut.conj())
    G = ((F @ W) / dec.sig) @ dec.Vt.T
    lam = dec.lam
    for k in range(len(lam)):
        j = int(np.argmin(np.abs(lam - lam[k].conj())))
        assert np.abs(G[:, j] - G[:, k].conj()).max() < 1e-12 * np.abs(G).max()


def test_manufactured_solution_convergence_rates():
    """u = sin(pi x1) sin(pi x2) t^2 under h_x = h_t halving: L2(Q) error
    rate -> 2 and H1(Q) rate -> 1 (Sec. 2 error estimates, p = 1)."""
    S = lambda x, y: np.sin(math.pi * x) * np.sin(math.pi * y)
    u = lambda x, y, tt: S(x, y) * tt ** 2
    gu = lambda x, y, tt: (math.pi * np.cos(math.pi * x) * np.sin(math.pi * y) * tt ** 2,
                           math.pi * np.sin(math.pi * x) * np.cos(math.pi * y) * tt ** 2)
    du = lambda x, y, tt: 2 * tt * S(x, y)
    errs = []
    for nc in (4, 8, 16, 32):
        t = w.uniform_times(nc)
        mesh, At, Mt, Mx, Ax, F = _problem(nc, t)
        U, _ = so.refine(At, Mt, Mx, Ax, F, max_iter=3)
        errs.append(er.space_time_errors(mesh, t, U, u, gu, du))
    errs = np.array(errs)
    eoc = np.log2(errs[:-1] / errs[1:])
    assert 1.95 < eoc[-1, 0] < 2.05, eoc
    assert 0.97 < eoc[-1, 1] < 1.03, eoc
    # the paper's error pattern: both errors decrease monotonically
    assert np.all(np.diff(errs[:, 0]) < 0) and np.all(np.diff(errs[:, 1]) < 0)


def test_refinement_reaches_rounding_on_conditioned_mesh():
    """Uniform N_t = 64: plain FD is visibly perturbed by kappa_2(X_t), FP64
    refinement brings the relative residual to rounding level."""
    _, At, Mt, Mx, Ax, F = _problem(8, w.uniform_times(64), rhs="random")
    U, hist = so.refine(At, Mt, Mx, Ax, F, max_iter=5)
    assert hist[-1] < 1e-13
    Ud = so.direct(At, Mt, Mx, Ax, F)
    assert np.linalg.norm(U - Ud) / np.linalg.norm(Ud) < 1e-12
