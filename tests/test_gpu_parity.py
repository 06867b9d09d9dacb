"""GPU parity of the FD solve (through the C-ABI) against the FP64 oracle.

Inputs come from the shared seeded generators; the oracle builds its own
matrices and load from them and solves in FP64 (sparse LU of K_h on tiny
meshes, Algorithm FD + refinement otherwise).  The GPU receives the same
matrices (parity of the solver) or assembles everything itself (end to end).
Tolerance: relative l2 error <= 1e-10 and relative residual <= 1e-10 for both
precisions (the FP32 form is refined in FP64 to the same target).  The error
is the residual times a problem-dependent amplification of order one to ten,
so these solves refine to a residual of 1e-11 to make the 1e-10 agreement
hold; the benchmark solves to the metric's 1e-10 and reports its error.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import workloads as w
from oracle import load
from oracle import solvers as so
from oracle import space_matrices as sm
from oracle import time_matrices as tm

torch = pytest.importorskip("torch")
from paper_2008_01996_amd import stfd  # noqa: E402

pytestmark = pytest.mark.gpu

RTOL = 1e-10
SOLVE_RTOL = 1e-11


def _oracle_case(mesh, t, rhs, seeds=(3000,)):
    At, Mt, Ct = tm.kernel(t)
    Mx, Ax, M10 = sm.assemble(mesh)
    Fs = []
    for sd in seeds:
        if rhs == "manufactured":
            F = load.manufactured_cell_means(mesh, t)
        else:
            F = load.modes_cell_means(mesh, t, w.random_modes(sd))
        Fs.append(load.assemble_load(M10, F, Ct))
    return At, Mt, Mx, Ax, Fs


def _oracle_solution(At, Mt, Mx, Ax, F):
    if Mx.shape[0] * At.shape[0] <= 40000:
        return so.direct(At, Mt, Mx, Ax, F)
    U, _ = so.refine(At, Mt, Mx, Ax, F, max_iter=6)
    return U


def _to_dev(Fs):
    arr = np.stack([F.T for F in Fs])            # (nrhs, Nt, Mx) = [rhs][k][i]
    return torch.from_numpy(np.ascontiguousarray(arr)).to("cuda:0")


def _gpu_solve(space, At, Mt, Fs, precision, fp64_transforms=5, max_refine=30, rtol=SOLVE_RTOL):
    prob = stfd.Problem(space, At, Mt, precision=precision, fp64_transforms=fp64_transforms, max_refine=max_refine,
                        rtol=rtol)
    prob.factor()
    F = _to_dev(Fs)
    U = torch.empty_like(F)
    rep = prob.solve(F, U)
    torch.cuda.synchronize()
    Us = [u.T.copy() for u in U.cpu().numpy()]
    return Us, rep, prob


def _check(At, Mt, Mx, Ax, Fs, Us, rep, tol=RTOL):
    assert rep["converged"], rep
    for F, U in zip(Fs, Us):
        Uo = _oracle_solution(At, Mt, Mx, Ax, F)
        err = np.linalg.norm(U - Uo) / np.linalg.norm(Uo)
        res = so.rel_residual(At, Mt, Mx, Ax, F, U)
        print(f"  rel err vs oracle {err:.2e}  rel residual (oracle K_h) {res:.2e}  iters {rep['iterations']}")
        assert res <= tol
        assert err <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_unit_square_manufactured(precision):
    """h = 1/16, uniform N_t = 16 (3600 space-time DOFs), manufactured load."""
    mesh = w.square_mesh(16)
    t = w.uniform_times(16)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "manufactured")
    Us, rep, _ = _gpu_solve(stfd.Space(mesh), At, Mt, Fs, precision)
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nc,t,nrhs", [
    (9, w.graded_times(7), 3),          # M_x = 64, b = 9 (padded to 16), odd N_t -> a real eigenvalue
    (12, w.paper_times(2), 1),          # M_x = 121 (ragged last panel), nonuniform paper mesh
    (6, w.uniform_times(10, T=0.5), 17),  # two right-hand-side groups, the second ragged
], ids=["graded7_rhs3", "paper2_rhs1", "uniform10_rhs17"])
def test_ragged_shapes(precision, nc, t, nrhs):
    mesh = w.square_mesh(nc)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[4000 + r for r in range(nrhs)])
    Us, rep, prob = _gpu_solve(stfd.Space(mesh), At, Mt, Fs, precision)
    if len(t) - 1 == 7:
        assert prob.setup_report["n_real"] >= 1
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("ncx,ncy,nrhs", [(101, 4, 2), (128, 3, 1), (120, 6, 9), (131, 3, 1), (250, 3, 17)],
                         ids=["band101", "band128", "band120_rhs9", "band131", "band250_rhs17"])
def test_wide_bands(precision, ncx, ncy, nrhs):
    """Thin rectangles: half-bandwidth ncx (padded to 112, 128, 128, 144,
    256), which exercises every band-kernel configuration at small M_x
    (padded 128 in FP32 is the register-resident factorization)."""
    mesh = w.rect_mesh(ncx, ncy)
    t = w.uniform_times(12)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[6000 + r for r in range(nrhs)])
    sp = stfd.Space(mesh)
    assert sp.half_band == ncx
    Us, rep, _ = _gpu_solve(sp, At, Mt, Fs, precision)
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


# Right-hand-side counts that take every sweep variant (one, on a narrow band
# and on padded half-bandwidth 128, where it has a variant of its own; five
# and six, where the far-band work switches to reading L once for all
# right-hand sides; eight, a full group; nine, a full group and a group of
# one) on meshes of padded half-bandwidth 16, 128 and 256.
SWEEP_CASES = [(9, 9, 1), (9, 9, 6), (120, 3, 1), (120, 3, 5), (120, 3, 9), (250, 3, 8)]
SWEEP_IDS = ["sq9_rhs1", "sq9_rhs6", "band120_rhs1", "band120_rhs5", "band120_rhs9", "band250_rhs8"]
UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("ncx,ncy,nrhs", SWEEP_CASES, ids=SWEEP_IDS)
def test_spatial_step_matches_oracle_solves(precision, ncx, ncy, nrhs):
    """Step 3 alone (band LDL^T and both sweeps) against the oracle's sparse
    complex solves of (M_x + lambda_k A_x) z = g, per system and right-hand
    side.  The systems' eigenvalues must match the oracle's; the oracle solves
    with its own.  Bound: banded LU without pivoting has backward error of
    order (b + 1) u |L||U| (Higham, Thm. 9.3), and for these complex
    symmetric systems with positive definite real and imaginary parts |L||U|
    stays of the size of |S|, so the relative forward error is within
    4 (b + 1) u kappa_2(S_k)."""
    mesh = w.rect_mesh(ncx, ncy)
    t = w.graded_times(7)                       # odd N_t: three pairs and one real eigenvalue
    At, Mt, Ct = tm.kernel(t)
    Mx, Ax, _ = sm.assemble(mesh)
    dec = so.decompose(At, Mt)
    prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision=precision)
    prob.factor()
    lam = prob.system_lambdas()
    n, m = len(lam), Mx.shape[0]
    assert prob.setup_report["n_real"] == 1
    rng = np.random.default_rng(8000 + nrhs)
    G = rng.standard_normal((nrhs, 2 * n, m))
    dt = torch.float64 if precision == "fp64" else torch.float32
    Gd = torch.from_numpy(G).to("cuda:0", dt)
    Z = torch.empty_like(Gd)
    prob.spatial_solve(Gd, Z)
    torch.cuda.synchronize()
    Z = Z.double().cpu().numpy()
    b = prob.setup_report["half_band"]
    u = UNIT_ROUNDOFF[precision]
    for k in range(n):
        j = int(np.argmin(np.abs(dec.lam - lam[k])))
        assert abs(dec.lam[j] - lam[k]) <= 1e-10 * abs(dec.lam[j])
        S = (Mx + dec.lam[j] * Ax).toarray()
        tol = 4 * (b + 1) * u * np.linalg.cond(S)
        for q in range(nrhs):
            g = G[q, k] + 1j * G[q, n + k]
            zo = so._spatial_solve((Mx, Ax, dec.lam[j], g))
            z = Z[q, k] + 1j * Z[q, n + k]
            err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
            assert err <= tol, (k, q, err, tol)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("ncx,ncy,nrhs", SWEEP_CASES, ids=SWEEP_IDS)
def test_single_application_matches_oracle_fd(precision, ncx, ncy, nrhs):
    """One application of Algorithm FD, no refinement (the refinement would
    hide a wrong step: it only needs a contraction), against the oracle's
    Algorithm FD.  Each side's error is within N_t u kappa_2(X_t) (transform
    products of length N_t, amplified by the eigenvector matrix's condition
    number), u the unit roundoff of the stages in the working precision, so
    the two agree within twice that."""
    mesh = w.rect_mesh(ncx, ncy)
    t = w.uniform_times(12)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[7000 + r for r in range(nrhs)])
    prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision=precision)
    prob.factor()
    X = _to_dev(Fs)
    U = torch.empty_like(X)
    prob.apply(X, U)
    torch.cuda.synchronize()
    Us = [u.T.copy() for u in U.cpu().numpy()]
    dec = so.decompose(At, Mt)
    tol = 2 * (len(t) - 1) * UNIT_ROUNDOFF[precision] * np.linalg.cond(dec.X)
    worst = 0.0
    for Fq, Uq in zip(Fs, Us):
        Uo = so.fd(At, Mt, Mx, Ax, Fq, dec)
        worst = max(worst, np.linalg.norm(Uq - Uo) / np.linalg.norm(Uo))
    print(f"  one application: worst rel diff vs oracle FD {worst:.2e} (bound {tol:.2e})")
    assert worst <= tol


# Algorithm BSc (Bartels-Stewart with the complex Schur form, Sec. 4.3): the
# N_t systems solved one after the other through the same band kernels.
BSC_CASES = [("square12", w.square_mesh(12), w.uniform_times(16), 1),
             ("graded7", w.square_mesh(9), w.graded_times(7), 2),
             ("band120", w.rect_mesh(120, 3), w.uniform_times(10), 3),
             ("lshape16", w.lshape_mesh(16), w.paper_times(2), 1)]


@pytest.mark.parametrize("name,mesh,t,nrhs", BSC_CASES, ids=[c[0] for c in BSC_CASES])
def test_bartels_stewart_solve_matches_oracle(name, mesh, t, nrhs):
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[9000 + r for r in range(nrhs)])
    prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp64", method="bsc", rtol=SOLVE_RTOL)
    assert prob.setup_report["n_sys"] == len(t) - 1 and prob.setup_report["kappa2"] == 1.0
    prob.factor()
    F = _to_dev(Fs)
    U = torch.empty_like(F)
    rep = prob.solve(F, U)
    torch.cuda.synchronize()
    Us = [u.T.copy() for u in U.cpu().numpy()]
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


@pytest.mark.parametrize("name,mesh,t,nrhs", BSC_CASES[:3], ids=[c[0] for c in BSC_CASES[:3]])
def test_bartels_stewart_single_application_matches_oracle(name, mesh, t, nrhs):
    """One application of Algorithm BSc against the oracle's.  W is unitary,
    so the transforms add only ~N_t u; each spatial solve adds up to
    (b + 1) u kappa_2(M_x + lambda_k A_x) (banded LU without pivoting), and
    the substitution over S passes those on: both sides are within
    N_t (b + 1) u max_k kappa_2(M_x + lambda_k A_x) of the exact solution."""
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[9100 + r for r in range(nrhs)])
    sp_ = stfd.Space(mesh)
    prob = stfd.Problem(sp_, At, Mt, precision="fp64", method="bsc")
    prob.factor()
    X = _to_dev(Fs)
    U = torch.empty_like(X)
    prob.apply(X, U)
    torch.cuda.synchronize()
    Us = [u.T.copy() for u in U.cpu().numpy()]
    lam = sl.eigvals(Mt, At)
    kmax = max(np.linalg.cond((Mx + l * Ax).toarray()) for l in lam)
    tol = 2 * (len(t) - 1) * (sp_.half_band + 1) * np.finfo(float).eps * kmax
    worst = 0.0
    for Fq, Uq in zip(Fs, Us):
        Uo = so.bartels_stewart(At, Mt, Mx, Ax, Fq)
        worst = max(worst, np.linalg.norm(Uq - Uo) / np.linalg.norm(Uo))
    print(f"  one BSc application: worst rel diff vs oracle {worst:.2e} (bound {tol:.2e})")
    assert worst <= tol


def test_bartels_stewart_requires_fp64():
    mesh = w.square_mesh(4)
    At, Mt, _, _, _ = _oracle_case(mesh, w.uniform_times(4), "random")
    with pytest.raises(stfd.StfdError) as e:
        stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp32", method="bsc")
    assert e.value.code == stfd.EINVAL


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lshape_variable_rows(precision):
    """L-shape (rows of 7 and 15 interior nodes), paper time mesh level 2."""
    mesh = w.lshape_mesh(16)
    t = w.paper_times(2)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[5000, 5001])
    Us, rep, _ = _gpu_solve(stfd.Space(mesh), At, Mt, Fs, precision)
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_of_uneven_problems(precision):
    """Three problems of different spatial and time sizes and right-hand-side
    counts solved as one batch: each matches the oracle, and each is identical
    to solving it alone (the batch only interleaves the same launches)."""
    cases = [(w.square_mesh(8), w.uniform_times(8), [4000, 4001]),
             (w.square_mesh(12), w.graded_times(12), [4008]),
             (w.lshape_mesh(8), w.paper_times(1), [4016, 4017, 4018])]
    probs, Fd, Ud, oracle = [], [], [], []
    for mesh, t, seeds in cases:
        At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=seeds)
        p = stfd.Problem(stfd.Space(mesh), At, Mt, precision=precision, max_refine=30, rtol=SOLVE_RTOL)
        probs.append(p)
        Fd.append(_to_dev(Fs))
        Ud.append(torch.empty_like(Fd[-1]))
        oracle.append((At, Mt, Mx, Ax, Fs))
    batch = stfd.Batch(probs)
    batch.factor()
    rc, reps = batch.solve(Fd, Ud)
    torch.cuda.synchronize()
    assert rc == 0
    for i, (At, Mt, Mx, Ax, Fs) in enumerate(oracle):
        Us = [u.T.copy() for u in Ud[i].cpu().numpy()]
        _check(At, Mt, Mx, Ax, Fs, Us, reps[i])
        # alone
        U1 = torch.empty_like(Fd[i])
        rep1 = probs[i].solve(Fd[i], U1)
        torch.cuda.synchronize()
        assert rep1["iterations"] == reps[i]["iterations"]
        assert torch.equal(U1, Ud[i])


def test_batch_rejects_bad_input():
    mesh = w.square_mesh(6)
    t = w.uniform_times(4)
    At, Mt, Ct = tm.kernel(t)
    p = stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp64")
    with pytest.raises(stfd.StfdError):
        stfd.Batch([p, p])
    b = stfd.Batch([p])
    F = torch.zeros((1, 4, p.Mx), dtype=torch.float64, device="cuda:0")
    U = torch.empty_like(F)
    rc, _ = b.solve([F], [U], check=False)
    assert rc == stfd.ESTATE


def test_end_to_end_library_assembly():
    """The library assembles time matrices, spatial matrices and the load
    itself; the result matches the all-oracle solution."""
    mesh = w.square_mesh(16)
    t = w.uniform_times(16)
    sp = stfd.Space(mesh)
    A, M, C = stfd.assemble_time(t)
    Fl = sp.assemble_load(C, sp.project_f(t, w.manufactured_modes(), kind=1))
    Us, rep, _ = _gpu_solve(sp, A, M, [Fl], "fp32")
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "manufactured")
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


def test_device_residual_is_kronecker_identity():
    """R = F - K_h U on the device equals F - (M_x U A_t^T + A_x U M_t^T)."""
    mesh = w.square_mesh(10)
    t = w.paper_times(2)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[7, 8])
    prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp64")
    rng = np.random.default_rng(1)
    Uh = [rng.standard_normal(F.shape) for F in Fs]
    F = _to_dev(Fs)
    U = _to_dev(Uh)
    R = torch.empty_like(F)
    norms = prob.kh_residual(F, U, R)
    Rh = [r.T for r in R.cpu().numpy()]
    for q in range(2):
        Ro = so.residual(At, Mt, Mx, Ax, Fs[q], Uh[q])
        assert np.abs(Rh[q] - Ro).max() <= 1e-13 * np.abs(Ro).max()
        assert abs(norms[q, 0] - (Ro ** 2).sum()) <= 1e-12 * (Ro ** 2).sum()
        assert abs(norms[q, 1] - (Fs[q] ** 2).sum()) <= 1e-12 * (Fs[q] ** 2).sum()


def test_fp32_forward_variant_still_converges():
    """With the first forward GEMM in FP32 the refinement still reaches 1e-10
    (more iterations: that GEMM amplifies FP32 rounding by kappa_2(X_t))."""
    mesh = w.square_mesh(12)
    t = w.uniform_times(32)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random")
    Us, rep, _ = _gpu_solve(stfd.Space(mesh), At, Mt, Fs, "fp32", fp64_transforms=0, max_refine=40)
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


@pytest.mark.parametrize("mask", [1, 2, 3, 6, 7])
def test_fp64_transform_variants(mask):
    """The FP32 form with other transform GEMMs on FP64 matrix cores: with
    bit 0 the forward transform is one FP64 GEMM with W1 W2, without it the
    two GEMMs (the first in FP32)."""
    mesh = w.square_mesh(12)
    t = w.graded_times(24)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[11, 12])
    Us, rep, _ = _gpu_solve(stfd.Space(mesh), At, Mt, Fs, "fp32", fp64_transforms=mask)
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_large_space_with_ragged_tiles(precision):
    """M_x = 33124: a ragged last GEMM tile (33124 = 517 * 64 + 36), a padded
    half-bandwidth of 192 (183 nodes per row), two right-hand sides."""
    mesh = w.square_mesh(183)
    t = w.uniform_times(6)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[7300, 7301])
    assert Mx.shape[0] == 33124
    Us, rep, _ = _gpu_solve(stfd.Space(mesh), At, Mt, Fs, precision)
    _check(At, Mt, Mx, Ax, Fs, Us, rep)


def test_solve_is_deterministic():
    mesh = w.square_mesh(16)
    t = w.uniform_times(16)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random", seeds=[1, 2])
    prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp32")
    prob.factor()
    F = _to_dev(Fs)
    U1 = torch.empty_like(F)
    U2 = torch.empty_like(F)
    prob.solve(F, U1)
    prob.factor()
    prob.solve(F, U2)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)


def test_nonconvergence_is_reported():
    """max_refine = 0 with an unreachable target returns ENOCONV (host-forced)."""
    mesh = w.square_mesh(8)
    t = w.uniform_times(64)
    At, Mt, Mx, Ax, Fs = _oracle_case(mesh, t, "random")
    prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp32", rtol=1e-16, max_refine=0)
    prob.factor()
    F = _to_dev(Fs)
    U = torch.empty_like(F)
    rep = prob.solve(F, U, check=False)
    assert rep["status"] == stfd.ENOCONV and rep["iterations"] == 1


def test_solve_before_factor():
    mesh = w.square_mesh(4)
    At, Mt, _, _, Fs = _oracle_case(mesh, w.uniform_times(4), "random")
    prob = stfd.Problem(stfd.Space(mesh), At, Mt)
    F = _to_dev(Fs)
    with pytest.raises(stfd.StfdError) as e:
        prob.solve(F, torch.empty_like(F))
    assert e.value.code == stfd.ESTATE
