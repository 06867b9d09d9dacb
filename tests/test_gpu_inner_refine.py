"""Refinement of the spatial solves inside each FD application
(stfd_opts.inner_refine = k): G is kept in FP64, solved once by the band
factors and k more times on its FP64 residual g_k - (M_x + lambda_k A_x) z_k
(Alg. FD step 3), the solutions summed in FP64 before the FP64 back
transform.  Checked against the oracle's direct solve of K_h (Sec. 3.1) on a
graded time mesh (kappa_2(X_t) large, so the spatial errors are amplified),
both precisions, one and two inner steps (in every application, or a separate
count for the application to the load), in captured rounds and launched one
by one (bitwise the same), and the option checks."""
import numpy as np
import pytest

import workloads as w
from oracle import load
from oracle import solvers as so
from oracle import space_matrices as sm
from oracle import time_matrices as tm

torch = pytest.importorskip("torch")
from paper_2008_01996_amd import stfd  # noqa: E402

pytestmark = pytest.mark.gpu

_CACHE = {}


def _case():
    if not _CACHE:
        mesh, t = w.lshape_mesh(24), w.graded_times(96, 1.0)
        At, Mt, Ct = tm.kernel(t)
        Mx, Ax, M10 = sm.assemble(mesh)
        Fs = [load.assemble_load(M10, load.modes_cell_means(mesh, t, w.random_modes(sd)), Ct) for sd in (9400, 9401)]
        Uo = [so.direct(At, Mt, Mx, Ax, Fq) for Fq in Fs]
        _CACHE.update(mesh=mesh, At=At, Mt=Mt, Mx=Mx, Ax=Ax, Fs=Fs, Uo=Uo)
    return _CACHE


def _solve(c, precision, inner, graph=True, first=-1):
    sp = stfd.Space(c["mesh"])
    prob = stfd.Problem(sp, c["At"], c["Mt"], precision=precision, rtol=1e-11, max_refine=30, inner_refine=inner,
                        graph=graph, inner_refine_first=first)
    prob.factor()
    F = torch.from_numpy(np.ascontiguousarray(np.stack([f.T for f in c["Fs"]]))).to("cuda:0")
    U = torch.empty_like(F)
    rep = prob.solve(F, U)
    torch.cuda.synchronize()
    return rep, U


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("inner,first", [(1, -1), (2, -1), (1, 2), (0, 2)])
def test_inner_refinement_matches_oracle(precision, inner, first):
    """inner steps in every application, or first steps in the application
    to the load and inner in those to a residual"""
    c = _case()
    rep0, _ = _solve(c, precision, 0)
    rep, U = _solve(c, precision, inner, first=first)
    Uh = U.cpu().numpy()
    assert rep["converged"], rep
    for q, Fq in enumerate(c["Fs"]):
        Uq = Uh[q].T
        err = np.linalg.norm(Uq - c["Uo"][q]) / np.linalg.norm(c["Uo"][q])
        res = so.rel_residual(c["At"], c["Mt"], c["Mx"], c["Ax"], Fq, Uq)
        assert err <= 1e-10 and res <= 1e-10, (q, err, res)
    # the spatial solves only get more accurate: never more applications
    assert rep["iterations"] <= rep0["iterations"]
    print(f"  {precision} inner {inner} first {first}: applications {rep['iterations']} (without: {rep0['iterations']}), "
          f"history {rep['rel_residual']}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_inner_refinement_graph_matches_eager(precision):
    c = _case()
    rg, Ug = _solve(c, precision, 1, graph=True)
    re, Ue = _solve(c, precision, 1, graph=False)
    assert rg["iterations"] == re["iterations"]
    assert torch.equal(Ug, Ue)


def test_inner_refinement_options():
    c = _case()
    sp = stfd.Space(c["mesh"])
    # FP32 G and Z would undo the FP64 residual: the FP32 form needs the
    # FP64 forward and back transforms
    for mask in (0, 1, 4):
        with pytest.raises(stfd.StfdError):
            stfd.Problem(sp, c["At"], c["Mt"], precision="fp32", fp64_transforms=mask, inner_refine=1)
    with pytest.raises(stfd.StfdError):
        stfd.Problem(sp, c["At"], c["Mt"], precision="fp64", inner_refine=4)
    for first in (-2, 4):
        with pytest.raises(stfd.StfdError):
            stfd.Problem(sp, c["At"], c["Mt"], precision="fp64", inner_refine_first=first)
    with pytest.raises(stfd.StfdError):
        stfd.Problem(sp, c["At"], c["Mt"], precision="fp32", fp64_transforms=1, inner_refine_first=1)
