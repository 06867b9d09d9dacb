"""Refinement rounds as captured HIP graphs (stfd_opts.graph = 1, the
default): every replay is bit-identical to the same solve launched kernel by
kernel (graph = 0), and matches the oracle.  The graph of a problem is built
on its first solve with given buffers and replayed afterwards; rounds after
convergence are gated off on the device.  Each replay here is separated from
the next by eager work of the program and a synchronisation, and every
replay is checked, so a graph node that went wrong on a later replay would
show.  Batches run every member's round on forked streams inside one graph."""
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


def _case(mesh, t, seeds):
    At, Mt, Ct = tm.kernel(t)
    Mx, Ax, M10 = sm.assemble(mesh)
    Fs = [load.assemble_load(M10, load.modes_cell_means(mesh, t, w.random_modes(sd)), Ct) for sd in seeds]
    F = torch.from_numpy(np.ascontiguousarray(np.stack([f.T for f in Fs]))).to("cuda:0")
    return At, Mt, Mx, Ax, Fs, F


def _eager_work(F):
    # unrelated device work and a synchronisation between replays
    x = (F * 2.0).sum()
    torch.cuda.synchronize()
    return x


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_eager_and_oracle(precision):
    mesh, t = w.square_mesh(16), w.uniform_times(16)
    At, Mt, Mx, Ax, Fs, F = _case(mesh, t, [9200, 9201, 9202])
    sp = stfd.Space(mesh)
    eager = stfd.Problem(sp, At, Mt, precision=precision, rtol=1e-11, graph=False)
    eager.factor()
    Ue = torch.empty_like(F)
    re = eager.solve(F, Ue)
    graph = stfd.Problem(sp, At, Mt, precision=precision, rtol=1e-11, graph=True)
    graph.factor()
    Ug = torch.empty_like(F)
    for replay in range(4):
        Ug.fill_(float("nan"))
        rg = graph.solve(F, Ug)
        torch.cuda.synchronize()
        assert torch.equal(Ug, Ue), replay
        assert rg["iterations"] == re["iterations"]
        assert rg["rel_residual"][:rg["iterations"]] == re["rel_residual"][:re["iterations"]]
        _eager_work(F)
    for q, Fq in enumerate(Fs):
        Uo = so.direct(At, Mt, Mx, Ax, Fq)
        Uq = Ug[q].cpu().numpy().T
        assert np.linalg.norm(Uq - Uo) / np.linalg.norm(Uo) <= 1e-10
        assert so.rel_residual(At, Mt, Mx, Ax, Fq, Uq) <= 1e-10
    print(f"  {re['iterations']} applications, 4 replays bit-identical to the eager solve", flush=True)


def test_graph_is_rebuilt_for_new_buffers_and_refactor():
    mesh, t = w.square_mesh(12), w.graded_times(10)
    At, Mt, _, _, _, F1 = _case(mesh, t, [9210, 9211])
    _, _, _, _, _, F2 = _case(mesh, t, [9212, 9213])
    sp = stfd.Space(mesh)
    eager = stfd.Problem(sp, At, Mt, precision="fp32", graph=False)
    graph = stfd.Problem(sp, At, Mt, precision="fp32", graph=True)
    for p in (eager, graph):
        p.factor()
    for F in (F1, F2, F1):
        Ue, Ug = torch.empty_like(F), torch.empty_like(F)
        eager.solve(F, Ue)
        graph.solve(F, Ug)
        torch.cuda.synchronize()
        assert torch.equal(Ue, Ug)
        graph.factor()                       # a refactor between solves keeps the graph valid
        _eager_work(F)


def test_graph_reports_nonconvergence():
    mesh, t = w.square_mesh(8), w.uniform_times(64)
    At, Mt, _, _, _, F = _case(mesh, t, [9220])
    for graph in (False, True):
        prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp32", rtol=1e-16, max_refine=2, graph=graph)
        prob.factor()
        rep = prob.solve(F, torch.empty_like(F), check=False)
        assert rep["status"] == stfd.ENOCONV and rep["iterations"] == 3 and not rep["converged"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_graph_matches_eager_batch(precision):
    cases = [(w.square_mesh(8), w.uniform_times(8), [9230, 9231]),
             (w.square_mesh(12), w.graded_times(12), [9232]),
             (w.lshape_mesh(8), w.paper_times(1), [9233, 9234, 9235]),
             (w.rect_mesh(40, 3), w.uniform_times(6), [9236])]
    built = {}
    for graph in (False, True):
        probs, Fd, Ud = [], [], []
        for mesh, t, seeds in cases:
            At, Mt, Mx, Ax, Fs, F = _case(mesh, t, seeds)
            probs.append(stfd.Problem(stfd.Space(mesh), At, Mt, precision=precision, rtol=1e-11, graph=graph))
            Fd.append(F)
            Ud.append(torch.empty_like(F))
        batch = stfd.Batch(probs)
        batch.factor()
        for replay in range(3 if graph else 1):
            rc, reps = batch.solve(Fd, Ud)
            torch.cuda.synchronize()
            assert rc == 0
            if graph:
                for i in range(len(cases)):
                    assert torch.equal(Ud[i], built[False][0][i]), (replay, i)
                    assert reps[i]["iterations"] == built[False][1][i]["iterations"]
                _eager_work(Fd[0])
        built[graph] = ([u.clone() for u in Ud], reps)
    for i, (mesh, t, seeds) in enumerate(cases):
        At, Mt, Mx, Ax, Fs, _ = _case(mesh, t, seeds)
        for q, Fq in enumerate(Fs):
            Uq = built[True][0][i][q].cpu().numpy().T
            Uo = so.direct(At, Mt, Mx, Ax, Fq)
            assert np.linalg.norm(Uq - Uo) / np.linalg.norm(Uo) <= 1e-10


def test_preallocated_problem_solves_like_the_lazy_one():
    """nrhs_max allocates factor and work memory at setup; solves up to that
    many right-hand sides (and beyond, growing) give the same result."""
    mesh, t = w.square_mesh(10), w.uniform_times(12)
    At, Mt, _, _, _, F = _case(mesh, t, [9240, 9241, 9242, 9243, 9244, 9245])
    sp = stfd.Space(mesh)
    lazy = stfd.Problem(sp, At, Mt, precision="fp32")
    pre = stfd.Problem(sp, At, Mt, precision="fp32", nrhs_max=4)
    for p in (lazy, pre):
        p.factor()
    for n in (2, 4, 6):
        Fn = F[:n].contiguous()
        U1, U2 = torch.empty_like(Fn), torch.empty_like(Fn)
        lazy.solve(Fn, U1)
        pre.solve(Fn, U2)
        torch.cuda.synchronize()
        assert torch.equal(U1, U2), n
