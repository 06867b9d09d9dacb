"""The K_h residual entry point that allocates nothing
(stfd_kh_residual_noalloc, for callers that cannot allocate device memory)
against the allocating one (stfd_kh_residual), through the C-ABI: the same
kernels on the same inputs, so the residual R = F - K_h U and the norms agree
bit for bit.  Two calls in a row on one device, the second with a smaller
input (fewer right-hand sides on a smaller problem), so the second finds the
fixed array holding the first call's data.  A request beyond the array is
refused before any launch."""
import numpy as np
import pytest

import workloads as w
from oracle import solvers as so
from oracle import space_matrices as sm
from oracle import time_matrices as tm

torch = pytest.importorskip("torch")
from paper_2008_01996_amd import stfd  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(nc, nt, nrhs, seed):
    mesh = w.square_mesh(nc)
    t = w.graded_times(nt)
    At, Mt, _ = tm.kernel(t)
    prob = stfd.Problem(stfd.Space(mesh), At, Mt, precision="fp64")
    rng = np.random.default_rng(seed)
    F = torch.from_numpy(rng.standard_normal((nrhs, nt, prob.Mx))).to("cuda:0")
    U = torch.from_numpy(rng.standard_normal((nrhs, nt, prob.Mx))).to("cuda:0")
    return mesh, At, Mt, prob, F, U


def test_noalloc_residual_matches_allocating_entry_point():
    for nc, nt, nrhs, seed in ((32, 24, 3, 9100), (12, 8, 1, 9101)):
        mesh, At, Mt, prob, F, U = _case(nc, nt, nrhs, seed)
        R0 = torch.empty_like(F)
        n0 = prob.kh_residual(F, U, R0)
        R1 = torch.full_like(F, float("nan"))
        n1 = torch.full((2 * nrhs,), float("nan"), dtype=torch.float64, device="cuda:0")
        prob.kh_residual_noalloc(F, U, R1, n1)
        torch.cuda.synchronize()
        assert torch.equal(R0, R1)
        assert np.array_equal(n1.cpu().numpy().reshape(nrhs, 2), n0)
        # and the residual itself is the Kronecker identity of the oracle
        Mx, Ax, _ = sm.assemble(mesh)
        for q in range(nrhs):
            Ro = so.residual(At, Mt, Mx, Ax, F[q].cpu().numpy().T, U[q].cpu().numpy().T)
            assert np.abs(R1[q].cpu().numpy().T - Ro).max() <= 1e-12 * np.abs(Ro).max()
        print(f"  M_x {prob.Mx}, N_t {nt}, {nrhs} RHS: equal to the allocating entry point", flush=True)


def test_noalloc_residual_rejects_oversize():
    cap = stfd.kh_residual_noalloc_max_bytes()
    mesh, At, Mt, prob, F, U = _case(64, 64, 1, 9102)
    nrhs = cap // (prob.Mx * 2 * 64 * 8) + 1          # one right-hand side more than fits
    F = torch.zeros((nrhs, 64, prob.Mx), dtype=torch.float64, device="cuda:0")
    R = torch.empty_like(F)
    with pytest.raises(stfd.StfdError, match="more than its fixed"):
        prob.kh_residual_noalloc(F, F, R)
