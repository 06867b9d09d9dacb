"""Solvers for the space-time system (oracle, FP64).

Global system (Sec. 2; Sec. 4 opening):
    K_h u = F~,   K_h = A_t (x) M_x + M_t (x) A_x,
with u = vec(U), U in R^{M_x x N_t} column-major, U[i, k] the coefficient of
psi_i(x) phi_k(t).  The Kronecker/vec identity of Sec. 3.1,
vec(A X B) = (B^T (x) A) vec(X), gives K_h vec(U) = vec(M_x U A_t^T + A_x U M_t^T).

Functions
  kh_matrix  the sparse K_h, written out with scipy's kron (tiny meshes).
  kh_apply   K_h vec(U) by the Kronecker identity.
  direct     sparse LU solve of the full K_h (textbook routine, tiny meshes).
  fd         Alg. FD (Sec. 4.4): diagonalise the time pencil, change the
             time basis of the load to the eigenvectors, solve one
             independent spatial system per eigenvalue, change back.
  refine     FP64 iterative refinement: R = F~ - K_h u, u += FD(R).
  bartels_stewart
             Alg. BSc (Sec. 4.3): triangularise the time pencil with a
             unitary basis instead, then solve the spatial systems in
             reverse order, each coupled to the ones already solved.

Parity status: ``direct`` is a library routine on the written-out matrix;
``fd``, ``refine`` and ``bartels_stewart`` are pinned against it on small
meshes, ``fd`` and ``refine`` also against the manufactured solution's
convergence rates.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def kh_matrix(At, Mt, Mx, Ax):
    """K_h = A_t (x) M_x + M_t (x) A_x as a sparse matrix."""
    return (sp.kron(sp.csr_matrix(At), Mx) + sp.kron(sp.csr_matrix(Mt), Ax)).tocsc()


def kh_apply(At, Mt, Mx, Ax, U):
    """K_h vec(U) returned as the M_x x N_t matrix M_x U A_t^T + A_x U M_t^T."""
    return Mx @ U @ np.asarray(At).T + Ax @ U @ np.asarray(Mt).T


def residual(At, Mt, Mx, Ax, F, U):
    """R = F~ - K_h u, as an M_x x N_t matrix."""
    return F - kh_apply(At, Mt, Mx, Ax, U)


def rel_residual(At, Mt, Mx, Ax, F, U) -> float:
    """||F~ - K_h u||_2 / ||F~||_2."""
    return float(np.linalg.norm(residual(At, Mt, Mx, Ax, F, U)) / np.linalg.norm(F))


def direct(At, Mt, Mx, Ax, F):
    """Solve the written-out K_h u = vec(F~) with sparse LU; returns U."""
    K = kh_matrix(At, Mt, Mx, Ax)
    u = spl.spsolve(K, np.asarray(F).reshape(-1, order="F"))
    return u.reshape(F.shape, order="F")


def lapack_normalize(X):
    """Scale each eigenvector so that its largest entry has |Re| + |Im| = 1
    (the normalisation of LAPACK's generalised eigensolver)."""
    return X / np.max(np.abs(X.real) + np.abs(X.imag), axis=0)


@dataclasses.dataclass
class Decomposition:
    lam: np.ndarray          # (Nt,) generalised eigenvalues of (M_t, A_t)
    X: np.ndarray            # (Nt, Nt) eigenvectors, M_t X = A_t X diag(lam)
    Ut: np.ndarray           # SVD X = Ut diag(sig) Vt^*
    sig: np.ndarray
    Vt: np.ndarray
    At_cho: tuple            # Cholesky factor of A_t

    @property
    def kappa(self) -> float:
        return float(self.sig.max() / self.sig.min())


def decompose(At, Mt, normalization: str = "lapack") -> Decomposition:
    """Steps 1a and 1b of Algorithm FD.

    1a: M_t z = lambda A_t z (equivalently A_t^-1 M_t = X D X^-1);
    1b: X = U_t Sigma V_t^*.
    ``normalization``: "lapack" (largest entry |Re|+|Im| = 1) or "unit"
    (unit 2-norm columns).
    """
    lam, X = sl.eig(np.asarray(Mt), np.asarray(At))
    if normalization == "lapack":
        X = lapack_normalize(X)
    elif normalization == "unit":
        X = X / np.linalg.norm(X, axis=0)
    else:
        raise ValueError(normalization)
    Ut, sig, Vh = np.linalg.svd(X)
    return Decomposition(lam=lam, X=X, Ut=Ut, sig=sig, Vt=Vh.conj().T,
                         At_cho=sl.cho_factor(np.asarray(At)))


def _spatial_solve(args):
    Mx, Ax, lam, g = args
    lu = spl.splu((Mx + lam * Ax).tocsc().astype(np.complex128))
    return lu.solve(g)


def fd(At, Mt, Mx, Ax, F, dec: Decomposition | None = None, pool_map=map):
    """Alg. FD; returns the real M_x x N_t solution U.

    Why it works: with M_t X = A_t X diag(lambda), write U = Z X^T.  Then
    M_x U A_t^T + A_x U M_t^T = (M_x Z + A_x Z diag(lambda)) (A_t X)^T, so
    K_h u = F~ splits into one spatial system per eigenvalue,
    (M_x + lambda_k A_x) z_k = g_k, for the columns g_k of
    G = F~ (A_t X)^-T = F~ A_t^-1 X^-T.  X^-T is applied through the SVD
    of X (X^-T = conj(U_t) Sigma^-1 V_t^T), as the paper does.

    ``pool_map`` maps the independent spatial solves (the paper's time
    parallelism); the default is the builtin serial ``map``.
    """
    if dec is None:
        dec = decompose(At, Mt)
    F = np.asarray(F, dtype=np.float64)
    # load in the eigenvector basis: F~ A_t^-1 X^-T, the SVD factors
    # applied one after the other (A_t^-1 conj(U_t), then Sigma^-1, then V_t^T)
    G = ((F @ sl.cho_solve(dec.At_cho, dec.Ut.conj())) / dec.sig[None, :]) @ dec.Vt.T
    # one spatial system per eigenvalue
    cols = list(pool_map(_spatial_solve,
                         [(Mx, Ax, dec.lam[k], G[:, k]) for k in range(len(dec.lam))]))
    Z = np.stack(cols, axis=1)
    # back to the hat basis in time: U = Z X^T with X^T through the same
    # factors (real for a real load)
    return (((Z @ dec.Vt.conj()) * dec.sig[None, :]) @ dec.Ut.T).real


def bartels_stewart(At, Mt, Mx, Ax, F):
    """Alg. BSc (Sec. 4.3); returns the real M_x x N_t solution U.

    With the unitary triangularisation A_t^-1 M_t W = W S (S upper
    triangular) and U = Z W^T, K_h u = F~ becomes
    M_x Z + A_x Z S^T = F~ A_t^-1 conj(W) =: G; column k of that reads
    (M_x + S_kk A_x) z_k = g_k - A_x sum_{j>k} S_kj z_j, so the columns are
    solved from the last to the first."""
    At = np.asarray(At)
    F = np.asarray(F, dtype=np.float64)
    S, W = sl.schur(np.linalg.solve(At, np.asarray(Mt)), output="complex")
    G = F @ np.linalg.solve(At, W.conj())
    nt = At.shape[0]
    Z = np.zeros(G.shape, dtype=np.complex128)
    for k in range(nt - 1, -1, -1):
        rhs = G[:, k] - Ax @ (Z[:, k + 1:] @ S[k, k + 1:])
        Z[:, k] = _spatial_solve((Mx, Ax, S[k, k], rhs))
    return (Z @ W.T).real


def refine(At, Mt, Mx, Ax, F, dec: Decomposition | None = None, rtol: float = 0.0,
           max_iter: int = 10, pool_map=map):
    """FD followed by FP64 iterative refinement on the K_h residual.

    Stops when the relative residual is <= rtol, or when it no longer
    decreases (stagnation at rounding level), or after max_iter corrections.
    Returns (U, history of relative residuals).
    """
    if dec is None:
        dec = decompose(At, Mt)
    normF = np.linalg.norm(F)
    U = fd(At, Mt, Mx, Ax, F, dec, pool_map)
    R = residual(At, Mt, Mx, Ax, F, U)
    hist = [float(np.linalg.norm(R) / normF)]
    for _ in range(max_iter):
        if hist[-1] <= rtol:
            break
        U_new = U + fd(At, Mt, Mx, Ax, R, dec, pool_map)
        R_new = residual(At, Mt, Mx, Ax, F, U_new)
        r = float(np.linalg.norm(R_new) / normF)
        if r >= hist[-1]:
            break
        U, R = U_new, R_new
        hist.append(r)
    return U, hist
