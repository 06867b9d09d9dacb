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
  fd         Algorithm FD of Sec. 4.4, as stated: (1a) eigendecomposition of
             the pencil (M_t, A_t), (1b) SVD X = U_t Sigma V_t^*, (2) forward
             transform G = F^ A_t^-1 conj(U_t) Sigma^-1 V_t^T, (3) the N_t
             independent spatial solves (M_x + lambda_k A_x) z_k = g_k, (4) the
             back transform U = Z conj(V_t) Sigma U_t^T.
  refine     FP64 iterative refinement: R = F~ - K_h u, u += FD(R).
  bartels_stewart
             Algorithm BSc of Sec. 4.3, as stated: (1) complex Schur form
             A_t^-1 M_t = W S W^*, (2) G = F^ A_t^-1 conj(W), (3) for
             k = N_t .. 1 the spatial solve (M_x + S_kk A_x) z_k =
             g_k - sum_{j>k} S_kj A_x z_j, (4) U = Re(Z W^T).

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
    """Algorithm FD (steps 1a-4); returns the real M_x x N_t solution U.

    ``pool_map`` runs the N_t independent spatial solves of step 3 (the
    paper solves them in parallel over the time modes); the default is the
    builtin serial ``map``.
    """
    if dec is None:
        dec = decompose(At, Mt)
    F = np.asarray(F, dtype=np.float64)
    # step 2: G = F^ A_t^-1 conj(U_t) Sigma^-1 V_t^T
    W = sl.cho_solve(dec.At_cho, dec.Ut.conj())          # A_t^-1 conj(U_t)
    G = ((F @ W) / dec.sig[None, :]) @ dec.Vt.T
    # step 3: (M_x + lambda_k A_x) z_k = g_k for every k, independently
    cols = list(pool_map(_spatial_solve,
                         [(Mx, Ax, dec.lam[k], G[:, k]) for k in range(len(dec.lam))]))
    Z = np.stack(cols, axis=1)
    # step 4: u = vec(Z conj(V_t) Sigma U_t^T)
    Uc = ((Z @ dec.Vt.conj()) * dec.sig[None, :]) @ dec.Ut.T
    return Uc.real


def bartels_stewart(At, Mt, Mx, Ax, F):
    """Algorithm BSc (Bartels-Stewart with the complex Schur form, Sec. 4.3);
    returns the real M_x x N_t solution U."""
    At = np.asarray(At)
    F = np.asarray(F, dtype=np.float64)
    # step 1: A_t^-1 M_t = W S W^*, W unitary, S upper triangular
    S, W = sl.schur(np.linalg.solve(At, np.asarray(Mt)), output="complex")
    # step 2: G = F^ A_t^-1 conj(W)   (column k of G is g_k)
    G = F @ np.linalg.solve(At, W.conj())
    # step 3: backward substitution over the triangular S, one spatial solve per k
    nt = At.shape[0]
    Z = np.zeros(G.shape, dtype=np.complex128)
    for k in range(nt - 1, -1, -1):
        rhs = G[:, k] - Ax @ (Z[:, k + 1:] @ S[k, k + 1:])
        Z[:, k] = _spatial_solve((Mx, Ax, S[k, k], rhs))
    # step 4: u = (W (x) I) z, i.e. U = Z W^T (real up to rounding)
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
