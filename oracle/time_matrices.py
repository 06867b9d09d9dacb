"""Time matrices of the modified Hilbert transformation H_T (oracle, FP64).

Definitions (Sec. 2, after the global linear system):
    M_t[l, k] = < phi_k , H_T phi_l >_{L2(0,T)}
    A_t[l, k] = < d/dt phi_k , H_T phi_l >_{L2(0,T)}
    C_t[k, l] = < chi_l , H_T phi_k >_{L2(0,T)}
for the piecewise-linear hats phi_1..phi_Nt (phi_0 is dropped because of the
zero initial condition; phi_Nt is the half hat with phi_Nt(T) = 1) and the
element indicators chi_l = phi^0_l.  Row index = test function.

H_T (Sec. 2, series definition): with mu_m = (pi/2 + m pi)/T,
    v = sum_m v_m sin(mu_m t)   ->   H_T v = sum_m v_m cos(mu_m t),
and v_m = (2/T) <v, sin(mu_m .)> because these sines are orthogonal on (0,T)
with squared norm T/2.

Route 1, ``series``: the definition, truncated after K modes.  The
per-mode coefficients are exact (integration by parts on each element,
using phi(0) = 0 and cos(mu_m T) = 0); the tail after K modes is bounded
rigorously and returned.  Terms decay like mu^-3, so this route is only
affordable on coarse meshes; it is the brute-force pin of route 2.

Route 2, ``kernel``: the same series summed in closed form.  With
s_m = sin(mu_m .), c_m = cos(mu_m .), integration by parts gives
<phi, s_m> = <phi', c_m>/mu_m, so every matrix is a double integral of the
piecewise-constant derivatives (and of the hats themselves) against
    L(s,t) = (2/T) sum_m c_m(s) c_m(t) / mu_m
           = -(1/pi) ln | tan(pi (s-t)/(4T)) * tan(pi (s+t)/(4T)) |,
by the Fourier series sum_{m>=0} cos((2m+1)y)/(2m+1) = -1/2 ln|tan(y/2)|:
    A_t[l,k] = int int phi_l'(s) phi_k'(t)  L(s,t) ds dt
    M_t[l,k] = int int phi_l'(s) phi_k(t)   L(s,t) ds dt
    C_t[k,l] = int int phi_k'(s) chi_l(t)   L(s,t) ds dt.
L has logarithmic singularities on s = t, at (0,0) and at (T,T); it is split
as  L = -(1/pi) [ln|s-t| + ln(s+t) - ln(2T-s-t)] + R  with R analytic on
[0,T]^2.  The logarithms are integrated over each element pair in closed
form where the pair is close to their singular set and by tensor
Gauss-Legendre elsewhere; R always by tensor Gauss-Legendre.

Parity status: pinned by tests (series vs kernel on small meshes, the
paper's eigenvalue table, closed-form integrals vs scipy dblquad, symmetry
and positivity, scale invariance).
"""
from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------------------------
# common helpers
# ----------------------------------------------------------------------------

def _check_times(t: np.ndarray) -> np.ndarray:
    t = np.asarray(t, dtype=np.float64)
    if t.ndim != 1 or len(t) < 2 or t[0] != 0.0 or np.any(np.diff(t) <= 0):
        raise ValueError("time nodes must be strictly increasing and start at 0")
    return t


def hat_derivatives(t: np.ndarray) -> np.ndarray:
    """D[e, k] = phi_{k+1}' on element e+1 (0-based arrays), shape (Nt, Nt).

    phi_k rises on (t_{k-1}, t_k) with slope 1/h_k and falls on
    (t_k, t_{k+1}) with slope -1/h_{k+1}; phi_Nt only rises.
    """
    t = _check_times(t)
    nt = len(t) - 1
    h = np.diff(t)
    D = np.zeros((nt, nt))
    for k in range(nt):
        D[k, k] = 1.0 / h[k]
        if k + 1 < nt:
            D[k + 1, k] = -1.0 / h[k + 1]
    return D


# ----------------------------------------------------------------------------
# route 1: truncated eigen-series with exact per-mode coefficients
# ----------------------------------------------------------------------------

def _mode_coefficients(t, mu):
    """Exact <phi_k, s_m>, <phi_k, c_m>, <chi_l, c_m> for a block of modes.

    Returns S (m, Nt), G (m, Nt), E (m, Nt).
    """
    nt = len(t) - 1
    D = hat_derivatives(t)                       # (e, k)
    mu = mu[:, None]
    sin_t = np.sin(mu * t[None, :])              # (m, Nt+1)
    cos_t = np.cos(mu * t[None, :])
    dsin = sin_t[:, 1:] - sin_t[:, :-1]          # sin(mu t_e) - sin(mu t_{e-1})
    dcos = cos_t[:, :-1] - cos_t[:, 1:]          # cos(mu t_{e-1}) - cos(mu t_e)
    # <phi_k, sin(mu t)> = mu^-2 sum_e phi_k'|_e (sin mu t_e - sin mu t_{e-1})
    S = (dsin @ D) / mu**2
    # <phi_k, cos(mu t)> = phi_k(T) sin(mu T)/mu
    #                      - mu^-2 sum_e phi_k'|_e (cos mu t_{e-1} - cos mu t_e)
    G = -(dcos @ D) / mu**2
    G[:, nt - 1] += np.sin(mu[:, 0] * t[-1]) / mu[:, 0]
    # <chi_l, cos(mu t)> = (sin mu t_l - sin mu t_{l-1}) / mu
    E = dsin / mu
    return S, G, E


def series(t, n_modes: int, chunk: int = 20000):
    """A_t, M_t, C_t from the first ``n_modes`` terms of the H_T series.

    Returns (A, M, C, tail) where ``tail`` bounds max |entry error| of the
    truncation for all three matrices.
    """
    t = _check_times(t)
    T = t[-1]
    nt = len(t) - 1
    A = np.zeros((nt, nt))
    M = np.zeros((nt, nt))
    C = np.zeros((nt, nt))
    # sum chunk partial sums in a second level to keep rounding small
    for m0 in range(0, n_modes, chunk):
        m = np.arange(m0, min(n_modes, m0 + chunk), dtype=np.float64)
        mu = (math.pi / 2 + m * math.pi) / T
        S, G, E = _mode_coefficients(t, mu)
        # A[l,k] = (2/T) sum_m mu_m S[m,l] S[m,k]
        A += (2.0 / T) * ((S * mu[:, None]).T @ S)
        # M[l,k] = (2/T) sum_m S[m,l] G[m,k]
        M += (2.0 / T) * (S.T @ G)
        # C[k,l] = (2/T) sum_m S[m,k] E[m,l]
        C += (2.0 / T) * (S.T @ E)
    tail = series_tail_bound(t, n_modes)
    return A, M, C, tail


def series_tail_bound(t, n_modes: int) -> float:
    """Rigorous bound of the entries of the neglected modes m >= n_modes.

    |<phi_k, s_m>| <= mu^-2 s_k with s_k = 2 sum_e |phi_k'|_e|,
    |<phi_k, c_m>| <= mu^-1 delta_{k,Nt} + mu^-2 s_k,  |<chi, c_m>| <= 2/mu,
    and sum_{m>=K} mu_m^-p <= (2T/pi)^p (2K)^(1-p) / (2(p-1)) (midpoint
    bound of a convex decreasing sum).
    """
    t = _check_times(t)
    T = t[-1]
    D = hat_derivatives(t)
    s = 2.0 * np.abs(D).sum(axis=0).max()
    K = float(n_modes)

    def tailsum(p):
        return (2 * T / math.pi) ** p * (2 * K) ** (1 - p) / (2 * (p - 1))

    bA = (2 / T) * s * s * tailsum(3)
    bM = (2 / T) * (s * tailsum(3) + s * s * tailsum(4))
    bC = (2 / T) * s * 2 * tailsum(3)
    return max(bA, bM, bC)


# ----------------------------------------------------------------------------
# route 2: summed series (log-tan kernel), element-pair integrals
# ----------------------------------------------------------------------------

def kernel_L(s, t, T):
    """L(s,t) = -(1/pi) ln|tan(pi(s-t)/(4T)) tan(pi(s+t)/(4T))|."""
    a = math.pi / (4 * T)
    return -(1 / math.pi) * np.log(np.abs(np.tan(a * (s - t)) * np.tan(a * (s + t))))


def _tanc(z):
    """tan(z)/z, with the removable value 1 at z = 0."""
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0
    out[nz] = np.tan(z[nz]) / z[nz]
    return out


def kernel_R(s, t, T):
    """Analytic remainder R = L + (1/pi)[ln|s-t| + ln(s+t) - ln(2T-s-t)].

    ln|tan(a x)| - ln|x| = ln(a tanc(a x)) with a = pi/(4T), and for y = s+t
    in (0, 2T):  tan(a y) (2T-y)/y = a tanc(a y) (2T-y)          (y <= T)
                                   = 1/(a tanc(a (2T-y)) y)        (y >  T),
    the second form because tan(a y) = 1/tan(a (2T-y)).
    """
    a = math.pi / (4 * T)
    s = np.asarray(s, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    x = s - t
    y = s + t
    r1 = np.log(a * _tanc(a * x))
    lo = y <= T
    r2 = np.empty(np.broadcast(s, t).shape)
    r2[lo] = np.log(a * _tanc(a * y[lo]) * (2 * T - y[lo]))
    hi = ~lo
    r2[hi] = -np.log(a * _tanc(a * (2 * T - y[hi])) * y[hi])
    return -(1 / math.pi) * (r1 + r2)


def _phi1(x):
    """Antiderivative of ln|x|:  x ln|x| - x."""
    x = np.asarray(x, dtype=np.float64)
    out = -x.copy()
    nz = x != 0
    out[nz] += x[nz] * np.log(np.abs(x[nz]))
    return out


def _phi2(x):
    """Second antiderivative of ln|x|:  x^2/2 ln|x| - 3x^2/4."""
    x = np.asarray(x, dtype=np.float64)
    out = -0.75 * x * x
    nz = x != 0
    out[nz] += 0.5 * x[nz] ** 2 * np.log(np.abs(x[nz]))
    return out


def _phi3(x):
    """Third antiderivative of ln|x|:  x^3/6 ln|x| - 11x^3/36."""
    x = np.asarray(x, dtype=np.float64)
    out = -(11.0 / 36.0) * x ** 3
    nz = x != 0
    out[nz] += x[nz] ** 3 / 6.0 * np.log(np.abs(x[nz]))
    return out


def log_rect_integrals(sig, tau, gam, h, hp):
    """Closed-form integrals over the rectangle [0,h] x [0,hp] of
    ln|sig x + tau y + gam| (weight 1) and (weight y/hp), sig, tau = +-1.

    With Phi1' = ln|.|, Phi2' = Phi1, Phi3' = Phi2:
      I0 = (1/(sig tau)) [Phi2(sig h + tau hp + gam) - Phi2(tau hp + gam)
                          - Phi2(sig h + gam) + Phi2(gam)]
      I1 = (hp/(sig tau)) [Phi2(sig h + tau hp + gam) - Phi2(tau hp + gam)]
           - (1/sig) [Phi3(sig h + tau hp + gam) - Phi3(tau hp + gam)
                      - Phi3(sig h + gam) + Phi3(gam)]
    (inner integral in y by parts, then the outer integral in x).
    Returns (I0, I1 / hp).
    """
    st = sig * tau
    a = sig * h + tau * hp + gam
    b = tau * hp + gam
    c = sig * h + gam
    d = gam
    I0 = (_phi2(a) - _phi2(b) - _phi2(c) + _phi2(d)) / st
    I1 = hp * (_phi2(a) - _phi2(b)) / st - (_phi3(a) - _phi3(b) - _phi3(c) + _phi3(d)) / sig
    return I0, I1 / hp


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w          # nodes/weights on [0,1]


def element_pair_integrals(t, n_near: int = 16, n_far: int = 8):
    """P[e,f] = int_{I_e} int_{I_f} L ds dt and
    Q[e,f] = int_{I_e} int_{I_f} L(s,t) (t - t_{f-1})/h_f ds dt
    (s on element e, t on element f, both 0-based), shape (Nt, Nt).
    """
    t = _check_times(t)
    T = t[-1]
    nt = len(t) - 1
    h = np.diff(t)
    a = t[:-1]
    E, F = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    E = E.ravel()
    F = F.ravel()
    he, hf = h[E], h[F]
    ae, af = a[E], a[F]
    hmax = np.maximum(he, hf)

    # distance of the rectangle to each singular set, relative to its size
    dist_diag = np.maximum(0.0, np.maximum(af - (ae + he), ae - (af + hf)))
    dist_orig = ae + af
    dist_end = 2 * T - (ae + he) - (af + hf)
    near_diag = dist_diag < hmax
    near_orig = dist_orig < hmax
    near_end = dist_end < hmax

    P = np.zeros(nt * nt)
    Q = np.zeros(nt * nt)

    # (i) analytic remainder R, and the logs on far pairs, by tensor Gauss
    ratio = np.minimum(np.minimum(np.where(near_diag, np.inf, dist_diag),
                                  np.where(near_orig, np.inf, dist_orig)),
                       np.where(near_end, np.inf, dist_end)) / hmax
    use_near_rule = (ratio < 8.0) | (hmax > T / 16)
    for rule_mask, n in ((use_near_rule, n_near), (~use_near_rule, n_far)):
        idx = np.nonzero(rule_mask)[0]
        if len(idx) == 0:
            continue
        xg, wg = _gauss(n)
        for c0 in range(0, len(idx), 4096):
            ii = idx[c0:c0 + 4096]
            s = ae[ii, None, None] + he[ii, None, None] * xg[None, :, None]
            y = xg[None, None, :]
            tt = af[ii, None, None] + hf[ii, None, None] * y
            w2 = (wg[:, None] * wg[None, :])[None] * (he[ii] * hf[ii])[:, None, None]
            val = kernel_R(s, tt, T)
            with np.errstate(divide="ignore", invalid="ignore"):
                lg = np.zeros_like(val)
                nd = ~near_diag[ii]
                lg[nd] += np.log(np.abs(s[nd] - tt[nd]))
                no = ~near_orig[ii]
                lg[no] += np.log(s[no] + tt[no])
                ne = ~near_end[ii]
                lg[ne] -= np.log(2 * T - s[ne] - tt[ne])
            val = val - lg / math.pi
            P[ii] += (w2 * val).sum(axis=(1, 2))
            Q[ii] += (w2 * val * y).sum(axis=(1, 2))

    # (ii) logs on near pairs in closed form; local coordinates x = s - a_e,
    # y = t - a_f
    for mask, sig, tau, gam, sign in (
        (near_diag, 1.0, -1.0, ae - af, 1.0),            # ln|s - t|
        (near_orig, 1.0, 1.0, ae + af, 1.0),             # ln(s + t)
        (near_end, -1.0, -1.0, 2 * T - ae - af, -1.0),   # -ln(2T - s - t)
    ):
        idx = np.nonzero(mask)[0]
        if len(idx) == 0:
            continue
        I0, I1 = log_rect_integrals(sig, tau, gam[idx], he[idx], hf[idx])
        P[idx] += -(sign / math.pi) * I0
        Q[idx] += -(sign / math.pi) * I1
    return P.reshape(nt, nt), Q.reshape(nt, nt)


def kernel(t, n_near: int = 16, n_far: int = 8):
    """A_t, M_t, C_t from the summed series (route 2)."""
    t = _check_times(t)
    nt = len(t) - 1
    P, Q = element_pair_integrals(t, n_near, n_far)
    D = hat_derivatives(t)                       # D[e,k] = phi_k' on element e
    # C[k,l] = sum_e phi_k'|_e P[e,l]
    C = D.T @ P
    # A[l,k] = sum_{e,f} phi_l'|_e phi_k'|_f P[e,f]
    A = D.T @ P @ D
    # phi_k on element f: rising part (t - t_{f-1})/h_f on f = k, falling part
    # 1 - (t - t_{f-1})/h_f on f = k+1 (0-based: f = k and f = k + 1)
    B = np.zeros((nt, nt))                       # B[e,k] = int_e int phi_k L
    for k in range(nt):
        B[:, k] += Q[:, k]
        if k + 1 < nt:
            B[:, k] += P[:, k + 1] - Q[:, k + 1]
    # M[l,k] = sum_e phi_l'|_e B[e,k]
    M = D.T @ B
    return A, M, C


def time_matrices(t, route: str = "kernel", **kw):
    """Dispatch helper: ``route`` in {"kernel", "series"}."""
    if route == "kernel":
        return kernel(t, **kw)
    if route == "series":
        A, M, C, _ = series(t, **kw)
        return A, M, C
    raise ValueError(route)
