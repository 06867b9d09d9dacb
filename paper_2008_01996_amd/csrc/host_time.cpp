// Time matrices A_t, M_t, C_t of the modified Hilbert transformation H_T.
//
// Sec. 2 defines, for the hats phi_1..phi_Nt and the element indicators chi_l,
//   M_t[l,k] = <phi_k, H_T phi_l>,  A_t[l,k] = <phi_k', H_T phi_l>,
//   C_t[k,l] = <chi_l, H_T phi_k>,
// with H_T the series map sin(mu_m t) -> cos(mu_m t), mu_m = (pi/2 + m pi)/T.
// Integrating by parts (phi(0) = 0, cos(mu_m T) = 0) turns every entry into a
// double integral of phi' (piecewise constant) and phi or chi against
//   L(s,t) = (2/T) sum_m cos(mu_m s) cos(mu_m t)/mu_m
//          = -(1/pi) ln|tan(pi(s-t)/4T) tan(pi(s+t)/4T)|,
// the closed sum following from sum_m cos((2m+1)y)/(2m+1) = -ln|tan(y/2)|/2.
// Hence everything reduces to the element-pair integrals
//   P[e][f] = int_{I_e} int_{I_f} L(s,t) dt ds,
//   Q[e][f] = int_{I_e} int_{I_f} L(s,t) (t - t_f^-)/h_f dt ds.
//
// Quadrature: pairs far from the singular set of L (the diagonal s = t and
// the corners (0,0), (T,T)) use a tensor Gauss-Legendre rule on L itself.
// Near pairs integrate over s in closed form for each logarithm that is
// singular on the pair (antiderivative x ln|x| - x), by Gauss-Legendre in s
// for the rest, and over t by a Gauss-Legendre rule graded towards both ends
// of the element (t = t0 + h psi(u), psi the quintic smoothstep), which
// removes the x ln x endpoint behaviour of the inner integral.
#include <cmath>
#include <vector>

#include "host_internal.hpp"

namespace stfd {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes/weights on [0, 1] by Newton iteration on P_n.
void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // final derivative at the converged node
                double q0 = 1.0, q1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double q2 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q0) / k;
                    q0 = q1;
                    q1 = q2;
                }
                const double d = n * (z * q1 - q0) / (z * z - 1.0);
                x[i] = 0.5 * (1.0 - z);
                w[i] = 1.0 / ((1.0 - z * z) * d * d);     // 2/((1-z^2)P'^2) on [-1,1], halved
                break;
            }
        }
    }
}

inline double xlogx_minus_x(double x) {      // antiderivative of ln|x|
    return x == 0.0 ? 0.0 : x * std::log(std::fabs(x)) - x;
}

struct Kernel {
    double T, alpha;   // alpha = pi / (4T)
    explicit Kernel(double T_) : T(T_), alpha(kPi / (4.0 * T_)) {}
    double L(double s, double t) const {
        return -(1.0 / kPi) * std::log(std::fabs(std::tan(alpha * (s - t)) * std::tan(alpha * (s + t))));
    }
    // ln(tan(alpha x)/x): smooth in x on [-T, T]
    double lt_over_x(double x) const {
        const double z = alpha * x;
        if (std::fabs(z) < 1e-8) return std::log(alpha * (1.0 + z * z / 3.0));
        return std::log(std::tan(z) / x);
    }
    // ln(tan(alpha y) (2T - y) / y): smooth in y on [0, 2T]
    double ly(double y) const {
        if (y <= T) {
            const double z = alpha * y;
            const double tz = (std::fabs(z) < 1e-8) ? alpha * (1.0 + z * z / 3.0) : std::tan(z) / y;
            return std::log(tz * (2.0 * T - y));
        }
        const double w = 2.0 * T - y;
        const double z = alpha * w;
        const double tz = (std::fabs(z) < 1e-8) ? alpha * (1.0 + z * z / 3.0) : std::tan(z) / w;
        return -std::log(tz * y);
    }
    // R(s,t) = L(s,t) + (1/pi)[ln|s-t| + ln(s+t) - ln(2T-s-t)]
    double R(double s, double t) const { return -(1.0 / kPi) * (lt_over_x(s - t) + ly(s + t)); }
};

}  // namespace

int assemble_time_impl(int Nt, const double* t, double* At, double* Mt, double* Ct) {
    const double T = t[Nt];
    const Kernel K(T);
    std::vector<double> h(Nt);
    for (int e = 0; e < Nt; ++e) h[e] = t[e + 1] - t[e];

    std::vector<double> gx_far, gw_far, gx_in, gw_in, gx_out, gw_out;
    gauss01(14, gx_far, gw_far);
    gauss01(20, gx_in, gw_in);
    gauss01(48, gx_out, gw_out);
    // graded outer rule: t = t0 + h psi(u), psi = 10u^3 - 15u^4 + 6u^5
    std::vector<double> go_x(gx_out.size()), go_w(gx_out.size());
    for (size_t i = 0; i < gx_out.size(); ++i) {
        const double u = gx_out[i];
        go_x[i] = u * u * u * (10.0 - 15.0 * u + 6.0 * u * u);
        go_w[i] = gw_out[i] * 30.0 * u * u * (1.0 - u) * (1.0 - u);
    }

    std::vector<double> P((size_t)Nt * Nt), Q((size_t)Nt * Nt);
#pragma omp parallel for schedule(dynamic, 4)
    for (int e = 0; e < Nt; ++e) {
        const double a = t[e], b = t[e + 1];
        for (int f = 0; f < Nt; ++f) {
            const double c = t[f], d = t[f + 1];
            const double hm = std::fmax(h[e], h[f]);
            const double dist = std::fmax(0.0, std::fmax(c - b, a - d));
            const bool nd = dist < 2.0 * hm;                 // near s = t
            const bool no = (a + c) < 2.0 * hm;              // near (0, 0)
            const bool ne = (2.0 * T - b - d) < 2.0 * hm;    // near (T, T)
            double p = 0.0, q = 0.0;
            if (!nd && !no && !ne) {
                for (size_t i = 0; i < gx_far.size(); ++i) {
                    const double s = a + h[e] * gx_far[i];
                    for (size_t j = 0; j < gx_far.size(); ++j) {
                        const double y = gx_far[j];
                        const double v = gw_far[i] * gw_far[j] * K.L(s, c + h[f] * y);
                        p += v;
                        q += v * y;
                    }
                }
                p *= h[e] * h[f];
                q *= h[e] * h[f];
            } else {
                for (size_t j = 0; j < go_x.size(); ++j) {
                    const double y = go_x[j];
                    const double tt = c + h[f] * y;
                    // inner integral over s in [a, b]
                    double logs = 0.0;      // sum of closed-form logarithms (with their signs)
                    if (nd) logs += xlogx_minus_x(b - tt) - xlogx_minus_x(a - tt);
                    if (no) logs += xlogx_minus_x(b + tt) - xlogx_minus_x(a + tt);
                    if (ne) logs -= xlogx_minus_x(2.0 * T - a - tt) - xlogx_minus_x(2.0 * T - b - tt);
                    double smooth = 0.0;    // R plus the logarithms that are smooth here
                    for (size_t i = 0; i < gx_in.size(); ++i) {
                        const double s = a + h[e] * gx_in[i];
                        double v = K.R(s, tt);
                        double lg = 0.0;
                        if (!nd) lg += std::log(std::fabs(s - tt));
                        if (!no) lg += std::log(s + tt);
                        if (!ne) lg -= std::log(2.0 * T - s - tt);
                        v -= lg / kPi;
                        smooth += gw_in[i] * v;
                    }
                    const double inner = -logs / kPi + h[e] * smooth;
                    const double wt = go_w[j] * h[f];
                    p += wt * inner;
                    q += wt * inner * y;
                }
            }
            P[(size_t)e * Nt + f] = p;
            Q[(size_t)e * Nt + f] = q;
        }
    }

    // phi_k' = +1/h_k on element k, -1/h_{k+1} on element k+1 (0-based)
    auto dphi = [&](int e, int k) -> double {
        if (e == k) return 1.0 / h[k];
        if (e == k + 1) return -1.0 / h[k + 1];
        return 0.0;
    };
    for (int l = 0; l < Nt; ++l) {
        for (int k = 0; k < Nt; ++k) {
            double a_lk = 0.0, m_lk = 0.0;
            for (int e = l; e <= l + 1 && e < Nt; ++e) {
                const double de = dphi(e, l);
                for (int f = k; f <= k + 1 && f < Nt; ++f) a_lk += de * dphi(f, k) * P[(size_t)e * Nt + f];
                // phi_k on element k rises, (t - t_k^-)/h_k; on element k+1 it falls
                double bk = Q[(size_t)e * Nt + k];
                if (k + 1 < Nt) bk += P[(size_t)e * Nt + k + 1] - Q[(size_t)e * Nt + k + 1];
                m_lk += de * bk;
            }
            At[(size_t)l * Nt + k] = a_lk;
            Mt[(size_t)l * Nt + k] = m_lk;
        }
    }
    if (Ct) {
        for (int k = 0; k < Nt; ++k)
            for (int l = 0; l < Nt; ++l) {
                double s = 0.0;
                for (int e = k; e <= k + 1 && e < Nt; ++e) s += dphi(e, k) * P[(size_t)e * Nt + l];
                Ct[(size_t)k * Nt + l] = s;
            }
    }
    return 0;
}

}  // namespace stfd
