// Dense FP64 host linear algebra for the FD setup; see host_linalg.hpp.
#include "host_linalg.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace stfd {

bool cholesky(int n, std::vector<double>& a) {
    for (int j = 0; j < n; ++j) {
        double d = a[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        d = std::sqrt(d);
        a[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = a[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
            a[(size_t)i * n + j] = s / d;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) a[(size_t)i * n + j] = 0.0;
    return true;
}

template <typename T>
static void fwd_impl(int n, const std::vector<double>& L, T* b, int nrhs) {
    for (int i = 0; i < n; ++i) {
        T* bi = b + (size_t)i * nrhs;
        for (int k = 0; k < i; ++k) {
            const double l = L[(size_t)i * n + k];
            const T* bk = b + (size_t)k * nrhs;
            for (int r = 0; r < nrhs; ++r) bi[r] -= l * bk[r];
        }
        const double d = L[(size_t)i * n + i];
        for (int r = 0; r < nrhs; ++r) bi[r] /= d;
    }
}

template <typename T>
static void bwd_impl(int n, const std::vector<double>& L, T* b, int nrhs) {
    for (int i = n - 1; i >= 0; --i) {
        T* bi = b + (size_t)i * nrhs;
        for (int k = i + 1; k < n; ++k) {
            const double l = L[(size_t)k * n + i];
            const T* bk = b + (size_t)k * nrhs;
            for (int r = 0; r < nrhs; ++r) bi[r] -= l * bk[r];
        }
        const double d = L[(size_t)i * n + i];
        for (int r = 0; r < nrhs; ++r) bi[r] /= d;
    }
}

void chol_forward(int n, const std::vector<double>& L, double* b, int nrhs) { fwd_impl(n, L, b, nrhs); }
void chol_backward(int n, const std::vector<double>& L, double* b, int nrhs) { bwd_impl(n, L, b, nrhs); }
void chol_forward(int n, const std::vector<double>& L, cd* b, int nrhs) { fwd_impl(n, L, b, nrhs); }
void chol_backward(int n, const std::vector<double>& L, cd* b, int nrhs) { bwd_impl(n, L, b, nrhs); }

// ---------------------------------------------------------------------------
// Householder reduction to upper Hessenberg form, H = Q^T A Q.
// ---------------------------------------------------------------------------
static void hessenberg(int n, std::vector<double>& a, std::vector<double>& q) {
    q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n);
    for (int k = 0; k + 2 < n; ++k) {
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += a[(size_t)i * n + k] * a[(size_t)i * n + k];
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        const double x0 = a[(size_t)(k + 1) * n + k];
        if (x0 > 0) alpha = -alpha;             // v = x - alpha e1, alpha = -sign(x0)|x|
        double vnorm2 = 0.0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = a[(size_t)i * n + k];
        }
        v[k + 1] -= alpha;
        for (int i = k + 1; i < n; ++i) vnorm2 += v[i] * v[i];
        if (vnorm2 == 0.0) continue;
        const double beta = 2.0 / vnorm2;
        // A <- (I - beta v v^T) A   (rows k+1..n-1); columns, rows and rows
        // of Q below are independent, each with its sums in the same order
#pragma omp parallel for schedule(static)
        for (int j = k; j < n; ++j) {
            double s = 0.0;
            for (int i = k + 1; i < n; ++i) s += v[i] * a[(size_t)i * n + j];
            s *= beta;
            for (int i = k + 1; i < n; ++i) a[(size_t)i * n + j] -= s * v[i];
        }
        // A <- A (I - beta v v^T)   (columns k+1..n-1)
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double* ai = &a[(size_t)i * n];
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += ai[j] * v[j];
            s *= beta;
            for (int j = k + 1; j < n; ++j) ai[j] -= s * v[j];
        }
        // Q <- Q (I - beta v v^T)
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double* qi = &q[(size_t)i * n];
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += qi[j] * v[j];
            s *= beta;
            for (int j = k + 1; j < n; ++j) qi[j] -= s * v[j];
        }
        for (int i = k + 2; i < n; ++i) a[(size_t)i * n + k] = 0.0;
    }
}

static inline double cabs1(cd z) { return std::fabs(z.real()) + std::fabs(z.imag()); }

// Unitary plane rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0].
static inline void givens(cd x, cd y, double& c, cd& s) {
    const double ay = std::abs(y);
    if (ay == 0.0) { c = 1.0; s = 0.0; return; }
    const double ax = std::abs(x);
    if (ax == 0.0) { c = 0.0; s = std::conj(y) / ay; return; }
    const double r = std::hypot(ax, ay);
    c = ax / r;
    s = (x / ax) * std::conj(y) / r;
}

// ---------------------------------------------------------------------------
// Single-shift complex QR on an upper Hessenberg matrix, full Schur form
// T = Z^H H Z accumulated into z.  Wilkinson shifts, exceptional shifts every
// ten iterations without deflation.
//
// A sweep's rotations act on the row pairs (k, k+1) of H and on the column
// pairs (k, k+1) of H and Z.  The bulge chase only reads columns up to ihi
// and, of the columns k, k+1, rows k-1..k+2 again.  So the column rotations
// of the rows above (and all of Z, which it never reads) and the row
// rotations of the columns right of the active window (which no column
// rotation of the sweep touches) are kept and applied after the sweep: row by
// row, resp. in blocks of columns, each over contiguous memory and in
// parallel.  Every entry sees the same operations in the same order as with
// immediate updates.
// ---------------------------------------------------------------------------
static bool schur_complex(int n, std::vector<cd>& h, std::vector<cd>& z, std::string* err) {
    const double eps = std::numeric_limits<double>::epsilon();
    double hnorm = 0.0;
    for (auto& x : h) hnorm = std::max(hnorm, cabs1(x));
    const double small = std::max(hnorm, 1.0) * std::numeric_limits<double>::min() / eps;
    int ihi = n - 1;
    int iter = 0, total = 0;
    std::vector<double> rot_c(n);
    std::vector<cd> rot_s(n);
    while (ihi > 0) {
        int l = ihi;
        for (; l > 0; --l) {
            const cd sub = h[(size_t)l * n + l - 1];
            double tst = cabs1(h[(size_t)(l - 1) * n + l - 1]) + cabs1(h[(size_t)l * n + l]);
            if (tst == 0.0) tst = hnorm;
            if (cabs1(sub) <= eps * tst || cabs1(sub) <= small) {
                h[(size_t)l * n + l - 1] = 0.0;
                break;
            }
        }
        if (l == ihi) {            // 1x1 block deflated
            --ihi;
            iter = 0;
            continue;
        }
        ++iter;
        if (++total > 60 * n) {
            if (err) *err = "complex QR iteration did not converge";
            return false;
        }
        cd mu;
        const cd a = h[(size_t)(ihi - 1) * n + ihi - 1];
        const cd b = h[(size_t)(ihi - 1) * n + ihi];
        const cd c = h[(size_t)ihi * n + ihi - 1];
        const cd d = h[(size_t)ihi * n + ihi];
        if (iter % 10 == 0) {
            mu = d + 0.75 * std::abs(c);          // exceptional shift
        } else {
            // eigenvalue of [[a, b], [c, d]] closest to d
            const cd tr2 = 0.5 * (a - d);
            const cd disc = std::sqrt(tr2 * tr2 + b * c);
            const cd e1 = 0.5 * (a + d) + disc;
            const cd e2 = 0.5 * (a + d) - disc;
            mu = (std::abs(e1 - d) < std::abs(e2 - d)) ? e1 : e2;
        }
        // shifted QR sweep on rows/columns l..ihi by a chase of rotations
        cd x = h[(size_t)l * n + l] - mu;
        cd y = h[(size_t)(l + 1) * n + l];
        for (int k = l; k < ihi; ++k) {
            if (k > l) {
                x = h[(size_t)k * n + k - 1];
                y = h[(size_t)(k + 1) * n + k - 1];
            }
            double cs;
            cd sn;
            givens(x, y, cs, sn);
            rot_c[k] = cs;
            rot_s[k] = sn;
            // rows k, k+1 from column max(k-1, l) to ihi; columns ihi+1..n-1
            // follow after the sweep
            const int j0 = (k > l) ? k - 1 : l;
            cd* rk = &h[(size_t)k * n];
            cd* rk1 = &h[(size_t)(k + 1) * n];
            for (int j = j0; j <= ihi; ++j) {
                const cd u = rk[j], v = rk1[j];
                rk[j] = cs * u + sn * v;
                rk1[j] = -std::conj(sn) * u + cs * v;
            }
            if (k > l) h[(size_t)(k + 1) * n + k - 1] = 0.0;
            // columns k, k+1 (times G^H) for the rows the chase reads again,
            // max(0, k-1)..min(k+2, ihi); rows 0..k-2 follow after the sweep
            const int i1 = std::min(k + 2, ihi);
            const cd snc = std::conj(sn);
            for (int i = std::max(0, k - 1); i <= i1; ++i) {
                cd* ri = &h[(size_t)i * n];
                const cd u = ri[k], v = ri[k + 1];
                ri[k] = cs * u + snc * v;
                ri[k + 1] = -sn * u + cs * v;
            }
        }
        // the deferred row rotations of columns ihi+1..n-1, in blocks of 16
        // columns (two contiguous row segments per rotation)
        constexpr int JB = 16;
#pragma omp parallel for schedule(static)
        for (int jb = ihi + 1; jb < n; jb += JB) {
            const int je = std::min(n, jb + JB);
            for (int k = l; k < ihi; ++k) {
                const double cs = rot_c[k];
                const cd sn = rot_s[k], snc = std::conj(sn);
                cd* rk = &h[(size_t)k * n];
                cd* rk1 = &h[(size_t)(k + 1) * n];
                for (int j = jb; j < je; ++j) {
                    const cd u = rk[j], v = rk1[j];
                    rk[j] = cs * u + sn * v;
                    rk1[j] = -snc * u + cs * v;
                }
            }
        }
        // the deferred column rotations: row i of H takes those of steps
        // k >= max(l, i+2), every row of Z those of all steps l..ihi-1
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            cd* zi = &z[(size_t)i * n];
            for (int k = l; k < ihi; ++k) {
                const double cs = rot_c[k];
                const cd sn = rot_s[k], snc = std::conj(sn);
                const cd u = zi[k], v = zi[k + 1];
                zi[k] = cs * u + snc * v;
                zi[k + 1] = -sn * u + cs * v;
            }
            if (i + 2 < ihi) {
                cd* ri = &h[(size_t)i * n];
                for (int k = std::max(l, i + 2); k < ihi; ++k) {
                    const double cs = rot_c[k];
                    const cd sn = rot_s[k], snc = std::conj(sn);
                    const cd u = ri[k], v = ri[k + 1];
                    ri[k] = cs * u + snc * v;
                    ri[k + 1] = -sn * u + cs * v;
                }
            }
        }
    }
    return true;
}

bool schur_real(int n, std::vector<double>& a, std::vector<cd>& t, std::vector<cd>& z, std::string* err) {
    std::vector<double> q;
    hessenberg(n, a, q);
    t.assign((size_t)n * n, 0.0);
    z.assign((size_t)n * n, 0.0);
    for (size_t i = 0; i < t.size(); ++i) {
        t[i] = a[i];
        z[i] = q[i];
    }
    if (!schur_complex(n, t, z, err)) return false;
    for (int i = 1; i < n; ++i)                          // exact zeros below the diagonal
        for (int j = 0; j < i; ++j) t[(size_t)i * n + j] = 0.0;
    return true;
}

bool eig_real(int n, std::vector<double>& a, std::vector<cd>& vals, std::vector<cd>& vecs,
              std::string* err) {
    std::vector<double> q;
    hessenberg(n, a, q);
    std::vector<cd> h((size_t)n * n), z((size_t)n * n);
    for (size_t i = 0; i < h.size(); ++i) {
        h[i] = a[i];
        z[i] = q[i];
    }
    if (!schur_complex(n, h, z, err)) return false;
    vals.resize(n);
    for (int k = 0; k < n; ++k) vals[k] = h[(size_t)k * n + k];
    // eigenvectors of the triangular T: (T - t_kk I) v = 0, v_k = 1
    double tnorm = 0.0;
    for (auto& x : h) tnorm = std::max(tnorm, cabs1(x));
    const double smin = std::max(std::numeric_limits<double>::epsilon() * tnorm,
                                 std::numeric_limits<double>::min());
    vecs.assign((size_t)n * n, 0.0);
    // the eigenvectors are independent of each other
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < n; ++k) {
        std::vector<cd> v(n, cd(0.0));
        v[k] = 1.0;
        const cd tkk = h[(size_t)k * n + k];
        for (int i = k - 1; i >= 0; --i) {
            cd s = 0.0;
            const cd* ti = &h[(size_t)i * n];
            for (int j = i + 1; j <= k; ++j) s += ti[j] * v[j];
            cd den = ti[i] - tkk;
            if (cabs1(den) < smin) den = smin;
            v[i] = -s / den;
            // rescale to avoid overflow on badly separated eigenvalues
            if (cabs1(v[i]) > 1e150) {
                for (int j = i; j <= k; ++j) v[j] *= 1e-150;
            }
        }
        // y = Z v
        for (int i = 0; i < n; ++i) {
            const cd* zi = &z[(size_t)i * n];
            cd s = 0.0;
            for (int j = 0; j <= k; ++j) s += zi[j] * v[j];
            vecs[(size_t)i * n + k] = s;
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD.  Columns of a are orthogonalised by plane
// rotations applied on the right; V accumulates the rotations.  Pairs are
// visited in a round-robin tournament so that each round's rotations are
// independent.  Columns are kept column-major with separate real and
// imaginary parts (the loops over a column vectorise), and the squared
// column norms are carried through each sweep by the rotation's closed form
// (||a_p||^2 - t g, ||a_q||^2 + t g) and recomputed at the start of the next,
// so that a pair needs one complex inner product.
// ---------------------------------------------------------------------------
bool svd_jacobi(int n, std::vector<cd>& a, std::vector<cd>& U, std::vector<double>& s,
                std::vector<cd>& V, std::string* err, const std::vector<cd>* v0) {
    const double eps = std::numeric_limits<double>::epsilon();
    // rotation threshold on the cosine between two columns: sqrt(n) eps, the
    // level the rounding of the column inner products allows
    const double tol = std::sqrt((double)n) * eps;
    const size_t nn = (size_t)n * n;
    std::vector<double> Ar(nn), Ai(nn), Wr(nn, 0.0), Wi(nn, 0.0), nrm(n);
    if (v0) {
        // start from a V0 that already nearly orthogonalises the columns:
        // columns a V0, accumulated rotations V0
        std::vector<cd> ac(nn);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) ac[(size_t)k * n + i] = a[(size_t)i * n + k];
#pragma omp parallel for schedule(static)
        for (int j = 0; j < n; ++j) {
            std::vector<cd> col(n, 0.0);
            for (int k = 0; k < n; ++k) {
                const cd w = (*v0)[(size_t)k * n + j];
                const cd* ak = &ac[(size_t)k * n];
                for (int i = 0; i < n; ++i) col[i] += ak[i] * w;
            }
            for (int i = 0; i < n; ++i) {
                Ar[(size_t)j * n + i] = col[i].real();
                Ai[(size_t)j * n + i] = col[i].imag();
                Wr[(size_t)j * n + i] = (*v0)[(size_t)i * n + j].real();
                Wi[(size_t)j * n + i] = (*v0)[(size_t)i * n + j].imag();
            }
        }
    } else {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                Ar[(size_t)j * n + i] = a[(size_t)i * n + j].real();
                Ai[(size_t)j * n + i] = a[(size_t)i * n + j].imag();
            }
        for (int j = 0; j < n; ++j) Wr[(size_t)j * n + j] = 1.0;
    }
    const int m = n + (n & 1);            // tournament size (pad with a dummy)
    std::vector<int> ring(m);
    for (int i = 0; i < m; ++i) ring[i] = i;
    bool converged = false;
    for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < n; ++j) {
            const double* xr = &Ar[(size_t)j * n];
            const double* xi = &Ai[(size_t)j * n];
            double t = 0.0;
            for (int i = 0; i < n; ++i) t += xr[i] * xr[i] + xi[i] * xi[i];
            nrm[j] = t;
        }
        double off = 0.0;
        for (int round = 0; round < m - 1; ++round) {
#pragma omp parallel for schedule(static) reduction(max : off)
            for (int pidx = 0; pidx < m / 2; ++pidx) {
                int p = ring[pidx], q = ring[m - 1 - pidx];
                if (p >= n || q >= n) continue;
                if (p > q) std::swap(p, q);
                double* pr = &Ar[(size_t)p * n];
                double* pi = &Ai[(size_t)p * n];
                double* qr = &Ar[(size_t)q * n];
                double* qi = &Ai[(size_t)q * n];
                const double al = nrm[p], be = nrm[q];
                // ga = <a_p, a_q> = sum conj(a_p) a_q
                double gr = 0.0, gi = 0.0;
                for (int i = 0; i < n; ++i) {
                    gr += pr[i] * qr[i] + pi[i] * qi[i];
                    gi += pr[i] * qi[i] - pi[i] * qr[i];
                }
                const double g = std::hypot(gr, gi);
                if (g == 0.0 || g <= tol * std::sqrt(al * be)) continue;
                off = std::max(off, g / std::sqrt(al * be));
                // D = diag(1, e^{-i phi}) makes the Gram matrix real; then a
                // real Jacobi rotation diagonalises it
                const double phr = gr / g, phi = -gi / g;          // e^{-i phi} = conj(ga) / |ga|
                const double zeta = (be - al) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t);
                const double sn = c * t;
                for (int i = 0; i < n; ++i) {
                    const double xr = pr[i], xi = pi[i];
                    const double yr = phr * qr[i] - phi * qi[i], yi = phr * qi[i] + phi * qr[i];
                    pr[i] = c * xr - sn * yr;
                    pi[i] = c * xi - sn * yi;
                    qr[i] = sn * xr + c * yr;
                    qi[i] = sn * xi + c * yi;
                }
                double* wpr = &Wr[(size_t)p * n];
                double* wpi = &Wi[(size_t)p * n];
                double* wqr = &Wr[(size_t)q * n];
                double* wqi = &Wi[(size_t)q * n];
                for (int i = 0; i < n; ++i) {
                    const double xr = wpr[i], xi = wpi[i];
                    const double yr = phr * wqr[i] - phi * wqi[i], yi = phr * wqi[i] + phi * wqr[i];
                    wpr[i] = c * xr - sn * yr;
                    wpi[i] = c * xi - sn * yi;
                    wqr[i] = sn * xr + c * yr;
                    wqi[i] = sn * xi + c * yi;
                }
                nrm[p] = al - t * g;
                nrm[q] = be + t * g;
            }
            // rotate the tournament (element 0 fixed)
            const int last = ring[m - 1];
            for (int i = m - 1; i > 1; --i) ring[i] = ring[i - 1];
            ring[1] = last;
        }
        if (off <= tol) converged = true;
    }
    if (!converged) {
        if (err) *err = "Jacobi SVD did not converge";
        return false;
    }
    std::vector<double> sv(n);
    for (int j = 0; j < n; ++j) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += Ar[(size_t)j * n + i] * Ar[(size_t)j * n + i] + Ai[(size_t)j * n + i] * Ai[(size_t)j * n + i];
        sv[j] = std::sqrt(t);
    }
    std::vector<int> order(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return sv[x] > sv[y]; });
    s.resize(n);
    U.assign(nn, 0.0);
    V.assign(nn, 0.0);
    for (int jj = 0; jj < n; ++jj) {
        const int j = order[jj];
        s[jj] = sv[j];
        const double inv = sv[j] > 0 ? 1.0 / sv[j] : 0.0;
        for (int i = 0; i < n; ++i) {
            U[(size_t)i * n + jj] = cd(Ar[(size_t)j * n + i], Ai[(size_t)j * n + i]) * inv;
            V[(size_t)i * n + jj] = cd(Wr[(size_t)j * n + i], Wi[(size_t)j * n + i]);
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// Right singular vectors by Householder QR with column pivoting and the
// one-sided Jacobi SVD of R^H (Drmac and Veselic): A P = Q R and
// R^H = U_R S V_R^H give A = (Q V_R) S (P U_R)^H, so V = P U_R.  The sweeps
// on R^H are far fewer than on A, whose columns are far from orthogonal.
// ---------------------------------------------------------------------------
static bool right_vectors_qrp(int n, const std::vector<cd>& a, std::vector<cd>& V, std::string* err) {
    const size_t nn = (size_t)n * n;
    std::vector<cd> A(nn);                 // column-major working copy
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)j * n + i] = a[(size_t)i * n + j];
    std::vector<int> perm(n);
    for (int j = 0; j < n; ++j) perm[j] = j;
    std::vector<double> cn(n);
    std::vector<cd> v(n);
    for (int k = 0; k < n; ++k) {
        // pivot: the remaining column of largest norm (rows k..n-1)
#pragma omp parallel for schedule(static)
        for (int j = k; j < n; ++j) {
            const cd* c = &A[(size_t)j * n];
            double t = 0.0;
            for (int i = k; i < n; ++i) t += std::norm(c[i]);
            cn[j] = t;
        }
        int p = k;
        for (int j = k + 1; j < n; ++j)
            if (cn[j] > cn[p]) p = j;
        if (p != k) {
            std::swap_ranges(A.begin() + (size_t)k * n, A.begin() + (size_t)(k + 1) * n, A.begin() + (size_t)p * n);
            std::swap(perm[k], perm[p]);
        }
        // reflector H = I - tau v v^H with H x = beta e_k, beta = -e^{i arg x_k} |x|
        cd* x = &A[(size_t)k * n];
        const double xnorm = std::sqrt(cn[p]);
        if (xnorm == 0.0) continue;
        const double ax0 = std::abs(x[k]);
        const cd ph = ax0 > 0.0 ? x[k] / ax0 : cd(1.0, 0.0);
        const cd beta = -ph * xnorm;
        for (int i = k; i < n; ++i) v[i] = x[i];
        v[k] -= beta;
        double vn2 = 0.0;
        for (int i = k; i < n; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        const double tau = 2.0 / vn2;
        x[k] = beta;
        for (int i = k + 1; i < n; ++i) x[i] = 0.0;
#pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {
            cd* c = &A[(size_t)j * n];
            cd t = 0.0;
            for (int i = k; i < n; ++i) t += std::conj(v[i]) * c[i];
            t *= tau;
            for (int i = k; i < n; ++i) c[i] -= t * v[i];
        }
    }
    // R^H, row-major: (R^H)[i][j] = conj(R[j][i]) = conj(A[i*n + j]) for j <= i
    std::vector<cd> rh(nn, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) rh[(size_t)i * n + j] = std::conj(A[(size_t)i * n + j]);
    std::vector<cd> UR, VR;
    std::vector<double> sr;
    if (!svd_jacobi(n, rh, UR, sr, VR, err)) return false;
    V.assign(nn, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(size_t)perm[i] * n + j] = UR[(size_t)i * n + j];
    return true;
}

bool svd_jacobi_preconditioned(int n, std::vector<cd>& a, std::vector<cd>& U, std::vector<double>& s,
                               std::vector<cd>& V, std::string* err) {
    std::vector<cd> V0;
    if (!right_vectors_qrp(n, a, V0, err)) return false;
    return svd_jacobi(n, a, U, s, V, err, &V0);
}

// ---------------------------------------------------------------------------
// max_k ||(M - lam_k A) x_k||_inf / ((||M||_inf + |lam_k| ||A||_inf) ||x_k||_inf)
// for real row-major A, M and the columns x_k of a row-major complex X.
// ---------------------------------------------------------------------------
double eig_residual(int n, const double* A, const double* M, const std::vector<cd>& lam,
                    const std::vector<cd>& X) {
    double nA = 0.0, nM = 0.0;
    for (int i = 0; i < n; ++i) {
        double ra = 0.0, rm = 0.0;
        for (int j = 0; j < n; ++j) {
            ra += std::fabs(A[(size_t)i * n + j]);
            rm += std::fabs(M[(size_t)i * n + j]);
        }
        nA = std::max(nA, ra);
        nM = std::max(nM, rm);
    }
    double res = 0.0;
#pragma omp parallel for schedule(dynamic, 8) reduction(max : res)
    for (int k = 0; k < n; ++k) {
        std::vector<cd> x(n);
        for (int j = 0; j < n; ++j) x[j] = X[(size_t)j * n + k];
        double r = 0.0, xn = 0.0;
        for (int i = 0; i < n; ++i) {
            cd s = 0.0;
            for (int j = 0; j < n; ++j) s += (M[(size_t)i * n + j] - lam[k] * A[(size_t)i * n + j]) * x[j];
            r = std::max(r, std::abs(s));
            xn = std::max(xn, std::abs(x[i]));
        }
        res = std::max(res, r / ((nM + std::abs(lam[k]) * nA) * xn));
    }
    return res;
}

void matmul_rowmajor(int m, int k, int n, const double* A, const double* B, double* C) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
        double* c = C + (size_t)i * n;
        for (int j = 0; j < n; ++j) c[j] = 0.0;
        for (int l = 0; l < k; ++l) {
            const double a = A[(size_t)i * k + l];
            const double* b = B + (size_t)l * n;
            for (int j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

}  // namespace stfd
