// P1 spatial matrices, the piecewise-constant projection of f and the load
// F~ = M10 F C_t^T (Sec. 2).  Host only.
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <thread>

#include "host_internal.hpp"

namespace stfd {

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

}  // namespace stfd

using stfd::fail;

extern "C" const char* stfd_last_error(void) { return stfd::last_error(); }

extern "C" int stfd_opts_default(stfd_opts* o) {
    if (!o) return fail(STFD_EINVAL, "null opts");
    o->precision = STFD_PREC_FP32;
    o->fp64_transforms = 5;
    o->rtol = 1e-10;
    o->max_refine = 30;
    o->method = STFD_METHOD_FD;
    o->inner_refine = -1;
    o->graph = 1;
    o->nrhs_max = 0;
    o->inner_refine_first = -1;
    return STFD_OK;
}

extern "C" int stfd_assemble_time(int Nt, const double* t, double* At, double* Mt, double* Ct) {
    if (Nt < 1 || !t || !At || !Mt) return fail(STFD_EINVAL, "assemble_time: bad arguments");
    if (t[0] != 0.0) return fail(STFD_EINVAL, "assemble_time: t[0] must be 0");
    for (int i = 0; i < Nt; ++i)
        if (!(t[i + 1] > t[i]) || !std::isfinite(t[i + 1]))
            return fail(STFD_EINVAL, "assemble_time: nodes must be finite and strictly increasing");
    stfd::clear_error();
    return stfd::assemble_time_impl(Nt, t, At, Mt, Ct);
}

extern "C" int stfd_space_create(int nv, const double* xy, int ntri, const int* tri, const int* dof,
                                 stfd_space** out) {
    if (!out || nv < 3 || ntri < 1 || !xy || !tri || !dof) return fail(STFD_EINVAL, "space_create: bad arguments");
    *out = nullptr;
    auto* s = new (std::nothrow) stfd_space();
    if (!s) return fail(STFD_ENOMEM, "space_create: out of memory");
    s->nv = nv;
    s->ntri = ntri;
    s->xy.assign(xy, xy + 2 * (size_t)nv);
    s->tri.assign(tri, tri + 3 * (size_t)ntri);
    s->dof.assign(dof, dof + nv);
    int Mx = 0;
    for (int v = 0; v < nv; ++v) Mx = std::max(Mx, dof[v] + 1);
    std::vector<int> seen(Mx, 0);
    for (int v = 0; v < nv; ++v) {
        if (dof[v] < -1) { delete s; return fail(STFD_EINVAL, "space_create: dof < -1"); }
        if (dof[v] >= 0) seen[dof[v]]++;
    }
    for (int i = 0; i < Mx; ++i)
        if (seen[i] != 1) { delete s; return fail(STFD_EINVAL, "space_create: dof numbers must be 0..Mx-1, once each"); }
    if (Mx == 0) { delete s; return fail(STFD_EINVAL, "space_create: no interior nodes"); }
    s->Mx = Mx;
    s->area.resize(ntri);
    // element matrices: mass |T|/12 (1 + delta), stiffness |T| grad l_a . grad l_b
    std::vector<std::map<int, std::pair<double, double>>> rows(Mx);
    std::vector<std::map<int, double>> rows10(Mx);
    std::vector<std::map<int, std::pair<double, double>>> rowsB(Mx);
    for (int e = 0; e < ntri; ++e) {
        int v[3];
        for (int a = 0; a < 3; ++a) {
            v[a] = tri[3 * (size_t)e + a];
            if (v[a] < 0 || v[a] >= nv) { delete s; return fail(STFD_EINVAL, "space_create: vertex index out of range"); }
        }
        const double x0 = xy[2 * v[0]], y0 = xy[2 * v[0] + 1];
        const double x1 = xy[2 * v[1]], y1 = xy[2 * v[1] + 1];
        const double x2 = xy[2 * v[2]], y2 = xy[2 * v[2] + 1];
        const double det = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0);
        if (!(det > 0.0)) { delete s; return fail(STFD_EINVAL, "space_create: triangle not counter-clockwise or degenerate"); }
        const double area = 0.5 * det;
        s->area[e] = area;
        // grad lambda_a = perp(opposite edge) / det
        const double gx[3] = {-(y2 - y1) / det, -(y0 - y2) / det, -(y1 - y0) / det};
        const double gy[3] = {(x2 - x1) / det, (x0 - x2) / det, (x1 - x0) / det};
        for (int a = 0; a < 3; ++a) {
            const int i = dof[v[a]];
            if (i < 0) continue;
            rows10[i][e] += area / 3.0;
            for (int b = 0; b < 3; ++b) {
                const int j = dof[v[b]];
                auto& ent = j < 0 ? rowsB[i][v[b]] : rows[i][j];
                ent.first += area / 12.0 * (a == b ? 2.0 : 1.0);
                ent.second += area * (gx[a] * gx[b] + gy[a] * gy[b]);
            }
        }
    }
    s->rowptr.assign(Mx + 1, 0);
    s->rowptr10.assign(Mx + 1, 0);
    int hb = 0;
    for (int i = 0; i < Mx; ++i) {
        s->rowptr[i + 1] = s->rowptr[i] + (int)rows[i].size();
        s->rowptr10[i + 1] = s->rowptr10[i] + (int)rows10[i].size();
        for (auto& kv : rows[i]) {
            s->col.push_back(kv.first);
            s->valM.push_back(kv.second.first);
            s->valA.push_back(kv.second.second);
            hb = std::max(hb, std::abs(kv.first - i));
        }
        for (auto& kv : rows10[i]) {
            s->col10.push_back(kv.first);
            s->val10.push_back(kv.second);
        }
    }
    s->half_band = hb;
    {
        // the fill of column c stays above the last row any column k <= c
        // reaches: reach(c) = max_{k <= c} (last row of column k)
        const int nblk = (Mx + 15) / 16;
        s->block_reach.assign(nblk, 0);
        int last = -1;
        for (int i = 0; i < Mx; ++i) {
            for (int e = s->rowptr[i]; e < s->rowptr[i + 1]; ++e) last = std::max(last, s->col[e]);
            last = std::max(last, i);
            const int b = i / 16, lastblk = std::min(last, Mx - 1) / 16;
            s->block_reach[b] = std::max(s->block_reach[b], lastblk - b);
        }
    }
    s->rowptrB.assign(Mx + 1, 0);
    for (int i = 0; i < Mx; ++i) {
        s->rowptrB[i + 1] = s->rowptrB[i] + (int)rowsB[i].size();
        for (auto& kv : rowsB[i]) {
            s->colB.push_back(kv.first);
            s->valMB.push_back(kv.second.first);
            s->valAB.push_back(kv.second.second);
        }
    }
    *out = s;
    stfd::clear_error();
    return STFD_OK;
}

extern "C" void stfd_space_free(stfd_space* s) { delete s; }

extern "C" int stfd_space_info(const stfd_space* s, int* Mx, int* Ntri, int* half_band, long long* nnz) {
    if (!s) return fail(STFD_EINVAL, "space_info: null space");
    if (Mx) *Mx = s->Mx;
    if (Ntri) *Ntri = s->ntri;
    if (half_band) *half_band = s->half_band;
    if (nnz) *nnz = (long long)s->col.size();
    return STFD_OK;
}

extern "C" int stfd_space_csr_size(const stfd_space* s, int which, int* rows, int* cols, long long* nnz) {
    if (!s || which < 0 || which > 2) return fail(STFD_EINVAL, "space_csr_size: bad arguments");
    if (rows) *rows = s->Mx;
    if (cols) *cols = which == 2 ? s->ntri : s->Mx;
    if (nnz) *nnz = (long long)(which == 2 ? s->col10.size() : s->col.size());
    return STFD_OK;
}

extern "C" int stfd_space_export_csr(const stfd_space* s, int which, int* rowptr, int* col, double* val) {
    if (!s || which < 0 || which > 2 || !rowptr || !col || !val)
        return fail(STFD_EINVAL, "space_export_csr: bad arguments");
    const auto& rp = which == 2 ? s->rowptr10 : s->rowptr;
    const auto& cl = which == 2 ? s->col10 : s->col;
    const auto& vl = which == 0 ? s->valM : which == 1 ? s->valA : s->val10;
    std::copy(rp.begin(), rp.end(), rowptr);
    std::copy(cl.begin(), cl.end(), col);
    std::copy(vl.begin(), vl.end(), val);
    return STFD_OK;
}

namespace {

constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre on [0,1] (Newton on the three-term recurrence)
void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 + z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

// Source of the L-shape example of Sec. 5: u = G sin(pi x1 x2) with
// G = 5/(2 pi t) exp(-|x - c|^2/(4t)), c = (1/4, -1/4), and G_t = Laplace G
// (ten times the heat kernel), so f = u_t - Laplace u = -2 grad G . grad s
// - G Laplace s = G [pi cos(pi x1 x2) ((x1 - c1) x2 + (x2 - c2) x1) / t
// + pi^2 (x1^2 + x2^2) sin(pi x1 x2)].
static inline double lshape_source(double x1, double x2, double t) {
    const double c1 = 0.25, c2 = -0.25;
    const double r2 = (x1 - c1) * (x1 - c1) + (x2 - c2) * (x2 - c2);
    const double G = 5.0 / (2.0 * kPi * t) * std::exp(-r2 / (4.0 * t));
    const double sn = std::sin(kPi * x1 * x2), cs = std::cos(kPi * x1 * x2);
    return G * (kPi * cs * ((x1 - c1) * x2 + (x2 - c2) * x1) / t + kPi * kPi * (x1 * x1 + x2 * x2) * sn);
}

// Prism means of the Sec. 5 source: the 10 x 10 collapsed triangle rule
// times 12-point Gauss-Legendre on every time element.
static void project_lshape_source(const stfd_space* s, int Nt, const double* t, double* F) {
    const int n = 10, nt = 12;
    std::vector<double> gx, gw, tx, tw;
    gauss01(n, gx, gw);
    gauss01(nt, tx, tw);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < s->ntri; ++e) {
        const int* v = &s->tri[3 * (size_t)e];
        const double p0x = s->xy[2 * v[0]], p0y = s->xy[2 * v[0] + 1];
        const double p1x = s->xy[2 * v[1]], p1y = s->xy[2 * v[1] + 1];
        const double p2x = s->xy[2 * v[2]], p2y = s->xy[2 * v[2] + 1];
        double px[100], py[100], pw[100];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double u = gx[i], vv = gx[j];
                px[i * n + j] = p2x + u * (p0x - p2x) + u * vv * (p1x - p0x);
                py[i * n + j] = p2y + u * (p0y - p2y) + u * vv * (p1y - p0y);
                pw[i * n + j] = gw[i] * gw[j] * 2.0 * u;
            }
        for (int l = 0; l < Nt; ++l) {
            const double t0 = t[l], h = t[l + 1] - t[l];
            double acc = 0.0;
            for (int k = 0; k < nt; ++k) {
                const double tk = t0 + tx[k] * h;
                double sk = 0.0;
                for (int q = 0; q < n * n; ++q) sk += pw[q] * lshape_source(px[q], py[q], tk);
                acc += tw[k] * sk;
            }
            F[(size_t)l * s->ntri + e] = acc;
        }
    }
}

extern "C" int stfd_project_f(const stfd_space* s, int Nt, const double* t, int kind, int nmodes, const int* a,
                              const int* b, const int* d, const double* c, const double* box, double* F) {
    if (!s || Nt < 1 || !t || !F || kind < 0 || kind > 2)
        return fail(STFD_EINVAL, "project_f: bad arguments");
    if (kind != 2 && (nmodes < 1 || !a || !b || !c || !box || (kind == 0 && !d)))
        return fail(STFD_EINVAL, "project_f: bad arguments");
    for (int l = 0; l < Nt; ++l)
        if (!(t[l + 1] > t[l])) return fail(STFD_EINVAL, "project_f: t must increase");
    if (kind == 2) {
        if (!(t[0] >= 0.0)) return fail(STFD_EINVAL, "project_f: kind 2 needs t[0] >= 0");
        project_lshape_source(s, Nt, t, F);
        return STFD_OK;
    }
    const double T = t[Nt];
    const double bx = box[1] - box[0], by = box[3] - box[2];
    if (!(bx > 0) || !(by > 0)) return fail(STFD_EINVAL, "project_f: empty box");
    // collapsed Gauss rule on the triangle, collapsed towards vertex 2:
    // point = p2 + u (p0 - p2) + u v (p1 - p0), Jacobian 2|T| u
    const int n = 10;
    std::vector<double> gx, gw;
    gauss01(n, gx, gw);
    std::vector<double> sx((size_t)s->ntri * nmodes);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < s->ntri; ++e) {
        const int* v = &s->tri[3 * (size_t)e];
        const double p0x = s->xy[2 * v[0]], p0y = s->xy[2 * v[0] + 1];
        const double p1x = s->xy[2 * v[1]], p1y = s->xy[2 * v[1] + 1];
        const double p2x = s->xy[2 * v[2]], p2y = s->xy[2 * v[2] + 1];
        for (int q = 0; q < nmodes; ++q) {
            double acc = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const double u = gx[i], vv = gx[j];
                    const double px = p2x + u * (p0x - p2x) + u * vv * (p1x - p0x);
                    const double py = p2y + u * (p0y - p2y) + u * vv * (p1y - p0y);
                    const double xi1 = (px - box[0]) / bx, xi2 = (py - box[2]) / by;
                    acc += gw[i] * gw[j] * 2.0 * u * std::sin(a[q] * kPi * xi1) * std::sin(b[q] * kPi * xi2);
                }
            sx[(size_t)e * nmodes + q] = acc;     // mean over the triangle
        }
    }
#pragma omp parallel for schedule(static)
    for (int l = 0; l < Nt; ++l) {
        const double t0 = t[l], t1 = t[l + 1], h = t1 - t0;
        for (int q = 0; q < nmodes; ++q) {
            double st;
            if (kind == 1) {
                // mean of 2t + 2 pi^2 t^2: (t^2 + 2 pi^2 t^3 / 3) differences
                auto G = [](double x) { return x * x + 2.0 * kPi * kPi * x * x * x / 3.0; };
                st = (G(t1) - G(t0)) / h;
            } else if (d[q] == 0) {
                st = 1.0;
            } else {
                const double w = d[q] * kPi / T;
                st = (std::sin(w * t1) - std::sin(w * t0)) / (w * h);
            }
            const double cs = c[q] * st;
            for (int e = 0; e < s->ntri; ++e) {
                double& out = F[(size_t)l * s->ntri + e];
                if (q == 0) out = 0.0;
                out += cs * sx[(size_t)e * nmodes + q];
            }
        }
    }
    return STFD_OK;
}

extern "C" int stfd_assemble_load(const stfd_space* s, int Nt, const double* Ct, const double* F, double* Ft) {
    if (!s || Nt < 1 || !Ct || !F || !Ft) return fail(STFD_EINVAL, "assemble_load: bad arguments");
    const int Mx = s->Mx, nt = s->ntri;
    // G = M10 F (Mx x Nt), one time interval per task
    std::vector<double> G((size_t)Mx * Nt, 0.0);
#pragma omp parallel for schedule(static)
    for (int l = 0; l < Nt; ++l)
        for (int i = 0; i < Mx; ++i) {
            double acc = 0.0;
            for (int e = s->rowptr10[i]; e < s->rowptr10[i + 1]; ++e)
                acc += s->val10[e] * F[(size_t)l * nt + s->col10[e]];
            G[(size_t)l * Mx + i] = acc;
        }
    // Ft = G Ct^T in blocks of rows (a block of G stays in cache over k),
    // KB columns of Ft at a time (each G entry loaded once for KB products)
    constexpr int RB = 128, KB = 8;
    const int nblk = (Mx + RB - 1) / RB;
#pragma omp parallel for schedule(static)
    for (int bi = 0; bi < nblk; ++bi) {
        const int i0 = bi * RB, nr = std::min(Mx, i0 + RB) - i0;
        double acc[KB][RB];
        for (int k0 = 0; k0 < Nt; k0 += KB) {
            const int nk = std::min(KB, Nt - k0);
            for (int j = 0; j < KB; ++j)
                for (int i = 0; i < RB; ++i) acc[j][i] = 0.0;
            for (int l = 0; l < Nt; ++l) {
                double c[KB];
                for (int j = 0; j < KB; ++j) c[j] = j < nk ? Ct[(size_t)(k0 + j) * Nt + l] : 0.0;
                const double* g = &G[(size_t)l * Mx + i0];
                for (int i = 0; i < nr; ++i) {
                    const double gi = g[i];
                    for (int j = 0; j < KB; ++j) acc[j][i] += c[j] * gi;
                }
            }
            for (int j = 0; j < nk; ++j) {
                double* out = Ft + (size_t)(k0 + j) * Mx + i0;
                for (int i = 0; i < nr; ++i) out[i] = acc[j][i];
            }
        }
    }
    return STFD_OK;
}

extern "C" int stfd_dirichlet_lift(const stfd_space* s, int Nt, const double* At, const double* Mt,
                                   const double* G, double* Ft) {
    if (!s || Nt < 1 || !At || !Mt || !G || !Ft) return fail(STFD_EINVAL, "dirichlet_lift: bad arguments");
    const int Mx = s->Mx, nv = s->nv;
    // only rows next to the boundary couple to it: P = M_B G, Q = A_B G on
    // those rows, then Ft[i, l] -= sum_k P[i, k] At[l, k] + Q[i, k] Mt[l, k]
    std::vector<int> brow;
    for (int i = 0; i < Mx; ++i)
        if (s->rowptrB[i + 1] > s->rowptrB[i]) brow.push_back(i);
    const int nb = (int)brow.size();
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nb; ++r) {
        const int i = brow[r];
        std::vector<double> P(Nt, 0.0), Q(Nt, 0.0);
        for (int e = s->rowptrB[i]; e < s->rowptrB[i + 1]; ++e) {
            const int v = s->colB[e];
            for (int k = 0; k < Nt; ++k) {
                const double g = G[(size_t)k * nv + v];
                P[k] += s->valMB[e] * g;
                Q[k] += s->valAB[e] * g;
            }
        }
        for (int l = 0; l < Nt; ++l) {
            double acc = 0.0;
            for (int k = 0; k < Nt; ++k)
                acc += P[k] * At[(size_t)l * Nt + k] + Q[k] * Mt[(size_t)l * Nt + k];
            Ft[(size_t)l * Mx + i] -= acc;
        }
    }
    stfd::clear_error();
    return STFD_OK;
}
