/*
 * stfd: space-time Fast Diagonalization solver for the heat equation on one
 * AMD Instinct MI355X (gfx950).
 *
 * Solves the space-time Galerkin system of Langer & Zank (arXiv 2008.01996)
 *
 *     K_h u = F~,   K_h = A_t (x) M_x + M_t (x) A_x            (Sec. 2)
 *
 * with P1 elements in 2D space, piecewise-linear time elements and the
 * modified Hilbert transformation H_T, by the Fast Diagonalization method
 * (Sec. 4.4, Algorithm FD):
 *   1a  generalised eigendecomposition  M_t X = A_t X diag(lambda)
 *   1b  singular value decomposition    X = U_t Sigma V_t^*
 *   2   forward transform  G = F^ A_t^-1 conj(U_t) Sigma^-1 V_t^T
 *   3   independent spatial solves  (M_x + lambda_k A_x) z_k = g_k
 *   4   back transform  u = vec(Z X^T)
 * followed by FP64 iterative refinement on the K_h residual.
 *
 * Conventions
 *   - Every matrix passed as a plain pointer is dense FP64.  Time matrices
 *     (N_t x N_t) are row-major with row = test index l and column = ansatz
 *     index k, as in the definitions of Sec. 2.
 *   - A space-time coefficient block U (or load F~) is M_x x N_t in
 *     column-major order: U[i + M_x k] is the coefficient of psi_i(x) phi_k(t),
 *     so that u = vec(U) as in Sec. 3.1.  Several right-hand sides are stored
 *     one block after the other ([rhs][k][i]).
 *   - Pointers named *_dev are device (HIP) pointers; all others are host.
 *   - hip_stream arguments are hipStream_t values passed as void* (NULL =
 *     the null stream).  Device work is ordered on that stream.
 *   - Return value: STFD_OK (0) or a negative STFD_E* code; the message of
 *     the last error of the calling thread is returned by stfd_last_error().
 *     Nothing aborts the process.  On error, outputs are left unspecified
 *     unless stated otherwise, and handles stay valid.
 *   - The caller owns all buffers it passes; the library owns the opaque
 *     handles and everything they hold until the matching *_free.
 */
#ifndef STFD_H
#define STFD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STFD_OK 0
#define STFD_EINVAL (-1)   /* invalid argument (null pointer, bad size, bad mesh) */
#define STFD_ENOMEM (-2)   /* host or device allocation failed, or size overflow */
#define STFD_EHIP (-3)     /* a HIP runtime call failed */
#define STFD_ENUMERIC (-4) /* A_t not SPD, Re(lambda) <= 0, zero/non-finite pivot, NaN input */
#define STFD_ENOCONV (-5)  /* refinement did not reach rtol within max_refine */
#define STFD_ESTATE (-6)   /* call out of order (e.g. solve before factor) */

#define STFD_PREC_FP64 0   /* every step in (complex) FP64 */
#define STFD_PREC_FP32 1   /* factor, sweeps, second forward and back transform in
                              complex FP32 with FP32 accumulation; residual and
                              update in FP64 */

#define STFD_MAX_HIST 64

/* solution method (stfd_opts.method) */
#define STFD_METHOD_FD 0   /* Fast Diagonalization, Algorithm FD (Sec. 4.4) */
#define STFD_METHOD_BSC 1  /* Bartels-Stewart with the complex Schur form,
                              Algorithm BSc (Sec. 4.3): unitary transforms, the
                              N_t spatial systems solved one after the other;
                              FP64 only */

typedef struct stfd_space stfd_space;
typedef struct stfd_problem stfd_problem;
typedef struct stfd_batch stfd_batch;

typedef struct {
    int precision;        /* STFD_PREC_FP64 or STFD_PREC_FP32 (default FP32) */
    int fp64_transforms;  /* FP32 precision only: bit mask of the transform GEMMs
                             computed with FP64 matrix cores on FP32-stored data:
                             bit 0 = first forward GEMM (F^ A_t^-1 conj(U_t) Sigma^-1),
                             bit 1 = second forward GEMM (x V_t^T),
                             bit 2 = back transform (Z X^T, update of U).
                             Default 5 (first forward GEMM and back transform:
                             their FP32 rounding is amplified by kappa_2(X_t)).
                             With bit 0 set (and always in the FP64 form) the
                             two forward GEMMs are one FP64 GEMM with the
                             product W1 W2 = A_t^-1 conj(U_t) Sigma^-1 V_t^T
                             restricted to the systems (N_t x 2 n_sys, formed
                             once at setup): half the flops of the first GEMM
                             alone, and bit 1 has no effect. */
    double rtol;          /* target ||F~ - K_h u||_2 / ||F~||_2 (default 1e-10) */
    int max_refine;       /* maximum number of refinement corrections (default 30) */
    int method;           /* STFD_METHOD_FD (default) or STFD_METHOD_BSC */
    int inner_refine;     /* FD only, -1 to 3: steps of refinement of the spatial
                             solves inside each application.  With k > 0, G is
                             kept in FP64, solved once by the band factors and
                             then k times on its residual g_k - (M_x + lambda_k
                             A_x) z_k (formed in FP64), the solutions summed in
                             FP64 for an FP64 back transform: in the FP32 form
                             neither G's nor Z's FP32 rounding reaches U, only
                             the factors' error, which each step contracts.  The
                             FP32 form then needs fp64_transforms bits 0 and 2
                             (STFD_EINVAL otherwise).  Costs one pair of sweeps
                             per step and 2 x 8 M_x x 2 n_sys bytes per
                             right-hand side of device memory.  Default -1
                             (automatic): 1 in the FP32 form with the FP64
                             transforms and N_t >= 512 (and 2 in the first
                             application, see inner_refine_first), 0
                             otherwise. */
    int graph;            /* FD only: 1 = the refinement rounds of stfd_fd_solve and
                             stfd_batch_solve run as captured HIP graphs
                             (apply, residual and a device-side convergence check;
                             rounds after convergence do no work), with one host
                             synchronisation per solve as a rule; 0 = launched one
                             by one, one host synchronisation per round.  The
                             graph is built on the first solve with a given
                             (F, U, nrhs) and reused.  Per-stage timing
                             (stfd_profile) runs the rounds one by one.  Default 1. */
    int nrhs_max;         /* > 0: stfd_fd_setup allocates the band factors and the
                             work buffers for this many right-hand sides, so that
                             factor and solve allocate nothing (up to nrhs_max
                             right-hand sides).  Default 0: allocated on first use. */
    int inner_refine_first; /* FD only, -1 to 3: inner_refine for an application to
                             the load itself (the first of a solve, and
                             stfd_fd_apply); the later applications, to a
                             residual, take inner_refine.  -1 (default): the
                             same as inner_refine, or with inner_refine -1 the
                             automatic choice (2 in the FP32 form).  The first application's
                             error is the rough one the FP32 rounding leaves on
                             the whole solution, the later ones' only on a
                             correction, so the first can take more steps. */
} stfd_opts;

typedef struct {
    double min_re_lambda; /* min_k Re(lambda_k) */
    double max_abs_lambda;
    double sigma_min;     /* singular values of X with unit 2-norm columns */
    double sigma_max;
    double kappa2;        /* sigma_max / sigma_min */
    double eig_residual;  /* max_k ||M_t x_k - lambda_k A_t x_k|| / ((||M_t|| + |lambda_k| ||A_t||) ||x_k||) */
    int n_real;           /* real eigenvalues */
    int n_pairs;          /* conjugate pairs */
    int n_sys;            /* spatial systems solved per application: n_real + n_pairs */
    int half_band;        /* half-bandwidth of the spatial matrices */
    double setup_seconds; /* host time of the decomposition and uploads */
    double factor_bytes;  /* device bytes of the stored band factors */
} stfd_setup_report;

typedef struct {
    int iterations;       /* FD applications performed (1 = no correction) */
    int converged;        /* 1 if rel_residual[iterations-1] <= rtol */
    int nrhs;
    double rel_residual[STFD_MAX_HIST]; /* after each application, max over RHS */
    double seconds;       /* wall time of the call, including the final sync */
} stfd_solve_report;

/* Fills *o with the defaults listed above. */
int stfd_opts_default(stfd_opts* o);

/* Message of the last error on this thread ("" if none).  Never NULL. */
const char* stfd_last_error(void);

/* ---------------------------------------------------------------------------
 * Time matrices (Sec. 2): for the hats phi_1..phi_Nt on 0 = t_0 < ... < t_Nt = T
 * and the element indicators chi_l,
 *   Mt[l,k] = <phi_k, H_T phi_l>,  At[l,k] = <phi_k', H_T phi_l>,
 *   Ct[k,l] = <chi_l, H_T phi_k>.
 * t: Nt+1 strictly increasing nodes with t[0] = 0.  At, Mt, Ct: caller-owned
 * Nt*Nt row-major outputs; Ct may be NULL.  Computed from the summed
 * H_T series (a log-tan kernel) with singularity-aware quadrature to about
 * 1e-14 relative accuracy.  Host only; needs no GPU.
 * Errors: STFD_EINVAL (Nt < 1, t not increasing, null output).
 * ------------------------------------------------------------------------- */
int stfd_assemble_time(int Nt, const double* t, double* At, double* Mt, double* Ct);

/* ---------------------------------------------------------------------------
 * Spatial discretisation (Sec. 2): P1 hats psi_i on a triangulation.
 *   xy : 2*nv vertex coordinates (x0, y0, x1, y1, ...)
 *   tri: 3*ntri vertex indices, counter-clockwise
 *   dof: nv interior-node numbers 0..M_x-1, or -1 for Dirichlet vertices;
 *        every number 0..M_x-1 must occur exactly once.
 * Builds M_x[i,j] = <psi_j, psi_i>, A_x[i,j] = <grad psi_j, grad psi_i> and
 * M10[i,j] = <chi_j, psi_i> (the M_{h_x}^{1,0} of Sec. 2) in CSR form, and
 * the half-bandwidth b = max |i-j| over the nonzeros of M_x and A_x.
 * The handle copies everything it needs.  Host only.
 * Errors: STFD_EINVAL (bad indices, clockwise or degenerate triangle),
 *         STFD_ENOMEM.
 * ------------------------------------------------------------------------- */
int stfd_space_create(int nv, const double* xy, int ntri, const int* tri, const int* dof,
                      stfd_space** out);
void stfd_space_free(stfd_space* s);

/* M_x (number of interior nodes), N_x (triangles), half-bandwidth, and the
 * number of nonzeros of M_x (= of A_x; the union pattern).  Any output may
 * be NULL. */
int stfd_space_info(const stfd_space* s, int* Mx, int* Ntri, int* half_band, long long* nnz);

/* CSR export.  which: 0 = M_x, 1 = A_x (both M_x x M_x, nnz entries, shared
 * pattern), 2 = M10 (M_x x N_x, 3 entries per triangle at most).
 * rowptr: rows+1 ints, col/val: nnz entries (query sizes with
 * stfd_space_csr_size).  Host only. */
int stfd_space_csr_size(const stfd_space* s, int which, int* rows, int* cols, long long* nnz);
int stfd_space_export_csr(const stfd_space* s, int which, int* rowptr, int* col, double* val);

/* ---------------------------------------------------------------------------
 * Right-hand side (Sec. 2): f is replaced by its mean on every prism
 * omega_j x (t_{l-1}, t_l), and the load is F~ = M10 F Ct^T.
 *
 * stfd_project_f: F[j + Ntri*l] = mean of f over triangle j x element l for
 *   kind 0: f = sum_q c_q sin(a_q pi xi1) sin(b_q pi xi2) cos(d_q pi t / T)
 *   kind 1: f = sum_q c_q sin(a_q pi xi1) sin(b_q pi xi2) (2t + 2 pi^2 t^2)
 *           (kind 1 with a = b = 1, c = 1 on the unit square is the load of
 *           u = sin(pi x1) sin(pi x2) t^2)
 *   kind 2: the source of the L-shape example of Sec. 5, f = u_t - Laplace u
 *           for u = 5/(2 pi t) exp(-|x - c|^2/(4t)) sin(pi x1 x2),
 *           c = (1/4, -1/4); the mode arguments and box are not read (may be
 *           NULL) and time means use 12-point Gauss-Legendre per element
 * with xi = (x - (xmin, ymin)) / (xmax - xmin, ymax - ymin) and box =
 * {xmin, xmax, ymin, ymax}.  Space means use a 10x10 collapsed Gauss rule per
 * triangle, time means are exact.  F: caller-owned Ntri*Nt, column-major.
 * stfd_assemble_load: Ftilde = M10 F Ct^T, Ftilde caller-owned M_x*Nt
 * column-major; Ct row-major as returned by stfd_assemble_time.  Host only.
 * ------------------------------------------------------------------------- */
int stfd_project_f(const stfd_space* s, int Nt, const double* t, int kind, int nmodes,
                   const int* a, const int* b, const int* d, const double* c,
                   const double* box, double* F);
int stfd_assemble_load(const stfd_space* s, int Nt, const double* Ct, const double* F,
                       double* Ftilde);

/* ---------------------------------------------------------------------------
 * Inhomogeneous Dirichlet data by homogenisation (Sec. 2 remark on Dirichlet
 * data; used by the L-shape example of Sec. 5): the discrete extension
 *   g_h(x, t) = sum over Dirichlet vertices v and k = 1..Nt of
 *               G[v, k] psi_v(x) phi_k(t)
 * (psi_v the P1 hat of vertex v, phi_k the time hats; g(., 0) = 0) is moved
 * to the right-hand side,
 *   Ftilde[i, l] -= sum_{v,k} (At[l,k] Mx[i,v] + Mt[l,k] Ax[i,v]) G[v, k],
 * where Mx[i,v], Ax[i,v] couple interior node i to Dirichlet vertex v.  The
 * discrete solution is then u_h = g_h + sum_{i,k} U[i,k] psi_i phi_k with U
 * the solution for the updated Ftilde.
 *   G     : nv*Nt column-major, G[v + nv*k] = g(x_v, t_{k+1}) (e.g. the
 *           nodal interpolant); entries of interior vertices are not read.
 *   At, Mt: row-major Nt*Nt as returned by stfd_assemble_time.
 *   Ftilde: M_x*Nt column-major, updated in place (caller-owned).
 * Host only.  Errors: STFD_EINVAL (null pointer, Nt < 1).
 * ------------------------------------------------------------------------- */
int stfd_dirichlet_lift(const stfd_space* s, int Nt, const double* At, const double* Mt,
                        const double* G, double* Ftilde);

/* ---------------------------------------------------------------------------
 * Steps 1a/1b of Algorithm FD on the host, for tests and reports.
 * Computes the generalised eigenvalues of (Mt, At) (Cholesky of At, Hessenberg
 * reduction, shifted QR), eigenvectors with unit 2-norm columns arranged as
 * [pairs with Im > 0 | their exact conjugates | real ones], and the singular
 * values of that X (one-sided Jacobi).  Outputs (caller-owned, any may be
 * NULL): lam_re/lam_im (Nt), X_re/X_im (Nt*Nt row-major: X[row*Nt + col],
 * column = eigenvector), sigma (Nt, descending), rep.
 * Errors: STFD_EINVAL, STFD_ENUMERIC (At not SPD, QR did not converge,
 * Re(lambda) <= 0).  Host only.
 * ------------------------------------------------------------------------- */
int stfd_time_decompose(int Nt, const double* At, const double* Mt, double* lam_re,
                        double* lam_im, double* X_re, double* X_im, double* sigma,
                        stfd_setup_report* rep);

/* ---------------------------------------------------------------------------
 * Step 1 of Algorithm BSc (Sec. 4.3) on the host, for tests: the complex
 * Schur form A_t^-1 M_t = W S W^* with W unitary and S upper triangular, the
 * generalised eigenvalues of (Mt, At) on its diagonal (A_t^-1 M_t formed
 * with the Cholesky factor of At, then Householder-Hessenberg reduction and
 * shifted complex QR).  Outputs (caller-owned, Nt*Nt complex each, row-major,
 * re/im interleaved: S[2*(i*Nt + j)] = Re S_ij): S, W.
 * Errors: STFD_EINVAL, STFD_ENUMERIC (At not SPD, QR did not converge).
 * Host only.
 * ------------------------------------------------------------------------- */
int stfd_time_schur(int Nt, const double* At, const double* Mt, double* S, double* W);

/* ---------------------------------------------------------------------------
 * stfd_fd_setup: steps 1a/1b for the pencil (Mt, At) on the host in FP64,
 * plus the transform factors of steps 2 and 4, uploaded to the current HIP
 * device on hip_stream.  Copies At and Mt; space must outlive the problem.
 * opts may be NULL (defaults).  With opts->method = STFD_METHOD_BSC the
 * problem follows Algorithm BSc instead: step 1 is the complex Schur form
 * (as stfd_time_schur), the systems are all N_t diagonal entries of S (no
 * pairing), step 2 is G = F^ A_t^-1 conj(W), step 4 U = Re(Z W^T); the
 * factor, solve and apply entry points below then run that algorithm (FP64
 * precision required, else STFD_EINVAL).
 * Errors: STFD_EINVAL, STFD_ENUMERIC, STFD_ENOMEM, STFD_EHIP.
 * ------------------------------------------------------------------------- */
int stfd_fd_setup(const stfd_space* space, int Nt, const double* At, const double* Mt,
                  const stfd_opts* opts, void* hip_stream, stfd_problem** out);
int stfd_fd_setup_report(const stfd_problem* p, stfd_setup_report* rep);

/* ---------------------------------------------------------------------------
 * Kernel variants of a problem (what the autotuner of the Python package,
 * paper_2008_01996_amd/autotune.py, chooses per shape and writes to its
 * cache; the binding applies a cached choice right after setup).  None of
 * them changes the method, only the kernels that carry out its steps:
 *   sweep_tile_min_rhs  the substitution sweeps of step 3 (Alg. FD) run the
 *                       matrix-core tile kernels, up to 16 right-hand sides
 *                       per workgroup, from this many right-hand sides on;
 *                       0 = never (the lane-chain sweeps for every count).
 *                       Needs a padded half-bandwidth <= 256.  Default 8
 *                       (Algorithm FD; Algorithm BSc always takes the
 *                       lane-chain sweeps, one system at a time).
 *   gemm_tile_m_fp32    rows of the workgroup tile of the transform GEMMs
 *   gemm_tile_m_fp64    (Alg. FD steps 2 and 4) on FP32 and on FP64 matrix
 *                       cores: 64 or 128.
 *   gemm_tile_n_fp64    its columns on FP64 matrix cores: 64, or 128 with
 *                       128 rows (default 128 x 128; the residual GEMM
 *                       always takes the 128 x 128 tile).
 *   gemm_n_fast         1: consecutive workgroups of a GEMM walk along its
 *                       columns (those sharing a panel of the space-time
 *                       block run side by side); 0: along its rows.
 *   factor_kernel       the band LDL^T (step 3 of Alg. FD, first half):
 *                       0 = automatic (register window for FP32 with padded
 *                       half-bandwidth 128, LDS window where it fits, else
 *                       the panel kernel 3 in FP32 and 2 in FP64), 1 =
 *                       trailing tiles streamed with
 *                       the panel factored in LDS, 2 = panel factored in
 *                       registers with the trailing tiles streamed and the
 *                       next panel handed over on chip, 3 = the same with two
 *                       16-column panels per pass, the trailing tiles taking
 *                       both panels' update at once (FP32 only).
 *   factor_pack_real    1 (default): the panel kernel (2, and the automatic
 *                       choice where it takes that kernel) factors the real
 *                       systems of Alg. FD (real lambda, ordered last) two
 *                       to a workgroup in real arithmetic, e.g. 2 p + 2
 *                       systems on 2 p + 1 workgroups; 0: one complex
 *                       workgroup each.  The factors are the same bit for
 *                       bit.  The other kernels ignore it.
 *   sweep_pack_real     1 (default): inside an FD application the tile
 *                       sweeps take Alg. FD's real systems two to a
 *                       workgroup, one in the real and one in the imaginary
 *                       slot of the complex arithmetic (their imaginary
 *                       parts, zero up to the rounding of the forward
 *                       transform, are written as zeros; the back transform
 *                       weighs them with zeros, so U is the same bit for
 *                       bit); 0: one complex workgroup each.
 *                       stfd_spatial_solve always solves every system in
 *                       full.
 * stfd_set_tuning takes effect from the next stfd_fd_factor (the tile
 * sweeps need the inverses of the diagonal blocks, formed by the factor).
 * Errors: STFD_EINVAL (null pointers, a value out of range).  Host only.
 * ------------------------------------------------------------------------- */
typedef struct {
    int sweep_tile_min_rhs;
    int gemm_tile_m_fp32;
    int gemm_tile_m_fp64;
    int gemm_n_fast;
    int factor_kernel;
    int factor_pack_real;
    int gemm_tile_n_fp64;
    int sweep_pack_real;
} stfd_tuning;

int stfd_get_tuning(const stfd_problem* p, stfd_tuning* t);
int stfd_set_tuning(stfd_problem* p, const stfd_tuning* t);

/* ---------------------------------------------------------------------------
 * stfd_fd_factor: step 3, first half.  For every system k (one per
 * conjugate pair, Im(lambda_k) > 0, and one per real eigenvalue) factors
 *     M_x + lambda_k A_x = L_k D_k L_k^T
 * (complex symmetric: transpose, not conjugate transpose; no pivoting) in
 * band form of half-bandwidth b, on the device, in the precision of the
 * options.  Stream-ordered; no host synchronisation.  Calling it again
 * refactors.
 * Errors: STFD_ESTATE (no setup), STFD_ENOMEM, STFD_EHIP.  A zero or
 * non-finite pivot is reported by the next stfd_fd_solve as STFD_ENUMERIC.
 * ------------------------------------------------------------------------- */
int stfd_fd_factor(stfd_problem* p, void* hip_stream);

/* ---------------------------------------------------------------------------
 * stfd_fd_solve: steps 2-4 and FP64 refinement.
 *   F_dev: nrhs loads F~ (device FP64, [rhs][k][i], M_x*Nt each), read only
 *   U_dev: nrhs solutions (device FP64, same layout), overwritten
 * Iterates u <- u + FD(F~ - K_h u) until the relative residual of every RHS
 * is <= rtol or max_refine corrections were made.  Synchronises hip_stream
 * once per iteration to read the residual norms (a few bytes).  rep may be
 * NULL.  Work buffers are allocated on first use and kept for later calls
 * with up to the same nrhs.
 * Errors: STFD_ESTATE (not factored), STFD_EINVAL, STFD_ENUMERIC (zero or
 * non-finite pivot, non-finite residual), STFD_ENOCONV (rtol not reached;
 * U_dev then holds the last iterate), STFD_ENOMEM, STFD_EHIP.
 * ------------------------------------------------------------------------- */
int stfd_fd_solve(stfd_problem* p, int nrhs, const double* F_dev, double* U_dev,
                  stfd_solve_report* rep, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Single stages, for tests and for callers that drive their own iteration.
 *
 * stfd_fd_apply: one application of Algorithm FD without refinement,
 *   U_dev = FD(X_dev), X_dev and U_dev device FP64 [rhs][k][i] blocks
 *   (steps 2-4 of Sec. 4.4 with the precision of the options).
 * stfd_spatial_solve: step 3 alone.  G_dev/Z_dev hold, per RHS, the
 *   column-major M_x x 2 n_sys real matrix [Re g_0 .. Re g_{n-1} | Im g_0 ..
 *   Im g_{n-1}] in the working precision (float for STFD_PREC_FP32, double
 *   otherwise); system k solves (M_x + lambda_k A_x) z_k = g_k with lambda_k
 *   the k-th system eigenvalue (pairs with Im > 0 first, then real ones).
 *   Z_dev may equal G_dev.  Both need stfd_fd_factor first (STFD_ESTATE).
 * stfd_system_lambdas: the n_sys eigenvalues (host, 2 n_sys doubles re/im).
 * ------------------------------------------------------------------------- */
int stfd_fd_apply(stfd_problem* p, int nrhs, const double* X_dev, double* U_dev, void* hip_stream);
int stfd_spatial_solve(stfd_problem* p, int nrhs, const void* G_dev, void* Z_dev, void* hip_stream);
int stfd_system_lambdas(const stfd_problem* p, double* lam);

/* K_h applied on the device: R_dev = F_dev - K_h U_dev for nrhs blocks, and
 * the squared 2-norms of every R and F block in norms[2*nrhs] (host, may be
 * NULL; when given the call synchronises hip_stream).  Used by the solve and
 * exposed for tests (Kronecker identity of Sec. 3.1). */
int stfd_kh_residual(stfd_problem* p, int nrhs, const double* F_dev, const double* U_dev,
                     double* R_dev, double* norms, void* hip_stream);

/* stfd_kh_residual without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same kernels and result as
 * stfd_kh_residual: R_dev = F_dev - K_h U_dev (nrhs M_x x N_t FP64 blocks,
 * [rhs][k][i] as everywhere, device, caller-owned).
 * Its work memory ([M_x U | A_x U] per RHS and the per-workgroup partial
 * sums) is a fixed array of stfd_kh_residual_noalloc_max_bytes() bytes
 * (128 MiB) in device memory, one per GPU, held until the process ends;
 * its device address is looked up on the first call on each device.
 * norms_dev: NULL or 2*nrhs FP64 on the device, receiving (||R||^2, ||F||^2)
 * per RHS; no host synchronisation.  Calls that overlap on one GPU race on
 * the array; each call overwrites what the last one left there.
 * Errors: STFD_EINVAL (null arguments, nrhs < 1, or more work memory than
 * the array holds: (2 M_x N_t nrhs + 2 partials) doubles), STFD_EHIP. */
int stfd_kh_residual_noalloc(stfd_problem* p, int nrhs, const double* F_dev, const double* U_dev,
                             double* R_dev, double* norms_dev, void* hip_stream);
size_t stfd_kh_residual_noalloc_max_bytes(void);

/* ---------------------------------------------------------------------------
 * Per-stage device timing with HIP events recorded on the caller's stream
 * around every kernel launch (the survey of where time goes; off by default).
 * Stages: STFD_ST_BAND_INIT, STFD_ST_BAND_LDL (factor), STFD_ST_FWD1,
 * STFD_ST_FWD2 (forward transforms), STFD_ST_SWEEP_FWD, STFD_ST_SWEEP_BWD,
 * STFD_ST_BACK (back transform and update), STFD_ST_SPATIAL, STFD_ST_RESID,
 * STFD_ST_REDUCE (FP64 residual), STFD_ST_INNER (residual and update of the
 * spatial solves' inner refinement; its sweeps count as sweeps),
 * STFD_ST_BAND_INV (inverses of the factor's diagonal blocks, for the tile
 * sweeps).
 * stfd_profile(p, 1) enables and clears the accumulators, (p, 0) disables.
 * stfd_profile_read waits for the recorded events and returns, per stage, the
 * summed milliseconds and the number of launches since the last clear
 * (ms, counts: STFD_NSTAGE entries each, caller-owned).
 * ------------------------------------------------------------------------- */
#define STFD_NSTAGE 12
#define STFD_ST_BAND_INIT 0
#define STFD_ST_BAND_LDL 1
#define STFD_ST_FWD1 2
#define STFD_ST_FWD2 3
#define STFD_ST_SWEEP_FWD 4
#define STFD_ST_SWEEP_BWD 5
#define STFD_ST_BACK 6
#define STFD_ST_SPATIAL 7
#define STFD_ST_RESID 8
#define STFD_ST_REDUCE 9
#define STFD_ST_INNER 10
#define STFD_ST_BAND_INV 11
int stfd_profile(stfd_problem* p, int enable);
int stfd_profile_read(stfd_problem* p, double* ms, long long* counts);

void stfd_problem_free(stfd_problem* p);

/* ---------------------------------------------------------------------------
 * Batches of independent problems of uneven size (many (M_x, N_t) problems,
 * each with its own right-hand sides), solved by Algorithm FD (Sec. 4.4)
 * with FP64 refinement as in stfd_fd_solve, in lockstep: every refinement
 * round queues one FD application and one residual for every problem that
 * has not converged, then synchronises hip_stream once to read the residual
 * norms of all of them.
 *
 * stfd_batch_create: np problems (each from stfd_fd_setup, distinct, owned
 *   by the caller and kept alive while the batch is used; the batch only
 *   refers to them).  Errors: STFD_EINVAL (np < 1, null or repeated problem),
 *   STFD_ENOMEM.
 * stfd_batch_factor: stfd_fd_factor for every problem, stream-ordered.
 * stfd_batch_solve: nrhs[i] right-hand sides for problem i in F_dev[i]
 *   (device FP64 [rhs][k][i] blocks, read only) -> U_dev[i] (same layout,
 *   overwritten); reps: np reports (may be NULL).  Each problem stops at its
 *   own rtol / max_refine.  Returns STFD_OK when every problem converged,
 *   else the first failure (STFD_ENOCONV, STFD_ENUMERIC, ...); the reports
 *   say which problem did what.  Errors also: STFD_ESTATE (a problem not
 *   factored), STFD_EINVAL, STFD_ENOMEM, STFD_EHIP.
 * stfd_batch_free: frees the batch only, not the problems.
 * ------------------------------------------------------------------------- */
int stfd_batch_create(int np, stfd_problem* const* problems, stfd_batch** out);
int stfd_batch_factor(stfd_batch* b, void* hip_stream);
int stfd_batch_solve(stfd_batch* b, const int* nrhs, const double* const* F_dev, double* const* U_dev,
                     stfd_solve_report* reps, void* hip_stream);
void stfd_batch_free(stfd_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* STFD_H */
