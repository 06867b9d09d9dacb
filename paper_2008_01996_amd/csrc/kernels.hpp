// Launch interface of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace stfd {

enum { EPI_STORE_F32 = 0, EPI_STORE_F64 = 1, EPI_ADD_F64 = 2, EPI_RESID = 3 };

// C (M x N, col-major, ldc) = A (M x K, col-major, lda) * B (K x N, row-major,
// ldb), batched over blockIdx.z with strides strideA / strideC (elements).
// EPI_ADD_F64: C += alpha * A B.  EPI_RESID: C = F - A B (F with the layout of
// C and batch stride strideF), and per-workgroup sums of squares of C and F
// into partial[2 * (batch * blocks + block)].
struct GemmArgs {
    const void* A;
    const void* B;
    void* C;
    const void* F;
    double* partial;
    int M, N, K;
    long long lda, ldb, ldc;
    long long strideA, strideC, strideF;
    int batch;
    double alpha;
    const int* gate;    // launch_gate() at launch: the kernel returns at once while *gate != 0
    int bm;             // workgroup tile: 64 x 64, 128 x 64, or 0: 128 x 128 (FP64 matrix cores only;
                        // the residual always takes the 128 x 128 tile)
    int nfast;          // 1: consecutive workgroups run along N (share an A panel)
};

// Gate of the kernels of a refinement round.  While a device flag is set as
// the gate on the calling host thread, every launcher below passes it to its
// kernel, which returns at once when the flag is nonzero: replays of a
// captured round after the solve has converged do no work.
void set_launch_gate(const int* gate);
const int* launch_gate();

// one refinement round ends with this check: norms (2 nrhs: ||R||^2, ||F||^2)
// give the relative residual (max over the right-hand sides); ctl[0] = done,
// ctl[1] = applications so far, ctl[2] = status (0 running, 1 converged,
// 2 zero or non-finite pivot, 3 out of applications, 4 non-finite
// residual); hist[a] = the
// residual after application a.  Gated on ctl[0] itself.
hipError_t launch_refine_check(const double* norms, int nrhs, double rtol, const int* pivot_flag, int max_apps,
                               int* ctl, double* hist, hipStream_t st);
// ctl[0..2] = 0, *flag = 0 (no memset nodes in captured graphs)
hipError_t launch_reset_ints(int* p, int n, hipStream_t st);

enum GemmKind {
    GEMM_D_D_STORE_D,   // FP64 in, FP64 MFMA, FP64 out
    GEMM_D_D_STORE_F,   // FP64 in, FP64 MFMA, FP32 out
    GEMM_D_F_STORE_F,   // FP64 A rounded to FP32, FP32 MFMA, FP32 out
    GEMM_F_F_STORE_F,   // FP32 in/out
    GEMM_F_F_ADD_D,     // FP32 MFMA, FP64 accumulate into C
    GEMM_D_D_ADD_D,     // FP64 MFMA, FP64 accumulate into C
    GEMM_D_D_RESID,     // FP64 residual
    GEMM_F_D_STORE_F,   // FP32 A widened to FP64, FP64 B, FP64 MFMA, FP32 out
    GEMM_F_D_ADD_D,     // FP32 A widened to FP64, FP64 B, FP64 MFMA, FP64 accumulate into C
};

hipError_t launch_gemm(GemmKind kind, const GemmArgs& g, hipStream_t st);
size_t gemm_resid_partials(int M, int N, int batch);

hipError_t launch_spatial_apply(int Mx, int Nt, int nrhs, const int* rowptr, const int* col, const double* valM,
                                const double* valA, const double* U, double* P, hipStream_t st);
// R = G - (M_x + lambda_k A_x) Z for every system and right-hand side (FP64
// G and Z, FP64 arithmetic, R in TR)
template <typename TR>
hipError_t launch_spatial_resid(int Mx, int nsys, int nrhs, const int* rowptr, const int* col, const double* valM,
                                const double* valA, const double* lam, const double* G, const double* Z, void* R,
                                hipStream_t st);
// y = x (ACC false) or y += x (ACC true), n elements, x converted to TY
template <typename TY, typename TX, bool ACC>
hipError_t launch_convert(void* y, const void* x, size_t n, hipStream_t st);
hipError_t launch_reduce_partials(const double* partial, size_t blocks, int nrhs, double* norms, hipStream_t st);
hipError_t launch_fill_zero(double* p, size_t n, hipStream_t st);

template <typename T>
hipError_t launch_band_init(void* LB, int Mx, int bp, int nsys, const int* rowptr, const int* col,
                            const double* valM, const double* valA, const double* lam, hipStream_t st);
// factor kernel: automatic (the register window for FP32 with padded band
// 128, the LDS window where it fits, else the panel kernel: two panels per
// pass in FP32, one in FP64), or forced.  The
// last nreal systems are real (every imaginary part zero): the panel kernel
// factors them two to a workgroup in real arithmetic.
enum { FACTOR_AUTO = 0, FACTOR_STREAM = 1, FACTOR_PANEL = 2, FACTOR_PANEL2 = 3 };
template <typename T>
hipError_t launch_band_ldl(void* LB, int Mx, int bp, int nsys, int nreal, const int* reach, int* flag, int kernel,
                           hipStream_t st);
// sweeps of systems sys0 .. sys0 + nrun - 1 of the nsys (G, W laid out for all nsys)
template <typename T>
hipError_t launch_band_forward(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                               hipStream_t st, int sys0, int nrun);
template <typename T>
hipError_t launch_band_backward(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st,
                                int sys0, int nrun);
// Bartels-Stewart coupling after system k is solved (G [rhs][2 nsys][Mx], z_k
// in columns k and nsys + k): v = A_x z_k, then g_i -= S[i][k] v for i < k
// (S row-major nsys x nsys, complex interleaved)
hipError_t launch_bs_update(int Mx, int nsys, int nrhs, int k, const int* rowptr, const int* col,
                            const double* valA, const double* S, double* G, hipStream_t st);
// Tile sweeps (kernels_tile.hip): up to 16 right-hand sides per workgroup on
// the matrix cores, with the inverses of the 16 x 16 diagonal blocks of L
// (LI: n_sys x ceil(M_x / 16) blocks of 16 x 16, column-major).
constexpr int TILE_BPMAX = 256;
// the largest padded half-bandwidth any sweep kernel takes
constexpr int BAND_BPMAX = 256;
template <typename T>
hipError_t launch_band_diag_inverse(const void* LB, void* LI, int Mx, int bp, int nsys, hipStream_t st);
template <typename T>
// reach[b]: 16-row blocks below diagonal block b that the factor's columns
// reach (the envelope; blocks beyond are zero and skipped)
hipError_t launch_tile_forward(const void* LB, const void* LI, const int* reach, int Mx, int bp, int nsys, int nrhs,
                               const void* G, void* W, hipStream_t st, int sys0, int nrun, int nreal);
template <typename T>
hipError_t launch_tile_backward(const void* LB, const void* LI, const int* reach, int Mx, int bp, int nsys, int nrhs,
                                void* W, hipStream_t st, int sys0, int nrun, int nreal);
template <typename T>
size_t band_ldl_smem(int bp);
template <typename T>
size_t sweep_smem(int bp);

}  // namespace stfd
