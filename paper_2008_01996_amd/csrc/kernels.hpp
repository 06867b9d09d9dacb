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
};

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
hipError_t launch_reduce_partials(const double* partial, size_t blocks, int nrhs, double* norms, hipStream_t st);
hipError_t launch_fill_zero(double* p, size_t n, hipStream_t st);

template <typename T>
hipError_t launch_band_init(void* LB, int Mx, int bp, int nsys, const int* rowptr, const int* col,
                            const double* valM, const double* valA, const double* lam, hipStream_t st);
template <typename T>
hipError_t launch_band_ldl(void* LB, int Mx, int bp, int nsys, int* flag, hipStream_t st);
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
template <typename T>
size_t band_ldl_smem(int bp);
template <typename T>
size_t sweep_smem(int bp);

}  // namespace stfd
