// Batched complex-symmetric band LDL^T factorization (step 3 of Algorithm FD,
// Sec. 4.4, first half):
//     M_x + lambda_k A_x = L_k D_k L_k^T
// for all systems k at once (one workgroup per system); the sweeps that use
// the factors are in kernels_sweep.hip.  The spatial matrices
// are symmetric with half-bandwidth b, so L_k is unit lower triangular with
// the same bandwidth (no pivoting: the systems are complex symmetric with
// Re(lambda_k) > 0, Sec. 4.4 and 4.1).
//
// Band storage (column-oriented, complex interleaved, padded width bp >= b,
// bp a multiple of 16):
//     LB[k][c][0]   = D_k[c]
//     LB[k][c][d]   = L_k[c + d, c],  d = 1..bp   (zero outside the matrix)
// so the bp+1 entries of a column, and the 16 columns of a panel, are
// contiguous in memory.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace stfd {

// ---------------------------------------------------------------------------
// Band initialisation: LB[k][c][d] = M_x[c+d, c] + lambda_k A_x[c+d, c].  The
// matrices are symmetric, so column c below the diagonal is row c right of the
// diagonal in CSR form.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) band_init_kernel(cplx<T>* __restrict__ LB, int Mx, int bp,
                                                        const int* __restrict__ rowptr,
                                                        const int* __restrict__ col,
                                                        const double* __restrict__ valM,
                                                        const double* __restrict__ valA,
                                                        const double* __restrict__ lam) {
    constexpr int COLS = 8;
    const int bp1 = bp + 1;
    const int sys = blockIdx.y;
    const int c0 = blockIdx.x * COLS;
    const int ncols = min(COLS, Mx - c0);
    cplx<T>* base = LB + ((size_t)sys * Mx + c0) * bp1;
    for (int e = threadIdx.x; e < ncols * bp1; e += blockDim.x) base[e] = cplx<T>{T(0), T(0)};
    __syncthreads();
    const double lr = lam[2 * sys], li = lam[2 * sys + 1];
    for (int q = threadIdx.x; q < ncols * 32; q += blockDim.x) {
        const int cl = q / 32, slot = q % 32;
        const int c = c0 + cl;
        for (int e = rowptr[c] + slot; e < rowptr[c + 1]; e += 32) {
            const int j = col[e];
            const int d = j - c;
            if (d >= 0 && d <= bp) {
                const double m = valM[e], a = valA[e];
                base[(size_t)cl * bp1 + d] = cplx<T>{T(m + lr * a), T(li * a)};
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Right-looking blocked band LDL^T, panels of 16 columns, one workgroup
// (4 waves) per system.
//   1. the panel (16 columns x (bp+1) entries) is loaded into LDS and factored
//      column by column (divide by the pivot, rank-1 update of the later panel
//      columns);
//   2. the trailing bp x bp triangle is updated by the panel,
//          C[r, c'] -= sum_k L[r, k] D[k] L[c', k],
//      in 16x16 tiles on the matrix cores: each complex tile product is four
//      real 16x16x16 products (16x16x4 MFMA instructions).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) band_ldl_kernel(cplx<T>* __restrict__ LB, int Mx, int bp,
                                                       int* __restrict__ flag) {
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    T* PR = reinterpret_cast<T*>(smem_raw);        // [16][bp1] real parts
    T* PI = PR + 16 * bp1;                         // [16][bp1] imaginary parts
    __shared__ T DR[16], DI[16];
    const int sys = blockIdx.x;
    cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int ntile = bp / 16;
    const int tiles_total = ntile * (ntile + 1) / 2;

    for (int p0 = 0; p0 < Mx; p0 += 16) {
        const int nb = min(16, Mx - p0);
        // ---- load panel
        const cplx<T>* src = base + (size_t)p0 * bp1;
        for (int e = tid; e < 16 * bp1; e += blockDim.x) {
            cplx<T> v = (e < nb * bp1) ? src[e] : cplx<T>{T(0), T(0)};
            PR[e] = v.re;
            PI[e] = v.im;
        }
        __syncthreads();
        // ---- factor panel
        for (int k = 0; k < nb; ++k) {
            const cplx<T> dk = {PR[k * bp1], PI[k * bp1]};
            const cplx<T> inv = cinv(dk);
            if (tid == 0) {
                DR[k] = dk.re;
                DI[k] = dk.im;
                const T mag = fabs(dk.re) + fabs(dk.im);
                if (!(mag > T(0)) || !isfinite(mag)) atomicOr(flag, 1);
            }
            for (int d = 1 + tid; d <= bp; d += blockDim.x) {
                const cplx<T> v = cmul(cplx<T>{PR[k * bp1 + d], PI[k * bp1 + d]}, inv);
                PR[k * bp1 + d] = v.re;
                PI[k * bp1 + d] = v.im;
            }
            __syncthreads();
            // later panel columns k2 > k: A[k2 + d2, k2] -= L[k2+d2, k] D_k L[k2, k];
            // lane bits 0-3 pick the column, the rest stride down the rows
            {
                const int k2 = k + 1 + (tid & 15);
                if (k2 < nb) {
                    const int off = k2 - k;              // row offset of k2 from column k
                    const cplx<T> dl = cmul(dk, cplx<T>{PR[k * bp1 + off], PI[k * bp1 + off]});
                    for (int d2 = tid >> 4; d2 + off <= bp; d2 += 16) {
                        const cplx<T> t = cmul(cplx<T>{PR[k * bp1 + off + d2], PI[k * bp1 + off + d2]}, dl);
                        PR[k2 * bp1 + d2] -= t.re;
                        PI[k2 * bp1 + d2] -= t.im;
                    }
                }
            }
            __syncthreads();
        }
        // ---- write the finished panel (L columns and D)
        cplx<T>* dst = base + (size_t)p0 * bp1;
        for (int e = tid; e < nb * bp1; e += blockDim.x) dst[e] = cplx<T>{PR[e], PI[e]};
        // ---- trailing update on the matrix cores
        // tile (ti, tj), ti >= tj: rows r0 = p0 + 16 + 16 ti, columns c0 = p0 + 16 + 16 tj.
        // Each wave takes every 4th tile, CH tiles at a time: all their global
        // loads are issued before the first MFMA so the latency is paid once
        // per chunk.
        constexpr int CH = 8;
        const int li = lane & 15, lk = lane >> 4;
        for (int tbase = wave; tbase < tiles_total; tbase += 4 * CH) {
            cplx<T> cv[CH][4];
            int rr0[CH], cc0[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int t = tbase + 4 * u;
                rr0[u] = Mx;
                cc0[u] = Mx;
                if (t < tiles_total) {
                    int ti = 0;
                    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
                    const int tj = t - ti * (ti + 1) / 2;
                    rr0[u] = p0 + 16 + 16 * ti;
                    cc0[u] = p0 + 16 + 16 * tj;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = rr0[u] + li, c = cc0[u] + mfma_row<T>(lk, j);
                    const int d = r - c;
                    cv[u][j] = cplx<T>{T(0), T(0)};
                    if (r < Mx && c < Mx && d >= 0 && d <= bp) cv[u][j] = base[(size_t)c * bp1 + d];
                }
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                if (cc0[u] >= Mx || rr0[u] >= Mx) continue;
                typename vec4<T>::type accR = zero4<T>(), accI = zero4<T>();
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    // A operand: L[c', k] with c' = c0 + li; B operand: L[r, k] D[k], r = r0 + li
                    T ar = 0, ai = 0, br = 0, bi = 0;
                    if (k < nb) {
                        const int oc = cc0[u] + li - p0 - k;
                        if (oc >= 1 && oc <= bp) {
                            ar = PR[k * bp1 + oc];
                            ai = PI[k * bp1 + oc];
                        }
                        const int orr = rr0[u] + li - p0 - k;
                        if (orr >= 1 && orr <= bp) {
                            const cplx<T> l = {PR[k * bp1 + orr], PI[k * bp1 + orr]};
                            const cplx<T> ld = cmul(l, cplx<T>{DR[k], DI[k]});
                            br = ld.re;
                            bi = ld.im;
                        }
                    }
                    accR = mfma16x16x4<T>(ar, br, accR);
                    accR = mfma16x16x4<T>(-ai, bi, accR);
                    accI = mfma16x16x4<T>(ar, bi, accI);
                    accI = mfma16x16x4<T>(ai, br, accI);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    cv[u][j].re -= accR[j];
                    cv[u][j].im -= accI[j];
                }
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // D[c' = c0 + mfma_row(lk, j)][r = r0 + li]
                    const int r = rr0[u] + li, c = cc0[u] + mfma_row<T>(lk, j);
                    const int d = r - c;
                    if (r < Mx && c < Mx && d >= 0 && d <= bp) base[(size_t)c * bp1 + d] = cv[u][j];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_band_init(void* LB, int Mx, int bp, int nsys, const int* rowptr, const int* col,
                            const double* valM, const double* valA, const double* lam, hipStream_t st) {
    dim3 grid((Mx + 7) / 8, nsys);
    hipLaunchKernelGGL(band_init_kernel<T>, grid, dim3(256), 0, st, static_cast<cplx<T>*>(LB), Mx, bp,
                       rowptr, col, valM, valA, lam);
    return hipGetLastError();
}

template <typename T>
size_t band_ldl_smem(int bp) { return 2 * 16 * (size_t)(bp + 1) * sizeof(T); }

template <typename T>
hipError_t launch_band_ldl(void* LB, int Mx, int bp, int nsys, int* flag, hipStream_t st) {
    const size_t smem = band_ldl_smem<T>(bp);
    hipError_t e = hipFuncSetAttribute((const void*)band_ldl_kernel<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(band_ldl_kernel<T>, dim3(nsys), dim3(256), smem, st, static_cast<cplx<T>*>(LB), Mx, bp,
                       flag);
    return hipGetLastError();
}

template hipError_t launch_band_init<float>(void*, int, int, int, const int*, const int*, const double*,
                                            const double*, const double*, hipStream_t);
template hipError_t launch_band_init<double>(void*, int, int, int, const int*, const int*, const double*,
                                             const double*, const double*, hipStream_t);
template hipError_t launch_band_ldl<float>(void*, int, int, int, int*, hipStream_t);
template hipError_t launch_band_ldl<double>(void*, int, int, int, int*, hipStream_t);
template size_t band_ldl_smem<float>(int);
template size_t band_ldl_smem<double>(int);

}  // namespace stfd
