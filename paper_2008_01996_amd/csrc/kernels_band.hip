// Batched complex-symmetric band LDL^T factorization and the two triangular
// sweeps (step 3 of Algorithm FD, Sec. 4.4):
//     M_x + lambda_k A_x = L_k D_k L_k^T,   L_k y = g_k,  w = D_k^-1 y,
//     L_k^T z_k = w
// for all systems k at once (one workgroup per system).  The spatial matrices
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
            // later panel columns k2 > k: A[k2 + d2, k2] -= L[k2+d2, k] D_k L[k2, k]
            const int rest = nb - 1 - k;
            for (int q = tid; q < rest * bp1; q += blockDim.x) {
                const int k2 = k + 1 + q / bp1;
                const int d2 = q % bp1;
                const int dd = (k2 - k) + d2;           // row offset from column k
                if (dd <= bp) {
                    const cplx<T> lk2 = {PR[k * bp1 + (k2 - k)], PI[k * bp1 + (k2 - k)]};
                    const cplx<T> lr = {PR[k * bp1 + dd], PI[k * bp1 + dd]};
                    const cplx<T> t = cmul(cmul(lr, dk), lk2);
                    PR[k2 * bp1 + d2] -= t.re;
                    PI[k2 * bp1 + d2] -= t.im;
                }
            }
            __syncthreads();
        }
        // ---- write the finished panel (L columns and D)
        cplx<T>* dst = base + (size_t)p0 * bp1;
        for (int e = tid; e < nb * bp1; e += blockDim.x) dst[e] = cplx<T>{PR[e], PI[e]};
        // ---- trailing update on the matrix cores
        // tile (ti, tj), ti >= tj: rows r0 = p0 + 16 + 16 ti, columns c0 = p0 + 16 + 16 tj
        for (int t = wave; t < tiles_total; t += 4) {
            // map linear t to (ti, tj) with tj <= ti
            int ti = 0;
            while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
            const int tj = t - ti * (ti + 1) / 2;
            const int r0 = p0 + 16 + 16 * ti;
            const int c0 = p0 + 16 + 16 * tj;
            if (c0 >= Mx || r0 >= Mx) continue;
            typename vec4<T>::type accR = zero4<T>(), accI = zero4<T>();
            const int li = lane & 15, lk = lane >> 4;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                // A operand: L[c', k] with c' = c0 + li  (offset c' - p0 - k)
                // B operand: L[r, k] D[k] with r = r0 + li
                T ar = 0, ai = 0, br = 0, bi = 0;
                if (k < nb) {
                    const int oc = c0 + li - p0 - k;
                    if (oc >= 1 && oc <= bp) {
                        ar = PR[k * bp1 + oc];
                        ai = PI[k * bp1 + oc];
                    }
                    const int orr = r0 + li - p0 - k;
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
            // D[c' = c0 + mfma_row(lk, j)][r = r0 + li]
            const int r = r0 + li;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = c0 + mfma_row<T>(lk, j);
                const int d = r - c;
                if (r < Mx && c < Mx && d >= 0 && d <= bp) {
                    cplx<T>* p = base + (size_t)c * bp1 + d;
                    cplx<T> v = *p;
                    v.re -= accR[j];
                    v.im -= accI[j];
                    *p = v;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Forward sweep L y = g, w = D^-1 y, for one system per workgroup and up to
// 16 right-hand sides per workgroup (grid.y groups of 16).
//
// G/W layout (per RHS, column-major M_x x 2 n_sys): real part of system k in
// column k, imaginary part in column n_sys + k.
// The 16 L columns of a block are staged in LDS; the pending right-hand side
// values of the next bp + 16 rows live in an LDS ring.  The 16 x 16 unit
// diagonal block is solved with wave shuffles (lane = row within the block),
// the sub-diagonal rows are then updated by the block in parallel.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) band_forward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp,
                                                           int nsys, int nrhs,
                                                           const T* __restrict__ G, T* __restrict__ W) {
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ring = bp + 16;
    T* LR = reinterpret_cast<T*>(smem_raw);       // [16][bp1]
    T* LI = LR + 16 * bp1;
    T* QR = LI + 16 * bp1;                        // ring [ring][16]
    T* QI = QR + ring * 16;
    T* YR = QI + ring * 16;                       // [16][16] block solution
    T* YI = YR + 256;
    const int sys = blockIdx.x;
    const int r0 = blockIdx.y * 16;
    const int nr = min(16, nrhs - r0);
    const cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const size_t rstride = (size_t)Mx * 2 * nsys;   // per-RHS stride of G/W
    const int tid = threadIdx.x;

    auto gval = [&](int row, int t, T& re, T& im) {
        const T* g = G + (size_t)(r0 + t) * rstride;
        re = g[(size_t)sys * Mx + row];
        im = g[(size_t)(nsys + sys) * Mx + row];
    };
    // initial window rows [0, min(ring, Mx))
    for (int q = tid; q < ring * 16; q += blockDim.x) {
        const int row = q / 16, t = q % 16;
        T re = 0, im = 0;
        if (row < Mx && t < nr) gval(row, t, re, im);
        QR[(row % ring) * 16 + t] = re;
        QI[(row % ring) * 16 + t] = im;
    }
    for (int c0 = 0; c0 < Mx; c0 += 16) {
        const int nb = min(16, Mx - c0);
        const cplx<T>* src = base + (size_t)c0 * bp1;
        for (int e = tid; e < 16 * bp1; e += blockDim.x) {
            cplx<T> v = (e < nb * bp1) ? src[e] : cplx<T>{T(0), T(0)};
            LR[e] = v.re;
            LI[e] = v.im;
        }
        __syncthreads();
        // diagonal block: lane (row k2 = lane % 16, rhs t = 4 wave + lane / 16)
        {
            const int k2 = tid & 15, t = tid >> 4;
            const int slot = ((c0 + k2) % ring) * 16 + t;
            T vr = QR[slot], vi = QI[slot];
            for (int k = 0; k < nb; ++k) {
                const int src_lane = (tid & 48) | k;          // same 16-lane group, row k
                const T yr = __shfl(vr, src_lane, 64);
                const T yi = __shfl(vi, src_lane, 64);
                if (k2 > k && k2 < nb) {
                    const T lr = LR[k * bp1 + (k2 - k)], li = LI[k * bp1 + (k2 - k)];
                    vr -= lr * yr - li * yi;
                    vi -= lr * yi + li * yr;
                }
            }
            YR[k2 * 16 + t] = vr;
            YI[k2 * 16 + t] = vi;
        }
        __syncthreads();
        // outputs w = y / D
        {
            const int k2 = tid & 15, t = tid >> 4;
            if (k2 < nb && t < nr) {
                const cplx<T> inv = cinv(cplx<T>{LR[k2 * bp1], LI[k2 * bp1]});
                const cplx<T> w = cmul(cplx<T>{YR[k2 * 16 + t], YI[k2 * 16 + t]}, inv);
                T* wp = W + (size_t)(r0 + t) * rstride;
                wp[(size_t)sys * Mx + c0 + k2] = w.re;
                wp[(size_t)(nsys + sys) * Mx + c0 + k2] = w.im;
            }
        }
        // sub-diagonal rows r in [c0 + 16, c0 + 16 + bp): q -= sum_k L[r, c0+k] y_k
        for (int q = tid; q < bp * 16; q += blockDim.x) {
            const int rr = q / 16, t = q % 16;
            const int row = c0 + 16 + rr;
            if (row >= Mx || t >= nr) continue;
            T ar = 0, ai = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int d = row - c0 - k;
                if (k < nb && d <= bp) {
                    const T lr = LR[k * bp1 + d], li = LI[k * bp1 + d];
                    const T yr = YR[k * 16 + t], yi = YI[k * 16 + t];
                    ar += lr * yr - li * yi;
                    ai += lr * yi + li * yr;
                }
            }
            const int slot = (row % ring) * 16 + t;
            QR[slot] -= ar;
            QI[slot] -= ai;
        }
        // rows entering the window: [c0 + ring, c0 + ring + 16) reuse the slots of [c0, c0 + 16)
        {
            const int k2 = tid & 15, t = tid >> 4;
            const int row = c0 + ring + k2;
            T re = 0, im = 0;
            if (row < Mx && t < nr) gval(row, t, re, im);
            QR[(row % ring) * 16 + t] = re;
            QI[(row % ring) * 16 + t] = im;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Backward sweep L^T z = w (in place in W), columns in descending blocks of 16.
// z[c] = w[c] - sum_{d=1..bp} L[c+d, c] z[c+d]: the part from rows beyond the
// block is a dot product over the column (parallel over rows and split over
// lanes), the part inside the block is solved with wave shuffles.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) band_backward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp,
                                                            int nsys, int nrhs, T* __restrict__ W) {
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ring = bp + 16;
    T* LR = reinterpret_cast<T*>(smem_raw);       // [16][bp1]
    T* LI = LR + 16 * bp1;
    T* ZR = LI + 16 * bp1;                        // ring [ring][16] of finished z
    T* ZI = ZR + ring * 16;
    T* SR = ZI + ring * 16;                       // [16][16] off-block sums
    T* SI = SR + 256;
    const int sys = blockIdx.x;
    const int r0 = blockIdx.y * 16;
    const int nr = min(16, nrhs - r0);
    const cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const size_t rstride = (size_t)Mx * 2 * nsys;
    const int tid = threadIdx.x;
    // parts per (row, rhs) dot product
    const int parts = (nr <= 1) ? 16 : (nr <= 2) ? 8 : (nr <= 4) ? 4 : (nr <= 8) ? 2 : 1;

    for (int q = tid; q < ring * 16; q += blockDim.x) {
        ZR[q] = 0;
        ZI[q] = 0;
    }
    const int last = ((Mx - 1) / 16) * 16;
    for (int c0 = last; c0 >= 0; c0 -= 16) {
        const int nb = min(16, Mx - c0);
        const cplx<T>* src = base + (size_t)c0 * bp1;
        for (int e = tid; e < 16 * bp1; e += blockDim.x) {
            cplx<T> v = (e < nb * bp1) ? src[e] : cplx<T>{T(0), T(0)};
            LR[e] = v.re;
            LI[e] = v.im;
        }
        __syncthreads();
        // off-block sums S[k][t] = sum_{d >= nb - k} L[c0+k+d, c0+k] z[c0+k+d]
        {
            // 256 threads = 16 rows x nrs right-hand sides x parts
            const int nrs = 16 / parts;
            const int item = tid / parts, part = tid % parts;
            const int k = item / nrs;
            const int t = item % nrs;
            T ar = 0, ai = 0;
            if (k < nb && t < nr) {
                for (int d = (nb - k) + part; d <= bp; d += parts) {
                    const int row = c0 + k + d;
                    if (row >= Mx) break;
                    const int slot = (row % ring) * 16 + t;
                    const T lr = LR[k * bp1 + d], li = LI[k * bp1 + d];
                    const T zr = ZR[slot], zi = ZI[slot];
                    ar += lr * zr - li * zi;
                    ai += lr * zi + li * zr;
                }
            }
            for (int off = parts / 2; off > 0; off >>= 1) {
                ar += __shfl_down(ar, off, 64);
                ai += __shfl_down(ai, off, 64);
            }
            if (part == 0) {
                SR[k * 16 + t] = ar;
                SI[k * 16 + t] = ai;
            }
        }
        __syncthreads();
        // diagonal block, descending rows; lane (row k' = lane % 16, rhs t)
        {
            const int kp = tid & 15, t = tid >> 4;
            T vr = 0, vi = 0;
            if (kp < nb && t < nr) {
                const T* wp = W + (size_t)(r0 + t) * rstride;
                vr = wp[(size_t)sys * Mx + c0 + kp] - SR[kp * 16 + t];
                vi = wp[(size_t)(nsys + sys) * Mx + c0 + kp] - SI[kp * 16 + t];
            }
            for (int k = nb - 1; k >= 0; --k) {
                const int src_lane = (tid & 48) | k;
                const T zr = __shfl(vr, src_lane, 64);
                const T zi = __shfl(vi, src_lane, 64);
                if (kp < k) {
                    const T lr = LR[kp * bp1 + (k - kp)], li = LI[kp * bp1 + (k - kp)];
                    vr -= lr * zr - li * zi;
                    vi -= lr * zi + li * zr;
                }
            }
            const int slot = ((c0 + kp) % ring) * 16 + t;
            ZR[slot] = (kp < nb && t < nr) ? vr : T(0);
            ZI[slot] = (kp < nb && t < nr) ? vi : T(0);
            if (kp < nb && t < nr) {
                T* wp = W + (size_t)(r0 + t) * rstride;
                wp[(size_t)sys * Mx + c0 + kp] = vr;
                wp[(size_t)(nsys + sys) * Mx + c0 + kp] = vi;
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

template <typename T>
size_t sweep_smem(int bp) {
    return (2 * 16 * (size_t)(bp + 1) + 2 * (size_t)(bp + 16) * 16 + 2 * 256) * sizeof(T);
}

template <typename T>
hipError_t launch_band_forward(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                               hipStream_t st) {
    const size_t smem = sweep_smem<T>(bp);
    hipError_t e = hipFuncSetAttribute((const void*)band_forward_kernel<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + 15) / 16);
    hipLaunchKernelGGL(band_forward_kernel<T>, grid, dim3(256), smem, st, static_cast<const cplx<T>*>(LB), Mx,
                       bp, nsys, nrhs, static_cast<const T*>(G), static_cast<T*>(W));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_band_backward(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st) {
    const size_t smem = sweep_smem<T>(bp);
    hipError_t e = hipFuncSetAttribute((const void*)band_backward_kernel<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + 15) / 16);
    hipLaunchKernelGGL(band_backward_kernel<T>, grid, dim3(256), smem, st, static_cast<const cplx<T>*>(LB), Mx,
                       bp, nsys, nrhs, static_cast<T*>(W));
    return hipGetLastError();
}

template hipError_t launch_band_init<float>(void*, int, int, int, const int*, const int*, const double*,
                                            const double*, const double*, hipStream_t);
template hipError_t launch_band_init<double>(void*, int, int, int, const int*, const int*, const double*,
                                             const double*, const double*, hipStream_t);
template hipError_t launch_band_ldl<float>(void*, int, int, int, int*, hipStream_t);
template hipError_t launch_band_ldl<double>(void*, int, int, int, int*, hipStream_t);
template hipError_t launch_band_forward<float>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_forward<double>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_backward<float>(const void*, int, int, int, int, void*, hipStream_t);
template hipError_t launch_band_backward<double>(const void*, int, int, int, int, void*, hipStream_t);
template size_t band_ldl_smem<float>(int);
template size_t band_ldl_smem<double>(int);
template size_t sweep_smem<float>(int);
template size_t sweep_smem<double>(int);

}  // namespace stfd
