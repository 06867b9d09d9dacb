// Triangular sweeps of step 3 of Algorithm FD (Sec. 4.4) with the band
// factors M_x + lambda_k A_x = L_k D_k L_k^T:
//     forward   L_k y = g_k,  w = D_k^-1 y
//     backward  L_k^T z_k = w
// One workgroup (4 waves) per system and group of up to 16 right-hand sides.
//
// The sweeps stream every factor once from HBM, so they are bandwidth work
// with a sequential dependency along the band.  Columns are processed in
// blocks of CB; the L entries of block i + PD are loaded into registers while
// block i is computed (PD blocks in flight), then staged to LDS.  The pending
// right-hand-side values (forward) or finished solution values (backward) of
// the bp + CB rows a block can touch live in an LDS ring.  Inside a block
// the CB x CB unit-triangular part is solved with wave shuffles (one lane per
// row), and the sub-diagonal part is a rank-CB update with one thread per
// (row, right-hand side).
//
// Band storage as in kernels_band.hip: LB[k][c][0] = D, LB[k][c][d] =
// L[c + d, c]; the CB columns of a block are contiguous.
// G/W layout per RHS: column-major M_x x 2 n_sys, real parts of system k in
// column k, imaginary parts in column n_sys + k.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace stfd {

namespace {

constexpr int NT = 256;     // threads per workgroup
constexpr int NRS = 16;     // right-hand sides per workgroup
constexpr int BPMAX = 256;  // largest padded half-bandwidth

constexpr int ept_for(int cb) { return (cb * (BPMAX + 1) + NT - 1) / NT; }   // block elements per thread

// issue the global loads of one block (CB columns) into registers
template <typename T, int CB, int EPT>
__device__ __forceinline__ void load_block(cplx<T> (&r)[EPT], const cplx<T>* base, int blk, int nblk, int Mx,
                                           int bp1) {
    const int tid = threadIdx.x;
    if (blk < 0 || blk >= nblk) return;
    const int c0 = blk * CB;
    const int nbv = min(CB, Mx - c0);
    const int ne = nbv * bp1;
    const cplx<T>* src = base + (size_t)c0 * bp1;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = tid + NT * j;
        r[j] = (e < ne) ? src[e] : cplx<T>{T(0), T(0)};
    }
}

template <typename T, int CB, int EPT>
__device__ __forceinline__ void stage_block(const cplx<T> (&r)[EPT], T* LR, T* LI, int bp1) {
    const int tid = threadIdx.x;
    const int ne = CB * bp1;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = tid + NT * j;
        if (e < ne) {
            LR[e] = r[j].re;
            LI[e] = r[j].im;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
template <typename T, int CB, int PD>
__global__ void __launch_bounds__(NT) sweep_forward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp, int nsys,
                                                           int nrhs, const T* __restrict__ G, T* __restrict__ W) {
    constexpr int EPT = ept_for(CB);
    constexpr int GROUPS = NT / CB;        // right-hand sides per diagonal pass
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ring = bp + CB;
    T* LR = reinterpret_cast<T*>(smem_raw);       // [CB][bp1]
    T* LI = LR + CB * bp1;
    T* QR = LI + CB * bp1;                        // ring [ring][NRS]
    T* QI = QR + ring * NRS;
    T* YR = QI + ring * NRS;                      // [CB][NRS]
    T* YI = YR + CB * NRS;
    const int sys = blockIdx.x;
    const int r0 = blockIdx.y * NRS;
    const int nr = min(NRS, nrhs - r0);
    const cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const size_t rstride = (size_t)Mx * 2 * nsys;
    const T* gre = G + (size_t)r0 * rstride + (size_t)sys * Mx;
    const T* gim = G + (size_t)r0 * rstride + (size_t)(nsys + sys) * Mx;
    T* wre = W + (size_t)r0 * rstride + (size_t)sys * Mx;
    T* wim = W + (size_t)r0 * rstride + (size_t)(nsys + sys) * Mx;
    const int tid = threadIdx.x;
    const int nblk = (Mx + CB - 1) / CB;

    cplx<T> regs[PD][EPT];
#pragma unroll
    for (int s = 0; s < PD; ++s) load_block<T, CB, EPT>(regs[s], base, s, nblk, Mx, bp1);

    // initial window: rows [0, ring)
    for (int q = tid; q < ring * NRS; q += NT) {
        const int row = q / NRS, t = q % NRS;
        T re = 0, im = 0;
        if (row < Mx && t < nr) {
            re = gre[(size_t)t * rstride + row];
            im = gim[(size_t)t * rstride + row];
        }
        QR[q] = re;
        QI[q] = im;
    }

    for (int i0 = 0; i0 < nblk; i0 += PD) {
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            const int blk = i0 + s;
            if (blk >= nblk) break;
            const int c0 = blk * CB;
            const int nb = min(CB, Mx - c0);
            stage_block<T, CB, EPT>(regs[s], LR, LI, bp1);
            load_block<T, CB, EPT>(regs[s], base, blk + PD, nblk, Mx, bp1);
            // right-hand sides of the rows entering the window after this block
            T ent_re[(CB * NRS + NT - 1) / NT], ent_im[(CB * NRS + NT - 1) / NT];
#pragma unroll
            for (int j = 0; j < (CB * NRS + NT - 1) / NT; ++j) {
                const int q = tid + NT * j;
                const int row = c0 + ring + q / NRS, t = q % NRS;
                ent_re[j] = 0;
                ent_im[j] = 0;
                if (q < CB * NRS && row < Mx && t < nr) {
                    ent_re[j] = gre[(size_t)t * rstride + row];
                    ent_im[j] = gim[(size_t)t * rstride + row];
                }
            }
            __syncthreads();
            // unit lower-triangular diagonal block: lane = row k2 of the block
            for (int t0 = 0; t0 < nr; t0 += GROUPS) {
                const int k2 = tid % CB, t = t0 + tid / CB;
                const int slot = ((c0 + k2) % ring) * NRS + min(t, NRS - 1);
                T vr = QR[slot], vi = QI[slot];
                const int gbase = (tid & 63) & ~(CB - 1);
                for (int k = 0; k < nb; ++k) {
                    const T yr = __shfl(vr, gbase | k, 64);
                    const T yi = __shfl(vi, gbase | k, 64);
                    if (k2 > k && k2 - k <= bp) {
                        const T lr = LR[k * bp1 + (k2 - k)], li = LI[k * bp1 + (k2 - k)];
                        vr -= lr * yr - li * yi;
                        vi -= lr * yi + li * yr;
                    }
                }
                if (t < NRS) {
                    YR[k2 * NRS + t] = vr;
                    YI[k2 * NRS + t] = vi;
                }
            }
            __syncthreads();
            // w = y / D for the block
            for (int q = tid; q < CB * NRS; q += NT) {
                const int k2 = q % CB, t = q / CB;
                if (k2 < nb && t < nr) {
                    const cplx<T> inv = cinv(cplx<T>{LR[k2 * bp1], LI[k2 * bp1]});
                    const cplx<T> w = cmul(cplx<T>{YR[k2 * NRS + t], YI[k2 * NRS + t]}, inv);
                    wre[(size_t)t * rstride + c0 + k2] = w.re;
                    wim[(size_t)t * rstride + c0 + k2] = w.im;
                }
            }
            // rows below the block: q[row] -= sum_k L[row, c0 + k] y_k
            for (int q = tid; q < bp * nr; q += NT) {
                const int rr = q % bp, t = q / bp;
                const int row = c0 + CB + rr;
                if (row >= Mx) continue;
                T ar = 0, ai = 0;
                const int kmin = max(0, row - c0 - bp);
                for (int k = kmin; k < nb; ++k) {
                    const int d = row - c0 - k;
                    const T lr = LR[k * bp1 + d], li = LI[k * bp1 + d];
                    const T yr = YR[k * NRS + t], yi = YI[k * NRS + t];
                    ar += lr * yr - li * yi;
                    ai += lr * yi + li * yr;
                }
                const int slot = (row % ring) * NRS + t;
                QR[slot] -= ar;
                QI[slot] -= ai;
            }
            // the rows entering the window take the slots of the block's rows
#pragma unroll
            for (int j = 0; j < (CB * NRS + NT - 1) / NT; ++j) {
                const int q = tid + NT * j;
                if (q < CB * NRS) {
                    const int row = c0 + ring + q / NRS, t = q % NRS;
                    QR[(row % ring) * NRS + t] = ent_re[j];
                    QI[(row % ring) * NRS + t] = ent_im[j];
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB, int PD>
__global__ void __launch_bounds__(NT) sweep_backward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp,
                                                            int nsys, int nrhs, T* __restrict__ W) {
    constexpr int EPT = ept_for(CB);
    constexpr int GROUPS = NT / CB;
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ring = bp + CB;
    T* LR = reinterpret_cast<T*>(smem_raw);       // [CB][bp1]
    T* LI = LR + CB * bp1;
    T* ZR = LI + CB * bp1;                        // ring [ring][NRS] of finished z
    T* ZI = ZR + ring * NRS;
    T* SR = ZI + ring * NRS;                      // [CB][NRS] off-block sums
    T* SI = SR + CB * NRS;
    const int sys = blockIdx.x;
    const int r0 = blockIdx.y * NRS;
    const int nr = min(NRS, nrhs - r0);
    const cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const size_t rstride = (size_t)Mx * 2 * nsys;
    T* wre = W + (size_t)r0 * rstride + (size_t)sys * Mx;
    T* wim = W + (size_t)r0 * rstride + (size_t)(nsys + sys) * Mx;
    const int tid = threadIdx.x;
    const int nblk = (Mx + CB - 1) / CB;
    // (row, rhs) dot products split over `parts` lanes
    const int parts = max(1, NT / (CB * max(nr, 1)));
    const int pw = parts >= 8 ? 8 : parts >= 4 ? 4 : parts >= 2 ? 2 : 1;

    for (int q = tid; q < ring * NRS; q += NT) {
        ZR[q] = 0;
        ZI[q] = 0;
    }
    cplx<T> regs[PD][EPT];
#pragma unroll
    for (int s = 0; s < PD; ++s) load_block<T, CB, EPT>(regs[s], base, nblk - 1 - s, nblk, Mx, bp1);

    for (int i0 = 0; i0 < nblk; i0 += PD) {
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            const int it = i0 + s;
            if (it >= nblk) break;
            const int blk = nblk - 1 - it;
            const int c0 = blk * CB;
            const int nb = min(CB, Mx - c0);
            stage_block<T, CB, EPT>(regs[s], LR, LI, bp1);
            load_block<T, CB, EPT>(regs[s], base, blk - PD, nblk, Mx, bp1);
            __syncthreads();
            // off-block sums for rows c0 + k, k < nb
            {
                const int item = tid / pw, part = tid % pw;
                const int k = item % CB, t = item / CB;
                T ar = 0, ai = 0;
                if (k < nb && t < nr && item < CB * NRS) {
                    for (int d = (nb - k) + part; d <= bp; d += pw) {
                        const int row = c0 + k + d;
                        if (row >= Mx) break;
                        const int slot = (row % ring) * NRS + t;
                        const T lr = LR[k * bp1 + d], li = LI[k * bp1 + d];
                        const T zr = ZR[slot], zi = ZI[slot];
                        ar += lr * zr - li * zi;
                        ai += lr * zi + li * zr;
                    }
                }
                for (int off = pw / 2; off > 0; off >>= 1) {
                    ar += __shfl_down(ar, off, 64);
                    ai += __shfl_down(ai, off, 64);
                }
                if (part == 0 && k < CB && t < NRS) {
                    SR[k * NRS + t] = ar;
                    SI[k * NRS + t] = ai;
                }
                // items beyond one pass (many right-hand sides): plain loop
                for (int it2 = NT / pw + item; it2 < CB * nr; it2 += NT / pw) {
                    const int k3 = it2 % CB, t3 = it2 / CB;
                    T br = 0, bi = 0;
                    if (k3 < nb) {
                        for (int d = (nb - k3) + part; d <= bp; d += pw) {
                            const int row = c0 + k3 + d;
                            if (row >= Mx) break;
                            const int slot = (row % ring) * NRS + t3;
                            const T lr = LR[k3 * bp1 + d], li = LI[k3 * bp1 + d];
                            const T zr = ZR[slot], zi = ZI[slot];
                            br += lr * zr - li * zi;
                            bi += lr * zi + li * zr;
                        }
                    }
                    for (int off = pw / 2; off > 0; off >>= 1) {
                        br += __shfl_down(br, off, 64);
                        bi += __shfl_down(bi, off, 64);
                    }
                    if (part == 0) {
                        SR[k3 * NRS + t3] = br;
                        SI[k3 * NRS + t3] = bi;
                    }
                }
            }
            __syncthreads();
            // diagonal block, descending rows; lane = row k' of the block
            for (int t0 = 0; t0 < nr; t0 += GROUPS) {
                const int kp = tid % CB, t = t0 + tid / CB;
                const bool live = kp < nb && t < nr;
                T vr = 0, vi = 0;
                if (live) {
                    vr = wre[(size_t)t * rstride + c0 + kp] - SR[kp * NRS + t];
                    vi = wim[(size_t)t * rstride + c0 + kp] - SI[kp * NRS + t];
                }
                const int gbase = (tid & 63) & ~(CB - 1);
                for (int k = nb - 1; k >= 0; --k) {
                    const T zr = __shfl(vr, gbase | k, 64);
                    const T zi = __shfl(vi, gbase | k, 64);
                    if (kp < k && k - kp <= bp) {
                        const T lr = LR[kp * bp1 + (k - kp)], li = LI[kp * bp1 + (k - kp)];
                        vr -= lr * zr - li * zi;
                        vi -= lr * zi + li * zr;
                    }
                }
                if (t < NRS) {
                    const int slot = ((c0 + kp) % ring) * NRS + t;
                    ZR[slot] = live ? vr : T(0);
                    ZI[slot] = live ? vi : T(0);
                }
                if (live) {
                    wre[(size_t)t * rstride + c0 + kp] = vr;
                    wim[(size_t)t * rstride + c0 + kp] = vi;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB>
static size_t sweep_smem_cb(int bp) {
    return (2 * (size_t)CB * (bp + 1) + 2 * (size_t)(bp + CB) * NRS + 2 * (size_t)CB * NRS) * sizeof(T);
}

template <typename T>
size_t sweep_smem(int bp) {
    return sweep_smem_cb<T, 16>(bp);    // the smaller configuration always fits if this does
}

template <typename T, int CB, int PD>
static hipError_t launch_fwd(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                             hipStream_t st) {
    const size_t smem = sweep_smem_cb<T, CB>(bp);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_forward_kernel<T, CB, PD>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_forward_kernel<T, CB, PD>), grid, dim3(NT), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<const T*>(G),
                       static_cast<T*>(W));
    return hipGetLastError();
}

template <typename T, int CB, int PD>
static hipError_t launch_bwd(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st) {
    const size_t smem = sweep_smem_cb<T, CB>(bp);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_backward_kernel<T, CB, PD>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_backward_kernel<T, CB, PD>), grid, dim3(NT), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<T*>(W));
    return hipGetLastError();
}

// Column block 32 while it fits in LDS (fewer block steps), else 16.  The
// prefetch depth keeps about two blocks of FP32 or one of FP64 in registers.
template <typename T>
hipError_t launch_band_forward(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                               hipStream_t st) {
    if (bp > BPMAX) return hipErrorInvalidValue;
    constexpr int PD32 = sizeof(T) == 4 ? 2 : 1;
    if (sweep_smem_cb<T, 32>(bp) <= 160 * 1024 && bp <= 128)
        return launch_fwd<T, 32, PD32>(LB, Mx, bp, nsys, nrhs, G, W, st);
    return launch_fwd<T, 16, 2>(LB, Mx, bp, nsys, nrhs, G, W, st);
}

template <typename T>
hipError_t launch_band_backward(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st) {
    if (bp > BPMAX) return hipErrorInvalidValue;
    constexpr int PD32 = sizeof(T) == 4 ? 2 : 1;
    if (sweep_smem_cb<T, 32>(bp) <= 160 * 1024 && bp <= 128)
        return launch_bwd<T, 32, PD32>(LB, Mx, bp, nsys, nrhs, W, st);
    return launch_bwd<T, 16, 2>(LB, Mx, bp, nsys, nrhs, W, st);
}

template hipError_t launch_band_forward<float>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_forward<double>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_backward<float>(const void*, int, int, int, int, void*, hipStream_t);
template hipError_t launch_band_backward<double>(const void*, int, int, int, int, void*, hipStream_t);
template size_t sweep_smem<float>(int);
template size_t sweep_smem<double>(int);

}  // namespace stfd
