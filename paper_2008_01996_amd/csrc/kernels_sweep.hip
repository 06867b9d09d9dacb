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

constexpr int ept_for(int cb, int bpc) { return (cb * (bpc + 1) + NT - 1) / NT; }   // block elements per thread

// issue the global loads of one block (CB columns) into registers; branch-free
// (clamped addresses, masked values) so that the waits on them can be partial
template <typename T, int CB, int EPT>
__device__ __forceinline__ void load_block(cplx<T> (&r)[EPT], const cplx<T>* base, int blk, int nblk, int Mx,
                                           int bp1) {
    const int tid = threadIdx.x;
    const int b = min(max(blk, 0), nblk - 1);
    const int c0 = b * CB;
    const int ne = min(CB, Mx - c0) * bp1;
    const bool live = blk >= 0 && blk < nblk;
    const cplx<T>* src = base + (size_t)c0 * bp1;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = tid + NT * j;
        const cplx<T> v = src[min(e, ne - 1)];
        const bool ok = live && e < ne;
        r[j].re = ok ? v.re : T(0);
        r[j].im = ok ? v.im : T(0);
    }
}

// LDS block buffers hold EPT * NT entries so that staging needs no bounds test
template <typename T, int CB, int EPT>
__device__ __forceinline__ void stage_block(const cplx<T> (&r)[EPT], T* LR, T* LI) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = tid + NT * j;
        LR[e] = r[j].re;
        LI[e] = r[j].im;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
template <typename T, int CB, int PD, int BPC>
__global__ void __launch_bounds__(NT) sweep_forward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp, int nsys,
                                                           int nrhs, const T* __restrict__ G, T* __restrict__ W) {
    constexpr int EPT = ept_for(CB, BPC);
    constexpr int GROUPS = NT / CB;        // right-hand sides per diagonal pass
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ring = bp + CB;
    T* LR = reinterpret_cast<T*>(smem_raw);       // [CB][bp1] (EPT * NT entries)
    T* LI = LR + EPT * NT;
    T* QR = LI + EPT * NT;                        // ring [ring][NRS]
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

    int cs = 0;                           // c0 mod ring, kept incrementally
    auto wrap = [ring](int x) { return x >= ring ? x - ring : x; };
    for (int i0 = 0; i0 < nblk; i0 += PD) {
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            // blocks past the end are empty (nb = 0) so the loop stays uniform
            const int blk = i0 + s;
            const int c0 = blk * CB;
            const int nb = max(0, min(CB, Mx - c0));
            // right-hand sides of the rows entering the window after this block
            // (issued before the prefetch below, so waiting for them later
            // does not drain it)
            T ent_re[(CB * NRS + NT - 1) / NT], ent_im[(CB * NRS + NT - 1) / NT];
#pragma unroll
            for (int j = 0; j < (CB * NRS + NT - 1) / NT; ++j) {
                const int q = tid + NT * j;
                const int row = c0 + ring + q / NRS, t = q % NRS;
                const bool ok = q < CB * NRS && row < Mx && t < nr;
                const size_t off = ok ? (size_t)t * rstride + row : 0;
                const T a = gre[off], b = gim[off];
                ent_re[j] = ok ? a : T(0);
                ent_im[j] = ok ? b : T(0);
            }
            stage_block<T, CB, EPT>(regs[s], LR, LI);
            load_block<T, CB, EPT>(regs[s], base, blk + PD, nblk, Mx, bp1);
            __syncthreads();
            // unit lower-triangular diagonal block: lane = row k2 of the block
            for (int t0 = 0; t0 < nr; t0 += GROUPS) {
                const int k2 = tid % CB, t = t0 + tid / CB;
                const int slot = wrap(cs + k2) * NRS + min(t, NRS - 1);
                T vr = QR[slot], vi = QI[slot];
                const int grp = (tid & 63) / CB;
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    if (k >= nb) continue;
                    const T yr = group_bcast<CB>(vr, k, grp);
                    const T yi = group_bcast<CB>(vi, k, grp);
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
            for (int t = 0; t < nr; ++t)
            for (int rr = tid; rr < bp; rr += NT) {
                const int row = c0 + CB + rr;
                if (row >= Mx) continue;
                T ar = 0, ai = 0;
                const int kmin = row - c0 - bp;
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    // fully unrolled with masked terms: all LDS reads issue together
                    const int d = min(max(row - c0 - k, 0), bp);
                    const bool on = k < nb && k >= kmin;
                    const T lr = LR[k * bp1 + d], li = LI[k * bp1 + d];
                    const T yr = on ? YR[k * NRS + t] : T(0), yi = on ? YI[k * NRS + t] : T(0);
                    ar += lr * yr - li * yi;
                    ai += lr * yi + li * yr;
                }
                const int slot = wrap(cs + CB + rr) * NRS + t;
                QR[slot] -= ar;
                QI[slot] -= ai;
            }
            // the rows entering the window take the slots of the block's rows
#pragma unroll
            for (int j = 0; j < (CB * NRS + NT - 1) / NT; ++j) {
                const int q = tid + NT * j;
                if (q < CB * NRS) {
                    const int slot = wrap(cs + q / NRS) * NRS + q % NRS;
                    QR[slot] = ent_re[j];
                    QI[slot] = ent_im[j];
                }
            }
            cs = wrap(cs + CB);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB, int PD, int BPC>
__global__ void __launch_bounds__(NT) sweep_backward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp,
                                                            int nsys, int nrhs, T* __restrict__ W) {
    constexpr int EPT = ept_for(CB, BPC);
    constexpr int GROUPS = NT / CB;
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ring = bp + CB;
    T* LR = reinterpret_cast<T*>(smem_raw);       // [CB][bp1] (EPT * NT entries)
    T* LI = LR + EPT * NT;
    T* ZR = LI + EPT * NT;                        // ring [ring][NRS] of finished z
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
    const int lpw = parts >= 8 ? 3 : parts >= 4 ? 2 : parts >= 2 ? 1 : 0;
    const int pw = 1 << lpw;

    for (int q = tid; q < ring * NRS; q += NT) {
        ZR[q] = 0;
        ZI[q] = 0;
    }
    cplx<T> regs[PD][EPT];
#pragma unroll
    for (int s = 0; s < PD; ++s) load_block<T, CB, EPT>(regs[s], base, nblk - 1 - s, nblk, Mx, bp1);

    int cs = ((nblk - 1) * CB) % ring;    // c0 mod ring, kept incrementally
    auto wrap = [ring](int x) { return x >= ring ? x - ring : x; };
    for (int i0 = 0; i0 < nblk; i0 += PD) {
#pragma unroll
        for (int s = 0; s < PD; ++s) {
            // iterations past the first block are empty (nb = 0): uniform loop
            const int it = i0 + s;
            const int blk = nblk - 1 - it;
            const int c0 = blk * CB;
            const int nb = blk >= 0 ? min(CB, Mx - c0) : 0;
            // w of the block's rows, one (row, rhs) pair per lane and pass,
            // issued before the prefetch below
            constexpr int NP = (CB * NRS + NT - 1) / NT;
            T wv_re[NP], wv_im[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const int q = tid + NT * j;
                const int kp = q % CB, t = q / CB;
                const bool ok = kp < nb && t < nr;
                const size_t off = ok ? (size_t)t * rstride + c0 + kp : 0;
                const T a = wre[off], b = wim[off];
                wv_re[j] = ok ? a : T(0);
                wv_im[j] = ok ? b : T(0);
            }
            stage_block<T, CB, EPT>(regs[s], LR, LI);
            load_block<T, CB, EPT>(regs[s], base, blk - PD, nblk, Mx, bp1);
            __syncthreads();
            // off-block sums for rows c0 + k, k < nb
            {
                const int item = tid >> lpw, part = tid & (pw - 1);
                const int k = item % CB, t = item / CB;
                T ar = 0, ai = 0;
                if (k < nb && t < nr && item < CB * NRS) {
                    const int d0 = (nb - k) + part;
                    int rs = wrap(cs + k + d0);
                    for (int d = d0; d <= bp; d += pw) {
                        const int row = c0 + k + d;
                        if (row >= Mx) break;
                        const int slot = rs * NRS + t;
                        rs += pw;
                        if (rs >= ring) rs -= ring;
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
                for (int it2 = (NT >> lpw) + item; it2 < CB * nr; it2 += (NT >> lpw)) {
                    const int k3 = it2 % CB, t3 = it2 / CB;
                    T br = 0, bi = 0;
                    if (k3 < nb) {
                        int rs3 = wrap(cs + k3 + (nb - k3) + part);
                        for (int d = (nb - k3) + part; d <= bp; d += pw) {
                            const int row = c0 + k3 + d;
                            if (row >= Mx) break;
                            const int slot = rs3 * NRS + t3;
                            rs3 = wrap(rs3 + pw);
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
#pragma unroll
            for (int pass = 0; pass < NP; ++pass) {
                const int t0 = pass * GROUPS;
                if (t0 >= nr) break;
                const int kp = tid % CB, t = t0 + tid / CB;
                const bool live = kp < nb && t < nr;
                T vr = 0, vi = 0;
                if (live) {
                    vr = wv_re[pass] - SR[kp * NRS + t];
                    vi = wv_im[pass] - SI[kp * NRS + t];
                }
                const int grp = (tid & 63) / CB;
#pragma unroll
                for (int kk = 0; kk < CB; ++kk) {
                    const int k = CB - 1 - kk;
                    if (k >= nb) continue;
                    const T zr = group_bcast<CB>(vr, k, grp);
                    const T zi = group_bcast<CB>(vi, k, grp);
                    if (kp < k && k - kp <= bp) {
                        const T lr = LR[kp * bp1 + (k - kp)], li = LI[kp * bp1 + (k - kp)];
                        vr -= lr * zr - li * zi;
                        vi -= lr * zi + li * zr;
                    }
                }
                if (t < NRS && nb > 0) {
                    const int slot = wrap(cs + kp) * NRS + t;
                    ZR[slot] = live ? vr : T(0);
                    ZI[slot] = live ? vi : T(0);
                }
                if (live) {
                    wre[(size_t)t * rstride + c0 + kp] = vr;
                    wim[(size_t)t * rstride + c0 + kp] = vi;
                }
            }
            cs = cs >= CB ? cs - CB : cs - CB + ring;
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB, int BPC>
static size_t sweep_smem_cb(int bp) {
    return (2 * (size_t)ept_for(CB, BPC) * NT + 2 * (size_t)(bp + CB) * NRS + 2 * (size_t)CB * NRS) * sizeof(T);
}

template <typename T>
size_t sweep_smem(int bp) {
    return bp <= 128 ? sweep_smem_cb<T, 32, 128>(bp) : sweep_smem_cb<T, 16, 256>(bp);
}

template <typename T, int CB, int PD, int BPC>
static hipError_t launch_fwd(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                             hipStream_t st) {
    const size_t smem = sweep_smem_cb<T, CB, BPC>(bp);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_forward_kernel<T, CB, PD, BPC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_forward_kernel<T, CB, PD, BPC>), grid, dim3(NT), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<const T*>(G),
                       static_cast<T*>(W));
    return hipGetLastError();
}

template <typename T, int CB, int PD, int BPC>
static hipError_t launch_bwd(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st) {
    const size_t smem = sweep_smem_cb<T, CB, BPC>(bp);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_backward_kernel<T, CB, PD, BPC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_backward_kernel<T, CB, PD, BPC>), grid, dim3(NT), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<T*>(W));
    return hipGetLastError();
}

// bp <= 128: column blocks of 32 with 3 (FP32) or 2 (FP64) blocks in flight;
// bp <= 256: blocks of 16 with 3 / 2 in flight.
template <typename T>
hipError_t launch_band_forward(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                               hipStream_t st) {
    if (bp > BPMAX) return hipErrorInvalidValue;
    constexpr int PD = sizeof(T) == 4 ? 3 : 2;
    if (bp <= 128) return launch_fwd<T, 32, PD, 128>(LB, Mx, bp, nsys, nrhs, G, W, st);
    return launch_fwd<T, 16, PD, 256>(LB, Mx, bp, nsys, nrhs, G, W, st);
}

template <typename T>
hipError_t launch_band_backward(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st) {
    if (bp > BPMAX) return hipErrorInvalidValue;
    constexpr int PD = sizeof(T) == 4 ? 3 : 2;
    if (bp <= 128) return launch_bwd<T, 32, PD, 128>(LB, Mx, bp, nsys, nrhs, W, st);
    return launch_bwd<T, 16, PD, 256>(LB, Mx, bp, nsys, nrhs, W, st);
}

template hipError_t launch_band_forward<float>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_forward<double>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_backward<float>(const void*, int, int, int, int, void*, hipStream_t);
template hipError_t launch_band_backward<double>(const void*, int, int, int, int, void*, hipStream_t);
template size_t sweep_smem<float>(int);
template size_t sweep_smem<double>(int);

}  // namespace stfd
