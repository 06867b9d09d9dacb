// Triangular sweeps of step 3 of Algorithm FD (Sec. 4.4) with the band
// factors M_x + lambda_k A_x = L_k D_k L_k^T:
//     forward   L_k y = g_k,  w = D_k^-1 y
//     backward  L_k^T z_k = w
//
// Along one system the sweeps are a sequential chain of column blocks of CB
// columns, and every factor entry is read once.  One workgroup of four waves
// runs one system for up to NRS right-hand sides:
//   * wave 0 runs the critical path of each block alone, with no barrier
//     inside the block: the CB x CB unit-triangular solve (one lane per row
//     and right-hand side, values passed on by lane broadcasts, the lane's
//     row of L held in registers) and the coupling to the adjacent block
//     (forward: the update of the next block's rows; backward: the sums over
//     the rows of the block just finished);
//   * waves 1-3 stream the L entries of block i + 2 (with the right-hand-side
//     values that block needs) into one of three LDS slots, their global
//     loads issued two blocks ahead, and do the rest of the band coupling one
//     block off the critical path (forward: the update of rows two or more
//     blocks below by the block finished one step earlier; backward: the sums
//     over rows two or more blocks below for the block processed next).
// One workgroup barrier per block hands slots and buffers over.  The pending
// values of the bp + CB rows a block can touch (forward), or the finished z
// of the rows below it (backward), live in an LDS ring.
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

constexpr int NT = 256;      // threads per workgroup
constexpr int NL = 192;      // lanes of waves 1-3
constexpr int NRS = 8;       // right-hand sides per workgroup
constexpr int NSLOT = 3;     // LDS block slots
constexpr int BPMAX = 256;   // largest padded half-bandwidth

template <typename T, int CB, int BPC>
struct Cfg {
    static constexpr int EL = (CB * (BPC + 1) + NL - 1) / NL;  // L entries per loader lane
    static constexpr int ER = (CB * NRS + NL - 1) / NL;         // right-hand-side values per loader lane
    static constexpr int EPB = EL * NL + CB;                    // L entries of a slot, columns at stride bp + 2
    static constexpr int ERB = ER * NL;                         // right-hand-side values of a slot
    static constexpr int SLOT = 2 * EPB + 2 * ERB;              // T elements per slot
};

// LDS carve-up: [NSLOT slots][ring re][ring im][2 x block buffer re][im][block buffer re][im]
template <typename T, int CB, int BPC>
__host__ __device__ constexpr size_t smem_elems(int bp) {
    return (size_t)NSLOT * Cfg<T, CB, BPC>::SLOT + 2 * (size_t)(bp + CB) * NRS + 6 * (size_t)CB * NRS;
}

// Loader: global -> registers for block blk.  Addresses are clamped into the
// factor and right-hand-side arrays and the values are not masked, so the
// loads stay in flight until the registers are deposited two blocks later.
// Entries outside the block (columns past M_x, rows past M_x, right-hand
// sides past nrhs, blocks past the end) hold finite copies of valid entries;
// every use below masks them out.
template <typename T, int CB, int EL, int ER>
__device__ __forceinline__ void fetch(cplx<T> (&l)[EL], cplx<T> (&r)[ER], const cplx<T>* base, int blk, int nblk,
                                      int Mx, int bp1, const T* vre, const T* vim, size_t rstride, int nr, int rowoff,
                                      int li) {
    const int b = min(max(blk, 0), nblk - 1);
    const int c0 = b * CB;
    const int last = min(CB, Mx - c0) * bp1 - 1;
    const cplx<T>* src = base + (size_t)c0 * bp1;
#pragma unroll
    for (int j = 0; j < EL; ++j) l[j] = src[min(li + NL * j, last)];
    // right-hand-side values of rows blk*CB + rowoff + q / NRS, q in [0, CB * NRS)
#pragma unroll
    for (int j = 0; j < ER; ++j) {
        const int q = li + NL * j;
        const int row = min(max(blk * CB + rowoff + q / NRS, 0), Mx - 1);
        const int t = min(q % NRS, nr - 1);
        const size_t off = (size_t)t * rstride + row;
        r[j].re = vre[off];
        r[j].im = vim[off];
    }
}

// LDS offsets of a loader lane's L entries: in LDS the columns of a block
// are bp + 2 apart (entry d of column c at c * (bp + 2) + d), so that lanes
// reading one row of L across columns hit distinct banks.  Entries past the
// block's CB columns go to the end of the slot.
template <int CB, int EL>
__device__ __forceinline__ void lds_offsets(int (&off)[EL], int bp1, int li) {
#pragma unroll
    for (int j = 0; j < EL; ++j) {
        const int e = li + NL * j;
        off[j] = e + min(e / bp1, CB);
    }
}

// loader: registers -> LDS slot
template <typename T, int EPB, int ERB, int EL, int ER>
__device__ __forceinline__ void deposit(const cplx<T> (&l)[EL], const cplx<T> (&r)[ER], const int (&off)[EL],
                                        T* slot, int li) {
    T* LR = slot;
    T* LI = slot + EPB;
    T* GR = slot + 2 * EPB;
    T* GI = GR + ERB;
#pragma unroll
    for (int j = 0; j < EL; ++j) {
        LR[off[j]] = l[j].re;
        LI[off[j]] = l[j].im;
    }
#pragma unroll
    for (int j = 0; j < ER; ++j) {
        GR[li + NL * j] = r[j].re;
        GI[li + NL * j] = r[j].im;
    }
}

// Forward, off the critical path (waves 1-3): rows c0 + CB + rr, rr in
// [CB, bp), of the pending ring take the update by block (c0, nb) with its
// solution y.  cs = (c0 + CB) mod ring.
template <typename T, int CB>
__device__ __forceinline__ void forward_far_update(const T* LR, const T* LI, const T* YR, const T* YI, T* QR, T* QI,
                                                   int c0, int nb, int Mx, int bp, int ls, int nr, int cs, int ring,
                                                   int li) {
    const int nrow = bp - CB;
    for (int t = 0; t < nr; ++t) {
        for (int m = li; m < nrow; m += NL) {
            const int rr = CB + m;
            if (c0 + CB + rr >= Mx) break;
            const int kmin = CB + rr - bp;   // L[row, c0 + k] lies in the band for k >= kmin
            T ar = 0, ai = 0;
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const int d = min(CB + rr - k, bp);
                const bool on = k < nb && k >= kmin;
                const T yr = on ? YR[k * NRS + t] : T(0), yi = on ? YI[k * NRS + t] : T(0);
                cmac(ar, ai, LR[k * ls + d], LI[k * ls + d], yr, yi);
            }
            int s = cs + rr;
            s = s >= ring ? s - ring : s;
            QR[s * NRS + t] -= ar;
            QI[s * NRS + t] -= ai;
        }
    }
}

// Backward, off the critical path (waves 1-3): for the full block at c0,
// S[k][t] = sum over rows r in [c0 + 2 CB, min(c0 + k + bp, M_x)) of
// L[r, c0 + k] z[r][t].  cs = (c0 + CB) mod ring.
template <typename T, int CB>
__device__ __forceinline__ void backward_far_sums(const T* LR, const T* LI, const T* ZR, const T* ZI, T* SR, T* SI,
                                                  int c0, int Mx, int bp, int ls, int nr, int cs, int ring, int li) {
    const int items = CB * nr;
    int lpw = 0;                                  // 2^lpw lanes share one (k, t) sum
    while (lpw < 6 && (items << (lpw + 1)) <= NL) ++lpw;
    const int pw = 1 << lpw;
    for (int b0 = 0; b0 < items; b0 += NL >> lpw) {
        const int item = b0 + (li >> lpw), part = li & (pw - 1);
        const int k = item % CB, t = item / CB;
        T ar = 0, ai = 0;
        if (item < items) {
            const int dmax = min(bp, Mx - 1 - c0 - k);
            int s = cs + CB + part;               // ring slot of row c0 + k + d, d = 2 CB - k + part
            s = s >= ring ? s - ring : s;
            for (int d = 2 * CB - k + part; d <= dmax; d += pw) {
                cmac(ar, ai, LR[k * ls + d], LI[k * ls + d], ZR[s * NRS + t], ZI[s * NRS + t]);
                s += pw;
                s = s >= ring ? s - ring : s;
            }
        }
        for (int off = pw >> 1; off > 0; off >>= 1) {
            ar += __shfl_xor(ar, off, 64);
            ai += __shfl_xor(ai, off, 64);
        }
        if (part == 0 && item < items) {
            SR[k * NRS + t] = ar;
            SI[k * NRS + t] = ai;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
template <typename T, int CB, int BPC>
__global__ void __launch_bounds__(NT) sweep_forward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp, int nsys,
                                                           int nrhs, const T* __restrict__ G, T* __restrict__ W) {
    using C = Cfg<T, CB, BPC>;
    constexpr int GPW = 64 / CB;                  // right-hand sides per chain pass
    constexpr int KPER = CB / GPW;                // columns per lane in the next-block update
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ls = bp + 2;                        // LDS column stride of L
    const int ring = bp + CB;
    T* slots = reinterpret_cast<T*>(smem_raw);
    T* QR = slots + NSLOT * C::SLOT;              // pending rows, ring [ring][NRS]
    T* QI = QR + ring * NRS;
    T* YR = QI + ring * NRS;                      // y of a block, [2][CB][NRS] by step parity
    T* YI = YR + 2 * CB * NRS;
    T* PR = YI + 2 * CB * NRS;                    // update of the next block's rows, [CB][NRS]
    T* PI = PR + CB * NRS;
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
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nblk = (Mx + CB - 1) / CB;
    const int nbar = (nblk + 1) & ~1;             // block steps, rounded up to even
    auto wrap = [ring](int x) { return x >= ring ? x - ring : x; };

    // initial window: rows [0, ring); no update of block 0 yet
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
    for (int q = tid; q < CB * NRS; q += NT) {
        PR[q] = 0;
        PI[q] = 0;
    }

    if (wave > 0) {
        // The payload of block b is its L block and the g of the rows
        // b*CB + ring + [0, CB) that enter the window after it.  Register set
        // a holds even blocks, b odd ones; step s deposits block s + 1.
        const int li = tid - 64;
        cplx<T> la[C::EL], ra[C::ER], lb[C::EL], rb[C::ER];
        int off[C::EL];
        lds_offsets<CB, C::EL>(off, bp1, li);
        fetch<T, CB, C::EL, C::ER>(la, ra, base, 0, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
        deposit<T, C::EPB, C::ERB, C::EL, C::ER>(la, ra, off, slots, li);
        fetch<T, CB, C::EL, C::ER>(lb, rb, base, 1, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
        fetch<T, CB, C::EL, C::ER>(la, ra, base, 2, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
        __syncthreads();
        int cs = 0;                               // c0 of the current step, mod ring
        for (int s0 = 0; s0 < nbar; s0 += 2) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int s = s0 + h;
                T* dst = slots + ((s + 1) % NSLOT) * C::SLOT;
                if (h == 0) {
                    deposit<T, C::EPB, C::ERB, C::EL, C::ER>(lb, rb, off, dst, li);
                    fetch<T, CB, C::EL, C::ER>(lb, rb, base, s + 3, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
                } else {
                    deposit<T, C::EPB, C::ERB, C::EL, C::ER>(la, ra, off, dst, li);
                    fetch<T, CB, C::EL, C::ER>(la, ra, base, s + 3, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
                }
                // rows two or more blocks below block s - 1
                const int i = s - 1;
                if (i >= 0 && i < nblk) {
                    const T* LR = slots + (i % NSLOT) * C::SLOT;
                    const int yo = (i & 1) * CB * NRS;
                    forward_far_update<T, CB>(LR, LR + C::EPB, YR + yo, YI + yo, QR, QI, i * CB,
                                              min(CB, Mx - i * CB), Mx, bp, ls, nr, cs, ring, li);
                }
                __syncthreads();
                cs = wrap(cs + CB);
            }
        }
        return;
    }
    __syncthreads();

    // wave 0: the critical path
    const int k2 = lane % CB, grp = lane / CB;
    int cs = 0;
    for (int s = 0; s < nbar; ++s) {
        if (s < nblk) {
            const T* LR = slots + (s % NSLOT) * C::SLOT;
            const T* LI = LR + C::EPB;
            const T* SGR = LR + 2 * C::EPB;
            const T* SGI = SGR + C::ERB;
            T* YRs = YR + (s & 1) * CB * NRS;
            T* YIs = YI + (s & 1) * CB * NRS;
            const int c0 = s * CB;
            const int nb = min(CB, Mx - c0);
            // row k2 of the unit lower-triangular diagonal block, and D
            T lr[CB], lim[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const bool on = k < k2 && k2 - k <= bp && k < nb;
                const int d = min(max(k2 - k, 0), bp);
                lr[k] = on ? LR[k * ls + d] : T(0);
                lim[k] = on ? LI[k * ls + d] : T(0);
            }
            const cplx<T> dinv = cinv(cplx<T>{LR[k2 * ls], LI[k2 * ls]});
            const int qs = wrap(cs + k2) * NRS;
            for (int t0 = 0; t0 < nr; t0 += GPW) {
                const int t = t0 + grp;
                const int tt = min(t, nr - 1);
                T vr = QR[qs + tt] - PR[k2 * NRS + tt];
                T vi = QI[qs + tt] - PI[k2 * NRS + tt];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const T yr = group_bcast<CB>(vr, k, grp);
                    const T yi = group_bcast<CB>(vi, k, grp);
                    T nr_ = 0, ni_ = 0;
                    cmac(nr_, ni_, lr[k], lim[k], yr, yi);
                    vr -= nr_;
                    vi -= ni_;
                }
                if (t < nr) {
                    YRs[k2 * NRS + t] = vr;
                    YIs[k2 * NRS + t] = vi;
                    if (k2 < nb) {
                        const cplx<T> w = cmul(cplx<T>{vr, vi}, dinv);
                        wre[(size_t)t * rstride + c0 + k2] = w.re;
                        wim[(size_t)t * rstride + c0 + k2] = w.im;
                    }
                }
            }
            wave_lds_sync();
            // update of the next block's rows: P[j][t] = sum_k L[c0 + CB + j, c0 + k] y_k
            {
                const int j = lane % CB, part = lane / CB;
                for (int t = 0; t < nr; ++t) {
                    T ar = 0, ai = 0;
#pragma unroll
                    for (int kk = 0; kk < KPER; ++kk) {
                        const int k = part * KPER + kk;
                        const int dd = CB + j - k;
                        const bool on = k < nb && dd <= bp;
                        const int d = min(dd, bp);
                        const T yr = on ? YRs[k * NRS + t] : T(0), yi = on ? YIs[k * NRS + t] : T(0);
                        cmac(ar, ai, LR[k * ls + d], LI[k * ls + d], yr, yi);
                    }
                    for (int off = CB; off < 64; off <<= 1) {
                        ar += __shfl_xor(ar, off, 64);
                        ai += __shfl_xor(ai, off, 64);
                    }
                    if (part == 0) {
                        PR[j * NRS + t] = ar;
                        PI[j * NRS + t] = ai;
                    }
                }
            }
            // rows entering the window take the slots of the block's rows
            for (int q = lane; q < CB * NRS; q += 64) {
                const int slot = wrap(cs + q / NRS) * NRS + q % NRS;
                QR[slot] = SGR[q];
                QI[slot] = SGI[q];
            }
        }
        __syncthreads();
        cs = wrap(cs + CB);
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB, int BPC>
__global__ void __launch_bounds__(NT) sweep_backward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp,
                                                            int nsys, int nrhs, T* __restrict__ W) {
    using C = Cfg<T, CB, BPC>;
    constexpr int GPW = 64 / CB;
    constexpr int KPER = CB / GPW;                // rows per lane in the sums over the next block
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ls = bp + 2;                        // LDS column stride of L
    const int ring = bp + CB;
    T* slots = reinterpret_cast<T*>(smem_raw);
    T* ZR = slots + NSLOT * C::SLOT;              // finished z, ring [ring][NRS]
    T* ZI = ZR + ring * NRS;
    T* SR = ZI + ring * NRS;                      // off-block sums, [2][CB][NRS] by step parity
    T* SI = SR + 2 * CB * NRS;
    const int sys = blockIdx.x;
    const int r0 = blockIdx.y * NRS;
    const int nr = min(NRS, nrhs - r0);
    const cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const size_t rstride = (size_t)Mx * 2 * nsys;
    T* wre = W + (size_t)r0 * rstride + (size_t)sys * Mx;
    T* wim = W + (size_t)r0 * rstride + (size_t)(nsys + sys) * Mx;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nblk = (Mx + CB - 1) / CB;
    const int nbar = (nblk + 1) & ~1;
    auto wrap = [ring](int x) { return x >= ring ? x - ring : x; };

    for (int q = tid; q < ring * NRS; q += NT) {
        ZR[q] = 0;
        ZI[q] = 0;
    }
    for (int q = tid; q < 2 * CB * NRS; q += NT) {
        SR[q] = 0;
        SI[q] = 0;
    }
    const int cs0 = ((nblk - 1) * CB) % ring;     // c0 of the first block processed, mod ring

    if (wave > 0) {
        // step s processes block nblk - 1 - s; the payload of a block is its L
        // block and the w of its rows (stored q = k * NRS + t).  Step s
        // deposits the block of step s + 2.
        const int li = tid - 64;
        cplx<T> la[C::EL], ra[C::ER], lb[C::EL], rb[C::ER];
        int off[C::EL];
        lds_offsets<CB, C::EL>(off, bp1, li);
        fetch<T, CB, C::EL, C::ER>(la, ra, base, nblk - 1, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        fetch<T, CB, C::EL, C::ER>(lb, rb, base, nblk - 2, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        deposit<T, C::EPB, C::ERB, C::EL, C::ER>(la, ra, off, slots + 0 * C::SLOT, li);
        deposit<T, C::EPB, C::ERB, C::EL, C::ER>(lb, rb, off, slots + 1 * C::SLOT, li);
        fetch<T, CB, C::EL, C::ER>(la, ra, base, nblk - 3, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        fetch<T, CB, C::EL, C::ER>(lb, rb, base, nblk - 4, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        __syncthreads();
        int cs = cs0;
        for (int s0 = 0; s0 < nbar; s0 += 2) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int s = s0 + h;
                T* dst = slots + ((s + 2) % NSLOT) * C::SLOT;
                if (h == 0) {
                    deposit<T, C::EPB, C::ERB, C::EL, C::ER>(la, ra, off, dst, li);
                    fetch<T, CB, C::EL, C::ER>(la, ra, base, nblk - 1 - (s + 4), nblk, Mx, bp1, wre, wim, rstride,
                                               nr, 0, li);
                } else {
                    deposit<T, C::EPB, C::ERB, C::EL, C::ER>(lb, rb, off, dst, li);
                    fetch<T, CB, C::EL, C::ER>(lb, rb, base, nblk - 1 - (s + 4), nblk, Mx, bp1, wre, wim, rstride,
                                               nr, 0, li);
                }
                // sums over rows two or more blocks below the block of step s + 1
                const int a = nblk - 2 - s;
                if (a >= 0) {
                    const T* LR = slots + ((s + 1) % NSLOT) * C::SLOT;
                    const int so = ((s + 1) & 1) * CB * NRS;
                    backward_far_sums<T, CB>(LR, LR + C::EPB, ZR, ZI, SR + so, SI + so, a * CB, Mx, bp, ls, nr, cs,
                                             ring, li);
                }
                __syncthreads();
                cs = cs >= CB ? cs - CB : cs - CB + ring;
            }
        }
        return;
    }
    __syncthreads();

    // wave 0: the critical path
    const int kp = lane % CB, grp = lane / CB;
    int cs = cs0;
    for (int s = 0; s < nbar; ++s) {
        if (s < nblk) {
            const int blk = nblk - 1 - s;
            const T* LR = slots + (s % NSLOT) * C::SLOT;
            const T* LI = LR + C::EPB;
            const T* SWR = LR + 2 * C::EPB;
            const T* SWI = SWR + C::ERB;
            T* SRs = SR + (s & 1) * CB * NRS;
            T* SIs = SI + (s & 1) * CB * NRS;
            const int c0 = blk * CB;
            const int nb = min(CB, Mx - c0);
            // sums over the rows of the block below (finished in the previous step)
            {
                const int part = lane / CB;
                for (int t = 0; t < nr; ++t) {
                    T ar = 0, ai = 0;
#pragma unroll
                    for (int jj = 0; jj < KPER; ++jj) {
                        const int j = part * KPER + jj;
                        const int dd = CB + j - kp;
                        const bool on = kp < nb && dd <= bp && c0 + CB + j < Mx;
                        const int d = min(dd, bp);
                        const int slot = wrap(cs + CB + j) * NRS + t;
                        const T zr = on ? ZR[slot] : T(0), zi = on ? ZI[slot] : T(0);
                        cmac(ar, ai, LR[kp * ls + d], LI[kp * ls + d], zr, zi);
                    }
                    for (int off = CB; off < 64; off <<= 1) {
                        ar += __shfl_xor(ar, off, 64);
                        ai += __shfl_xor(ai, off, 64);
                    }
                    if (part == 0) {
                        SRs[kp * NRS + t] += ar;
                        SIs[kp * NRS + t] += ai;
                    }
                }
            }
            // column kp of the diagonal block (entries L[c0 + k, c0 + kp], k > kp)
            T lr[CB], lim[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const bool on = k > kp && k - kp <= bp && k < nb;
                const int d = min(max(k - kp, 0), bp);
                lr[k] = on ? LR[kp * ls + d] : T(0);
                lim[k] = on ? LI[kp * ls + d] : T(0);
            }
            wave_lds_sync();
            const int zs = wrap(cs + kp) * NRS;
            for (int t0 = 0; t0 < nr; t0 += GPW) {
                const int t = t0 + grp;
                const bool live = kp < nb && t < nr;
                const int tt = min(t, nr - 1);
                T vr = SWR[kp * NRS + tt] - SRs[kp * NRS + tt];
                T vi = SWI[kp * NRS + tt] - SIs[kp * NRS + tt];
#pragma unroll
                for (int kk = 0; kk < CB; ++kk) {
                    const int k = CB - 1 - kk;
                    const T zr = group_bcast<CB>(vr, k, grp);
                    const T zi = group_bcast<CB>(vi, k, grp);
                    T nr_ = 0, ni_ = 0;
                    cmac(nr_, ni_, lr[k], lim[k], zr, zi);
                    vr -= nr_;
                    vi -= ni_;
                }
                if (t < NRS) {
                    ZR[zs + t] = live ? vr : T(0);
                    ZI[zs + t] = live ? vi : T(0);
                }
                if (live) {
                    wre[(size_t)t * rstride + c0 + kp] = vr;
                    wim[(size_t)t * rstride + c0 + kp] = vi;
                }
            }
        }
        __syncthreads();
        cs = cs >= CB ? cs - CB : cs - CB + ring;
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB, int BPC>
static hipError_t launch_fwd(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                             hipStream_t st) {
    const size_t smem = smem_elems<T, CB, BPC>(bp) * sizeof(T);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_forward_kernel<T, CB, BPC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_forward_kernel<T, CB, BPC>), grid, dim3(NT), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<const T*>(G),
                       static_cast<T*>(W));
    return hipGetLastError();
}

template <typename T, int CB, int BPC>
static hipError_t launch_bwd(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st) {
    const size_t smem = smem_elems<T, CB, BPC>(bp) * sizeof(T);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_backward_kernel<T, CB, BPC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nsys, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_backward_kernel<T, CB, BPC>), grid, dim3(NT), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<T*>(W));
    return hipGetLastError();
}

// Block sizes keep a block near 4100 complex entries (32-64 KB) in every
// configuration: FP32 32 columns (bp <= 128) or 16 (bp <= 256), FP64 16 or 8.
template <typename T>
size_t sweep_smem(int bp) {
    if constexpr (sizeof(T) == 4)
        return bp <= 128 ? smem_elems<T, 32, 128>(bp) * 4 : smem_elems<T, 16, 256>(bp) * 4;
    else
        return bp <= 128 ? smem_elems<T, 16, 128>(bp) * 8 : smem_elems<T, 8, 256>(bp) * 8;
}

template <typename T>
hipError_t launch_band_forward(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                               hipStream_t st) {
    if (bp > BPMAX) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
        if (bp <= 128) return launch_fwd<T, 32, 128>(LB, Mx, bp, nsys, nrhs, G, W, st);
        return launch_fwd<T, 16, 256>(LB, Mx, bp, nsys, nrhs, G, W, st);
    } else {
        if (bp <= 128) return launch_fwd<T, 16, 128>(LB, Mx, bp, nsys, nrhs, G, W, st);
        return launch_fwd<T, 8, 256>(LB, Mx, bp, nsys, nrhs, G, W, st);
    }
}

template <typename T>
hipError_t launch_band_backward(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st) {
    if (bp > BPMAX) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
        if (bp <= 128) return launch_bwd<T, 32, 128>(LB, Mx, bp, nsys, nrhs, W, st);
        return launch_bwd<T, 16, 256>(LB, Mx, bp, nsys, nrhs, W, st);
    } else {
        if (bp <= 128) return launch_bwd<T, 16, 128>(LB, Mx, bp, nsys, nrhs, W, st);
        return launch_bwd<T, 8, 256>(LB, Mx, bp, nsys, nrhs, W, st);
    }
}

template hipError_t launch_band_forward<float>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_forward<double>(const void*, int, int, int, int, const void*, void*, hipStream_t);
template hipError_t launch_band_backward<float>(const void*, int, int, int, int, void*, hipStream_t);
template hipError_t launch_band_backward<double>(const void*, int, int, int, int, void*, hipStream_t);
template size_t sweep_smem<float>(int);
template size_t sweep_smem<double>(int);

}  // namespace stfd
