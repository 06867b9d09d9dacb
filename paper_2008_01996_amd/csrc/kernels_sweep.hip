// Triangular sweeps of step 3 of Algorithm FD (Sec. 4.4) with the band
// factors M_x + lambda_k A_x = L_k D_k L_k^T:
//     forward   L_k y = g_k,  w = D_k^-1 y
//     backward  L_k^T z_k = w
//
// Along one system the sweeps are a sequential chain of column blocks of CB
// columns, and every factor entry is read once.  One workgroup (4 or 8
// waves) runs one system for up to NRS right-hand sides:
//   * wave 0 runs the critical path of each block alone, with no barrier
//     inside the block: the CB x CB unit-triangular solve (one lane per row
//     and right-hand side, values passed on by lane broadcasts, the lane's
//     row of L held in registers) and the coupling to the adjacent block
//     (forward: the update of the next block's rows; backward: the sums over
//     the rows of the block just finished);
//   * the other (loader) waves stream the L entries of block i + 2 (with
//     the right-hand-side values that block needs) into one of three LDS
//     slots, their global loads issued two blocks ahead, and do the rest of
//     the band coupling one block off the critical path (forward: the update
//     of rows two or more blocks below by the block finished one step
//     earlier; backward: the sums over rows two or more blocks below for the
//     block processed next).
// One workgroup barrier per block hands slots and buffers over.  The pending
// values of the bp + CB rows a block can touch (forward), or the finished z
// of the rows below it (backward), live in an LDS ring.
//
// Band storage as in kernels_band.hip: LB[k][c][0] = D, LB[k][c][d] =
// L[c + d, c]; the CB columns of a block are contiguous.
// G/W layout per RHS: column-major M_x x 2 n_sys, real parts of system k in
// column k, imaginary parts in column n_sys + k.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace stfd {

namespace {

constexpr int NRS = 8;       // right-hand sides per workgroup
// kernel variants: any number of right-hand sides; the far band read once for
// all right-hand sides of a group; exactly one right-hand side; exactly one
// right-hand side and bp = BPC (every LDS offset a compile-time constant)
constexpr int MODE_ANY = 0, MODE_MULTI = 1, MODE_ONE = 2, MODE_ONE_EXACT = 3;
constexpr int NSLOT = 3;     // LDS block slots
constexpr int BPMAX = BAND_BPMAX;   // largest padded half-bandwidth

// NTH threads per workgroup: wave 0 runs the critical path, the NL lanes of
// the other NLW waves load blocks and apply the far band.
template <typename T, int CB, int BPC, int NTH>
struct Cfg {
    static constexpr int NT = NTH;
    static constexpr int NL = NTH - 64;
    static constexpr int NLW = NL / 64;
    static constexpr int EL = (CB * (BPC + 1) + NL - 1) / NL;  // L entries per loader lane
    static constexpr int ER = (CB * NRS + NL - 1) / NL;         // right-hand-side values per loader lane
    static constexpr int EPB = EL * NL + CB + 1;                // complex L entries of a slot, columns at stride bp + 2
    static constexpr int ZERO = EPB - 1;                        // a zero entry, never written by the loaders
    static constexpr int ERB = ER * NL;                         // right-hand-side values of a slot
    static constexpr int SLOT = 2 * EPB + 2 * ERB;              // T elements per slot: L (re, im interleaved),
                                                                // then right-hand-side re, im
};

// LDS carve-up: [NSLOT slots][ring re][ring im][block buffers: forward 2 x Y re/im + P re/im;
// backward 2 x NLW far-sum partials re/im + B re/im]
// (masked L reads below read the slot's zero entry instead of branching)
template <typename T, int CB, int BPC, int NTH>
__host__ __device__ constexpr size_t smem_elems(int bp) {
    using C = Cfg<T, CB, BPC, NTH>;
    return (size_t)NSLOT * C::SLOT + 2 * (size_t)(bp + CB) * NRS + (4 * (size_t)C::NLW + 2) * CB * NRS;
}

// Loader: global -> registers for block blk.  Addresses are clamped into the
// factor and right-hand-side arrays and the values are not masked, so the
// loads stay in flight until the registers are deposited two blocks later.
// Entries outside the block (columns past M_x, rows past M_x, right-hand
// sides past nrhs, blocks past the end) hold finite copies of valid entries;
// every use below masks them out.
template <typename T, int CB, int EL, int ER, int NL>
__device__ __forceinline__ void fetch(cplx<T> (&l)[EL], cplx<T> (&r)[ER], const cplx<T>* base, int blk, int nblk,
                                      int Mx, int bp1, const T* vre, const T* vim, size_t rstride, int nr, int rowoff,
                                      int li) {
    const int b = min(max(blk, 0), nblk - 1);
    const int c0 = b * CB;
    const int last = min(CB, Mx - c0) * bp1 - 1;
    const cplx<T>* src = base + (size_t)c0 * bp1;
    // field by field: a whole-struct copy of a 16-byte complex double stays a
    // memory copy that keeps l in scratch memory instead of registers
#pragma unroll
    for (int j = 0; j < EL; ++j) {
        const cplx<T>* e = src + min(li + NL * j, last);
        l[j].re = e->re;
        l[j].im = e->im;
    }
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
template <int CB, int EL, int NL>
__device__ __forceinline__ void lds_offsets(int (&off)[EL], int bp1, int li) {
#pragma unroll
    for (int j = 0; j < EL; ++j) {
        const int e = li + NL * j;
        off[j] = e + min(e / bp1, CB);
    }
}

// loader: registers -> LDS slot
template <typename T, int EPB, int ERB, int EL, int ER, int NL>
__device__ __forceinline__ void deposit(const cplx<T> (&l)[EL], const cplx<T> (&r)[ER], const int (&off)[EL],
                                        T* slot, int li) {
    cplx<T>* L = reinterpret_cast<cplx<T>*>(slot);
    T* GR = slot + 2 * EPB;
    T* GI = GR + ERB;
#pragma unroll
    for (int j = 0; j < EL; ++j) {
        L[off[j]].re = l[j].re;
        L[off[j]].im = l[j].im;
    }
#pragma unroll
    for (int j = 0; j < ER; ++j) {
        GR[li + NL * j] = r[j].re;
        GI[li + NL * j] = r[j].im;
    }
}

// Forward, off the critical path (loader waves): rows c0 + CB + rr, rr in
// [CB, bp), of the pending ring take the update by block (c0, nb) with its
// solution y.  cs = (c0 + CB) mod ring.  With PW > 1 the CB columns of a row
// are split over PW lanes 64 / PW apart in a wave.
template <typename T, int CB, int PW, int NL>
__device__ __forceinline__ void forward_far_update(const cplx<T>* L, const T* YR, const T* YI, T* QR, T* QI, int c0,
                                                   int nb, int Mx, int bp, int ls, int nr, int cs, int ring, int zero,
                                                   int li) {
    constexpr int KP = CB / PW;                   // columns per lane
    constexpr int IPP = NL / PW;                  // rows per pass
    constexpr int LPP = 64 / PW;                  // rows per wave and pass
    const int part = (li & 63) / LPP;
    const int slot_item = (li >> 6) * LPP + (li & (LPP - 1));
    const int nrow = bp - CB;
    for (int t = 0; t < nr; ++t) {
        for (int m0 = 0; m0 < nrow; m0 += IPP) {
            const int m = m0 + slot_item;
            const int rr = CB + m;
            const bool row_ok = m < nrow && c0 + CB + rr < Mx;
            const int kmin = CB + rr - bp;        // L[row, c0 + k] lies in the band for k >= kmin
            T ar = 0, ai = 0;
#pragma unroll
            for (int kk = 0; kk < KP; ++kk) {
                const int k = part * KP + kk;
                const int e = row_ok && k < nb && k >= kmin ? k * ls + CB + rr - k : zero;
                const cplx<T> l = L[e];
                cmac(ar, ai, l.re, l.im, YR[k * NRS + t], YI[k * NRS + t]);
            }
#pragma unroll
            for (int off = LPP; off < 64; off <<= 1) {
                ar += __shfl_xor(ar, off, 64);
                ai += __shfl_xor(ai, off, 64);
            }
            if (row_ok && part == 0) {
                int s = cs + rr;
                s = s >= ring ? s - ring : s;
                QR[s * NRS + t] -= ar;
                QI[s * NRS + t] -= ai;
            }
        }
    }
}

// The same for several right-hand sides at once: each L entry is read once
// and applied to all NRS of them (right-hand sides past nr see zero y).
template <typename T, int CB, int PW, int NL>
__device__ __forceinline__ void forward_far_update_multi(const cplx<T>* L, const T* YR, const T* YI, T* QR, T* QI,
                                                         int c0, int nb, int Mx, int bp, int ls, int nr, int cs,
                                                         int ring, int zero, int li) {
    constexpr int KP = CB / PW;
    constexpr int IPP = NL / PW;
    constexpr int LPP = 64 / PW;                  // rows per wave and pass
    const int part = (li & 63) / LPP;
    const int slot_item = (li >> 6) * LPP + (li & (LPP - 1));
    const int nrow = bp - CB;
    for (int m0 = 0; m0 < nrow; m0 += IPP) {
        const int m = m0 + slot_item;
        const int rr = CB + m;
        const bool row_ok = m < nrow && c0 + CB + rr < Mx;
        const int kmin = CB + rr - bp;
        T ar[NRS], ai[NRS];
#pragma unroll
        for (int t = 0; t < NRS; ++t) ar[t] = ai[t] = T(0);
#pragma unroll 4
        for (int kk = 0; kk < KP; ++kk) {
            const int k = part * KP + kk;
            const int e = row_ok && k < nb && k >= kmin ? k * ls + CB + rr - k : zero;
            const cplx<T> l = L[e];
#pragma unroll
            for (int t = 0; t < NRS; ++t) cmac(ar[t], ai[t], l.re, l.im, YR[k * NRS + t], YI[k * NRS + t]);
        }
#pragma unroll
        for (int t = 0; t < NRS; ++t)
#pragma unroll
            for (int off = LPP; off < 64; off <<= 1) {
                ar[t] += __shfl_xor(ar[t], off, 64);
                ai[t] += __shfl_xor(ai[t], off, 64);
            }
        if (row_ok && part == 0) {
            int s = cs + rr;
            s = s >= ring ? s - ring : s;
#pragma unroll
            for (int t = 0; t < NRS; ++t)
                if (t < nr) {
                    QR[s * NRS + t] -= ar[t];
                    QI[s * NRS + t] -= ai[t];
                }
        }
    }
}

// Backward, off the critical path (loader waves): for the full block at c0 and
// every column k, partial sums over rows r = c0 + 2 CB + m (m < bp - CB) of
// L[r, c0 + k] z[r][t].  Lane li takes column k = li % CB and the RPC rows of
// chunk li / CB; the chunks of a wave are added by shuffles and loader wave w
// writes its partial to S[w][k][t].  cs = (c0 + CB) mod ring.
template <typename T, int CB, int RPC>
__device__ __forceinline__ void backward_far_sums(const cplx<T>* L, const T* ZR, const T* ZI, T* SR, T* SI, int c0,
                                                  int Mx, int bp, int ls, int nr, int cs, int ring, int zero,
                                                  int li) {
    const int k = li % CB, ch = li / CB, w = li >> 6;
    const int nrow = bp - CB;
    for (int t = 0; t < nr; ++t) {
        T ar = 0, ai = 0;
#pragma unroll
        for (int i = 0; i < RPC; ++i) {
            const int m = ch * RPC + i;
            const int d = 2 * CB + m - k;          // r - (c0 + k)
            const bool on = m < nrow && d <= bp && c0 + 2 * CB + m < Mx;
            const cplx<T> l = L[on ? k * ls + d : zero];
            int sl = cs + CB + min(m, max(nrow - 1, 0));
            sl = sl >= ring ? sl - ring : sl;
            cmac(ar, ai, l.re, l.im, ZR[sl * NRS + t], ZI[sl * NRS + t]);
        }
        for (int off = CB; off < 64; off <<= 1) {
            ar += __shfl_xor(ar, off, 64);
            ai += __shfl_xor(ai, off, 64);
        }
        if ((li & 63) < CB) {
            SR[(w * CB + k) * NRS + t] = ar;
            SI[(w * CB + k) * NRS + t] = ai;
        }
    }
}

// The same for several right-hand sides at once (each L entry read once;
// finished z of right-hand sides past nr are zero).
template <typename T, int CB, int RPC>
__device__ __forceinline__ void backward_far_sums_multi(const cplx<T>* L, const T* ZR, const T* ZI, T* SR, T* SI,
                                                        int c0, int Mx, int bp, int ls, int nr, int cs, int ring,
                                                        int zero, int li) {
    const int k = li % CB, ch = li / CB, w = li >> 6;
    const int nrow = bp - CB;
    T ar[NRS], ai[NRS];
#pragma unroll
    for (int t = 0; t < NRS; ++t) ar[t] = ai[t] = T(0);
#pragma unroll 4
    for (int i = 0; i < RPC; ++i) {
        const int m = ch * RPC + i;
        const int d = 2 * CB + m - k;
        const bool on = m < nrow && d <= bp && c0 + 2 * CB + m < Mx;
        const cplx<T> l = L[on ? k * ls + d : zero];
        int sl = cs + CB + min(m, max(nrow - 1, 0));
        sl = sl >= ring ? sl - ring : sl;
#pragma unroll
        for (int t = 0; t < NRS; ++t) cmac(ar[t], ai[t], l.re, l.im, ZR[sl * NRS + t], ZI[sl * NRS + t]);
    }
#pragma unroll
    for (int t = 0; t < NRS; ++t)
        for (int off = CB; off < 64; off <<= 1) {
            ar[t] += __shfl_xor(ar[t], off, 64);
            ai[t] += __shfl_xor(ai[t], off, 64);
        }
    if ((li & 63) < CB) {
#pragma unroll
        for (int t = 0; t < NRS; ++t)
            if (t < nr) {
                SR[(w * CB + k) * NRS + t] = ar[t];
                SI[(w * CB + k) * NRS + t] = ai[t];
            }
    }
}

// Broadcast of lane k of this lane's group of CB lanes (G groups; G = 1:
// lane k of the wave).
template <typename T, int CB, int G>
__device__ __forceinline__ T bcast(T v, int k, int grp) {
    if constexpr (G == 1)
        return lane_bcast(v, k);
    else
        return group_bcast<CB>(v, k, grp);
}

// Chain over the CB rows of a diagonal block (ascending for the forward
// sweep, descending for the backward one): v -= l[k] * v_k, with v_k
// broadcast from lane k of the group once it is final.  A lane whose l[k]
// are zero for the rows not yet final solves its row; a lane with v = 0
// that holds other entries of L collects -sum_k l[k] v_k.
template <typename T, int CB, int G, bool DESC>
__device__ __forceinline__ void chain(T& vr, T& vi, const cplx<T> (&l)[CB], int grp) {
#pragma unroll
    for (int kk = 0; kk < CB; ++kk) {
        const int k = DESC ? CB - 1 - kk : kk;
        const T yr = bcast<T, CB, G>(vr, k, grp);
        const T yi = bcast<T, CB, G>(vi, k, grp);
        vr = fma(-l[k].re, yr, vr);
        vr = fma(l[k].im, yi, vr);
        vi = fma(-l[k].re, yi, vi);
        vi = fma(-l[k].im, yr, vi);
    }
}

// The same chain, also collecting a += sum_k p[k] v_k in the same lane.
template <typename T, int CB, int G, bool DESC>
__device__ __forceinline__ void chain2(T& vr, T& vi, T& ar, T& ai, const cplx<T> (&l)[CB], const cplx<T> (&p)[CB],
                                       int grp) {
#pragma unroll
    for (int kk = 0; kk < CB; ++kk) {
        const int k = DESC ? CB - 1 - kk : kk;
        const T yr = bcast<T, CB, G>(vr, k, grp);
        const T yi = bcast<T, CB, G>(vi, k, grp);
        vr = fma(-l[k].re, yr, vr);
        vr = fma(l[k].im, yi, vr);
        vi = fma(-l[k].re, yi, vi);
        vi = fma(-l[k].im, yr, vi);
        cmac(ar, ai, p[k].re, p[k].im, yr, yi);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
template <typename T, int CB, int BPC, int MODE, int NTH>
__global__ void __launch_bounds__(NTH) sweep_forward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp_in,
                                                           int nsys, int nrhs, const T* __restrict__ G,
                                                           T* __restrict__ W, int sys0, const int* __restrict__ gate) {
    if (gate && *gate) return;
    using C = Cfg<T, CB, BPC, NTH>;
    constexpr bool ONE = MODE == MODE_ONE || MODE == MODE_ONE_EXACT;
    const int bp = MODE == MODE_ONE_EXACT ? BPC : bp_in;
    constexpr int GPW = 64 / CB;                  // right-hand sides per chain pass
    // who copies the rows entering the pending window into the ring: the
    // loaders, a step after the block, where that measured faster (FP32 with
    // several right-hand sides; needs bp >= CB), else wave 0 at the block's end
    constexpr bool LOADER_ENTER = sizeof(T) == 4 && !ONE;
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
    const int sys = sys0 + blockIdx.x;             // systems sys0 .. sys0 + gridDim.x - 1
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
    for (int q = tid; q < ring * NRS; q += C::NT) {
        const int row = q / NRS, t = q % NRS;
        T re = 0, im = 0;
        if (row < Mx && t < nr) {
            re = gre[(size_t)t * rstride + row];
            im = gim[(size_t)t * rstride + row];
        }
        QR[q] = re;
        QI[q] = im;
    }
    for (int q = tid; q < CB * NRS; q += C::NT) {
        PR[q] = 0;
        PI[q] = 0;
    }
    for (int q = tid; q < 2 * CB * NRS; q += C::NT) {     // right-hand sides past nr stay zero
        YR[q] = 0;
        YI[q] = 0;
    }

    for (int q = tid; q < NSLOT; q += C::NT) reinterpret_cast<cplx<T>*>(slots + q * C::SLOT)[C::ZERO] = cplx<T>{0, 0};

    if (wave > 0) {
        // The payload of block b is its L block and the g of the rows
        // b*CB + ring + [0, CB) that enter the window after it.  Register set
        // a holds even blocks, b odd ones; step s deposits block s + 1.
        const int li = tid - 64;
        cplx<T> la[C::EL], ra[C::ER], lb[C::EL], rb[C::ER];
        int off[C::EL];
        lds_offsets<CB, C::EL, C::NL>(off, bp1, li);
        fetch<T, CB, C::EL, C::ER, C::NL>(la, ra, base, 0, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
        deposit<T, C::EPB, C::ERB, C::EL, C::ER, C::NL>(la, ra, off, slots, li);
        fetch<T, CB, C::EL, C::ER, C::NL>(lb, rb, base, 1, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
        fetch<T, CB, C::EL, C::ER, C::NL>(la, ra, base, 2, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
        __syncthreads();
        int cs = 0;                               // c0 of the current step, mod ring
        // One step on register set (lx, rx).  The two sets are passed in
        // straight-line calls, never chosen by a branch, so that both stay in
        // registers (a choice between them would put them in scratch memory).
        auto step = [&](int s, cplx<T>(&lx)[C::EL], cplx<T>(&rx)[C::ER]) {
            T* dst = slots + ((s + 1) % NSLOT) * C::SLOT;
            deposit<T, C::EPB, C::ERB, C::EL, C::ER, C::NL>(lx, rx, off, dst, li);
            fetch<T, CB, C::EL, C::ER, C::NL>(lx, rx, base, s + 3, nblk, Mx, bp1, gre, gim, rstride, nr, ring, li);
            if (LOADER_ENTER && bp >= CB && s >= 1 && s <= nblk) {
                // the rows entering the window after block s - 1 take the
                // ring slots of its rows (first read by the far update of
                // block s, next step; with bp < CB some of them belong to
                // block s itself, and wave 0 copies them in step s - 1)
                const T* SGR = slots + ((s - 1) % NSLOT) * C::SLOT + 2 * C::EPB;
                const T* SGI = SGR + C::ERB;
                const int csp = cs >= CB ? cs - CB : cs - CB + ring;
                for (int q = li; q < CB * NRS; q += C::NL) {
                    const int sl = wrap(csp + q / NRS) * NRS + q % NRS;
                    QR[sl] = SGR[q];
                    QI[sl] = SGI[q];
                }
            }
            {
                // rows two or more blocks below block s - 1
                const int i = s - 1;
                if (i >= 0 && i < nblk) {
                    const T* LR = slots + (i % NSLOT) * C::SLOT;
                    const int yo = (i & 1) * CB * NRS;
                    const cplx<T>* L = reinterpret_cast<const cplx<T>*>(LR);
                    const int nbi = min(CB, Mx - i * CB);
                    // lanes per row: as many as the rows leave room for
                    auto far = [&](auto PWc) {
                        constexpr int PW = decltype(PWc)::value;
                        if constexpr (MODE == MODE_MULTI)
                            forward_far_update_multi<T, CB, PW, C::NL>(L, YR + yo, YI + yo, QR, QI, i * CB, nbi, Mx,
                                                                       bp, ls, nr, cs, ring, C::ZERO, li);
                        else
                            forward_far_update<T, CB, PW, C::NL>(L, YR + yo, YI + yo, QR, QI, i * CB, nbi, Mx, bp,
                                                                 ls, nr, cs, ring, C::ZERO, li);
                    };
                    // (fixed at compile time where it holds for every bp <= BPC)
                    if constexpr (CB >= 4 && C::NL >= 4 * (BPC - CB))
                        far(std::integral_constant<int, 4>{});
                    else if constexpr (C::NL >= 2 * (BPC - CB))
                        far(std::integral_constant<int, 2>{});
                    else if ((bp - CB) * 2 <= C::NL)
                        far(std::integral_constant<int, 2>{});
                    else
                        far(std::integral_constant<int, 1>{});
                }
            }
            __syncthreads();
            cs = wrap(cs + CB);
        };
        for (int s0 = 0; s0 < nbar; s0 += 2) {
            step(s0, lb, rb);
            step(s0 + 1, la, ra);
        }
        return;
    }
    __syncthreads();

    // wave 0: the critical path
    const int k2 = lane % CB, grp = lane / CB;
    constexpr int ZERO = C::ZERO;
    int cs = 0;
    for (int s = 0; s < nbar; ++s) {
        if (s < nblk) {
            const T* slot = slots + (s % NSLOT) * C::SLOT;
            const cplx<T>* L = reinterpret_cast<const cplx<T>*>(slot);
            const T* SGR = slot + 2 * C::EPB;
            const T* SGI = SGR + C::ERB;
            T* YRs = YR + (s & 1) * CB * NRS;
            T* YIs = YI + (s & 1) * CB * NRS;
            const int c0 = s * CB;
            const int nb = min(CB, Mx - c0);
            const cplx<T> dinv = cinv_fast(L[k2 * ls]);
            const int qs = wrap(cs + k2) * NRS;
            auto put_y = [&](int t, T vr, T vi) {
                YRs[k2 * NRS + t] = vr;
                YIs[k2 * NRS + t] = vi;
                if (k2 < nb) {
                    const cplx<T> w = cmul(cplx<T>{vr, vi}, dinv);
                    wre[(size_t)t * rstride + c0 + k2] = w.re;
                    wim[(size_t)t * rstride + c0 + k2] = w.im;
                }
            };
            if (ONE || nr == 1) {
                // group 0: row k2 of the unit lower-triangular diagonal block;
                // group 1: row k2 of the block below (collects -P)
                cplx<T> l[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const int dd = grp * CB + k2 - k;
                    l[k] = L[grp < 2 && dd > 0 && dd <= bp && k < nb ? k * ls + dd : ZERO];
                }
                T vr = 0, vi = 0;
                if (grp == 0) {
                    vr = QR[qs] - PR[k2 * NRS];
                    vi = QI[qs] - PI[k2 * NRS];
                }
                chain<T, CB, 1, false>(vr, vi, l, grp);
                wave_lds_sync();
                if (grp == 0) put_y(0, vr, vi);
                if (grp == 1) {
                    PR[k2 * NRS] = -vr;
                    PI[k2 * NRS] = -vi;
                }
            } else if constexpr (!ONE) {
                cplx<T> l[CB], p[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const int da = k2 - k, db = CB + k2 - k;
                    l[k] = L[da > 0 && da <= bp && k < nb ? k * ls + da : ZERO];
                    p[k] = L[db <= bp && k < nb ? k * ls + db : ZERO];
                }
                for (int t0 = 0; t0 < nr; t0 += GPW) {
                    const int t = t0 + grp;
                    const int tt = min(t, nr - 1);
                    T vr = QR[qs + tt] - PR[k2 * NRS + tt], vi = QI[qs + tt] - PI[k2 * NRS + tt];
                    T ar = 0, ai = 0;
                    chain2<T, CB, GPW, false>(vr, vi, ar, ai, l, p, grp);
                    if (t < nr) {
                        put_y(t, vr, vi);
                        PR[k2 * NRS + t] = ar;
                        PI[k2 * NRS + t] = ai;
                    }
                }
            }
            if (!LOADER_ENTER || bp < CB) {
                // the rows entering the window take the slots of the block's
                // rows (with one right-hand side only its slot t = 0)
                wave_lds_sync();
                if constexpr (ONE) {
                    if (lane < CB) {
                        const int sl = wrap(cs + lane) * NRS;
                        QR[sl] = SGR[lane * NRS];
                        QI[sl] = SGI[lane * NRS];
                    }
                } else {
                    for (int q = lane; q < CB * NRS; q += 64) {
                        const int sl = wrap(cs + q / NRS) * NRS + q % NRS;
                        QR[sl] = SGR[q];
                        QI[sl] = SGI[q];
                    }
                }
            }
        }
        __syncthreads();
        cs = wrap(cs + CB);
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB, int BPC, int MODE, int NTH>
__global__ void __launch_bounds__(NTH) sweep_backward_kernel(const cplx<T>* __restrict__ LB, int Mx, int bp_in,
                                                            int nsys, int nrhs, T* __restrict__ W, int sys0,
                                                            const int* __restrict__ gate) {
    if (gate && *gate) return;
    using C = Cfg<T, CB, BPC, NTH>;
    constexpr bool ONE = MODE == MODE_ONE || MODE == MODE_ONE_EXACT;
    const int bp = MODE == MODE_ONE_EXACT ? BPC : bp_in;
    constexpr int GPW = 64 / CB;
    extern __shared__ unsigned char smem_raw[];
    const int bp1 = bp + 1;
    const int ls = bp + 2;                        // LDS column stride of L
    const int ring = bp + CB;
    T* slots = reinterpret_cast<T*>(smem_raw);
    T* ZR = slots + NSLOT * C::SLOT;              // finished z, ring [ring][NRS]
    T* ZI = ZR + ring * NRS;
    constexpr int NP = C::NLW;                    // far-sum partials, one per loader wave
    T* SR = ZI + ring * NRS;                      // far-sum partials, [2][NP][CB][NRS] by step parity
    T* SI = SR + 2 * NP * CB * NRS;
    T* BR = SI + 2 * NP * CB * NRS;               // sums over the block just finished, [CB][NRS]
    T* BI = BR + CB * NRS;
    const int sys = sys0 + blockIdx.x;             // systems sys0 .. sys0 + gridDim.x - 1
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

    for (int q = tid; q < ring * NRS; q += C::NT) {
        ZR[q] = 0;
        ZI[q] = 0;
    }
    for (int q = tid; q < 2 * NP * CB * NRS; q += C::NT) {
        SR[q] = 0;
        SI[q] = 0;
    }
    for (int q = tid; q < CB * NRS; q += C::NT) {
        BR[q] = 0;
        BI[q] = 0;
    }
    const int cs0 = ((nblk - 1) * CB) % ring;     // c0 of the first block processed, mod ring

    for (int q = tid; q < NSLOT; q += C::NT) reinterpret_cast<cplx<T>*>(slots + q * C::SLOT)[C::ZERO] = cplx<T>{0, 0};

    if (wave > 0) {
        // step s processes block nblk - 1 - s; the payload of a block is its L
        // block and the w of its rows (stored q = k * NRS + t).  Step s
        // deposits the block of step s + 2.
        const int li = tid - 64;
        cplx<T> la[C::EL], ra[C::ER], lb[C::EL], rb[C::ER];
        int off[C::EL];
        lds_offsets<CB, C::EL, C::NL>(off, bp1, li);
        fetch<T, CB, C::EL, C::ER, C::NL>(la, ra, base, nblk - 1, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        fetch<T, CB, C::EL, C::ER, C::NL>(lb, rb, base, nblk - 2, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        deposit<T, C::EPB, C::ERB, C::EL, C::ER, C::NL>(la, ra, off, slots + 0 * C::SLOT, li);
        deposit<T, C::EPB, C::ERB, C::EL, C::ER, C::NL>(lb, rb, off, slots + 1 * C::SLOT, li);
        fetch<T, CB, C::EL, C::ER, C::NL>(la, ra, base, nblk - 3, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        fetch<T, CB, C::EL, C::ER, C::NL>(lb, rb, base, nblk - 4, nblk, Mx, bp1, wre, wim, rstride, nr, 0, li);
        __syncthreads();
        int cs = cs0;
        // one step on register set (lx, rx), straight-line calls as in the forward sweep
        auto step = [&](int s, cplx<T>(&lx)[C::EL], cplx<T>(&rx)[C::ER]) {
            T* dst = slots + ((s + 2) % NSLOT) * C::SLOT;
            deposit<T, C::EPB, C::ERB, C::EL, C::ER, C::NL>(lx, rx, off, dst, li);
            fetch<T, CB, C::EL, C::ER, C::NL>(lx, rx, base, nblk - 1 - (s + 4), nblk, Mx, bp1, wre, wim, rstride, nr, 0,
                                       li);
            {
                // sums over rows two or more blocks below the block of step s + 1
                const int a = nblk - 2 - s;
                if (a >= 0) {
                    const T* LR = slots + ((s + 1) % NSLOT) * C::SLOT;
                    const int so = ((s + 1) & 1) * NP * CB * NRS;
                    constexpr int RPC = (BPC - CB + C::NL / CB - 1) / (C::NL / CB);
                    if constexpr (MODE == MODE_MULTI)
                        backward_far_sums_multi<T, CB, RPC>(reinterpret_cast<const cplx<T>*>(LR), ZR, ZI, SR + so,
                                                            SI + so, a * CB, Mx, bp, ls, nr, cs, ring, C::ZERO, li);
                    else
                        backward_far_sums<T, CB, RPC>(reinterpret_cast<const cplx<T>*>(LR), ZR, ZI, SR + so, SI + so,
                                                      a * CB, Mx, bp, ls, nr, cs, ring, C::ZERO, li);
                }
            }
            __syncthreads();
            cs = cs >= CB ? cs - CB : cs - CB + ring;
        };
        for (int s0 = 0; s0 < nbar; s0 += 2) {
            step(s0, la, ra);
            step(s0 + 1, lb, rb);
        }
        return;
    }
    __syncthreads();

    // wave 0: the critical path
    const int kp = lane % CB, grp = lane / CB;
    constexpr int ZERO = C::ZERO;
    int cs = cs0;
    for (int s = 0; s < nbar; ++s) {
        if (s < nblk) {
            const int blk = nblk - 1 - s;
            const T* slot = slots + (s % NSLOT) * C::SLOT;
            const cplx<T>* L = reinterpret_cast<const cplx<T>*>(slot);
            // block blk - 1, deposited a step ago
            const cplx<T>* LN = reinterpret_cast<const cplx<T>*>(slots + ((s + 1) % NSLOT) * C::SLOT);
            const T* SWR = slot + 2 * C::EPB;
            const T* SWI = SWR + C::ERB;
            const T* SRs = SR + (s & 1) * NP * CB * NRS;  // far sums: NP partials
            const T* SIs = SI + (s & 1) * NP * CB * NRS;
            auto far_r = [&](int q) {
                T v = SRs[q];
#pragma unroll
                for (int w = 1; w < NP; ++w) v += SRs[w * CB * NRS + q];
                return v;
            };
            auto far_i = [&](int q) {
                T v = SIs[q];
#pragma unroll
                for (int w = 1; w < NP; ++w) v += SIs[w * CB * NRS + q];
                return v;
            };
            const int c0 = blk * CB;
            const int nb = min(CB, Mx - c0);
            const int zs = wrap(cs + kp) * NRS;
            auto put_z = [&](int t, bool live, T vr, T vi) {
                ZR[zs + t] = live ? vr : T(0);
                ZI[zs + t] = live ? vi : T(0);
                if (live) {
                    wre[(size_t)t * rstride + c0 + kp] = vr;
                    wim[(size_t)t * rstride + c0 + kp] = vi;
                }
            };
            if (ONE || nr == 1) {
                // group 0: column kp of the diagonal block (rows c0 + k);
                // group 1: column kp of the block to the left (collects -B)
                const cplx<T>* src = grp == 0 ? L : LN;
                cplx<T> l[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const int dd = grp * CB + k - kp;
                    const bool on = grp < 2 && dd > 0 && dd <= bp && k < nb && (grp == 0 || blk > 0);
                    l[k] = src[on ? kp * ls + dd : ZERO];
                }
                const bool live = kp < nb;
                T vr = 0, vi = 0;
                if (grp == 0 && live) {
                    vr = SWR[kp * NRS] - far_r(kp * NRS) - BR[kp * NRS];
                    vi = SWI[kp * NRS] - far_i(kp * NRS) - BI[kp * NRS];
                }
                chain<T, CB, 1, true>(vr, vi, l, grp);
                wave_lds_sync();
                if (grp == 0) put_z(0, live, vr, vi);
                if (grp == 1) {
                    BR[kp * NRS] = -vr;
                    BI[kp * NRS] = -vi;
                }
            } else if constexpr (!ONE) {
                cplx<T> l[CB], p[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const int da = k - kp, db = CB + k - kp;
                    l[k] = L[da > 0 && da <= bp && k < nb ? kp * ls + da : ZERO];
                    p[k] = LN[blk > 0 && db <= bp && k < nb ? kp * ls + db : ZERO];
                }
                for (int t0 = 0; t0 < nr; t0 += GPW) {
                    const int t = t0 + grp;
                    const bool live = kp < nb && t < nr;
                    const int tt = min(t, nr - 1);
                    T vr = live ? SWR[kp * NRS + tt] - far_r(kp * NRS + tt) - BR[kp * NRS + tt] : T(0);
                    T vi = live ? SWI[kp * NRS + tt] - far_i(kp * NRS + tt) - BI[kp * NRS + tt] : T(0);
                    T ar = 0, ai = 0;
                    chain2<T, CB, GPW, true>(vr, vi, ar, ai, l, p, grp);
                    if (t < NRS) {
                        put_z(t, live, vr, vi);
                        BR[kp * NRS + t] = ar;
                        BI[kp * NRS + t] = ai;
                    }
                }
            }
        }
        __syncthreads();
        cs = cs >= CB ? cs - CB : cs - CB + ring;
    }
}

// ---------------------------------------------------------------------------
template <typename T, int CB, int BPC, int MODE, int NTH>
static hipError_t launch_fwd(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                             hipStream_t st, int sys0, int nrun) {
    const size_t smem = smem_elems<T, CB, BPC, NTH>(bp) * sizeof(T);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_forward_kernel<T, CB, BPC, MODE, NTH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nrun, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_forward_kernel<T, CB, BPC, MODE, NTH>), grid, dim3(NTH), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<const T*>(G),
                       static_cast<T*>(W), sys0, launch_gate());
    return hipGetLastError();
}

template <typename T, int CB, int BPC, int MODE, int NTH>
static hipError_t launch_bwd(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st, int sys0,
                             int nrun) {
    const size_t smem = smem_elems<T, CB, BPC, NTH>(bp) * sizeof(T);
    hipError_t e = hipFuncSetAttribute((const void*)sweep_backward_kernel<T, CB, BPC, MODE, NTH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    dim3 grid(nrun, (nrhs + NRS - 1) / NRS);
    hipLaunchKernelGGL((sweep_backward_kernel<T, CB, BPC, MODE, NTH>), grid, dim3(NTH), smem, st,
                       static_cast<const cplx<T>*>(LB), Mx, bp, nsys, nrhs, static_cast<T*>(W), sys0, launch_gate());
    return hipGetLastError();
}

// Configurations (block columns CB, threads per workgroup) by precision,
// band and right-hand-side count, as measured fastest.  A block holds near
// 4100 complex entries (CB = 32 FP32 / 16 FP64 for bp <= 128, half that for
// bp <= 256).  One right-hand side has a variant of its own, without the
// registers of the general chain; in FP32 it runs seven loader waves (two
// waves on every SIMD, one issuing while the other waits), and so does the
// forward sweep from five right-hand sides on; the FP64 slots leave LDS room
// for three.  With three or more right-hand sides the backward sweep's
// diagonal chain (work per column proportional to nrhs * CB) bounds it and
// its blocks halve.  From five (forward) and six (backward) right-hand sides
// on, the far band is read once for all right-hand sides of a group.
constexpr int MULTI_RHS = 3;
constexpr int FWD_MULTI_MIN = 5;
constexpr int BWD_MULTI_MIN = 6;

// general or multi-right-hand-side variant by the right-hand-side count
template <typename T, int CB, int BPC, int NTH>
static hipError_t launch_fwd_rhs(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                                 hipStream_t st, int sys0, int nrun) {
    return nrhs >= FWD_MULTI_MIN ? launch_fwd<T, CB, BPC, MODE_MULTI, NTH>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun)
                                 : launch_fwd<T, CB, BPC, MODE_ANY, NTH>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
}

template <typename T, int CB, int BPC, int NTH>
static hipError_t launch_bwd_rhs(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st,
                                 int sys0, int nrun) {
    return nrhs >= BWD_MULTI_MIN ? launch_bwd<T, CB, BPC, MODE_MULTI, NTH>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun)
                                 : launch_bwd<T, CB, BPC, MODE_ANY, NTH>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
}

template <typename T>
size_t sweep_smem(int bp) {
    if constexpr (sizeof(T) == 4)
        return bp <= 128 ? std::max({smem_elems<T, 32, 128, 512>(bp), smem_elems<T, 16, 128, 512>(bp),
                                     smem_elems<T, 32, 128, 256>(bp), smem_elems<T, 16, 128, 256>(bp)}) * 4
                         : smem_elems<T, 16, 256, 256>(bp) * 4;
    else
        return bp <= 128 ? std::max(smem_elems<T, 16, 128, 256>(bp), smem_elems<T, 8, 128, 256>(bp)) * 8
                         : smem_elems<T, 8, 256, 256>(bp) * 8;
}

template <typename T>
hipError_t launch_band_forward(const void* LB, int Mx, int bp, int nsys, int nrhs, const void* G, void* W,
                               hipStream_t st, int sys0, int nrun) {
    if (bp > BPMAX || sys0 < 0 || nrun < 1 || sys0 + nrun > nsys) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
        if (bp == 128 && nrhs == 1)
            return launch_fwd<T, 32, 128, MODE_ONE_EXACT, 512>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
        if (bp <= 128 && nrhs == 1) return launch_fwd<T, 32, 128, MODE_ONE, 512>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
        if (bp <= 128 && nrhs < FWD_MULTI_MIN)
            return launch_fwd<T, 32, 128, MODE_ANY, 256>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
        if (bp <= 128) return launch_fwd<T, 16, 128, MODE_MULTI, 512>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
        return launch_fwd_rhs<T, 16, 256, 256>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
    } else {
        if (bp == 128 && nrhs == 1)
            return launch_fwd<T, 16, 128, MODE_ONE_EXACT, 256>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
        if (bp <= 128 && nrhs == 1) return launch_fwd<T, 16, 128, MODE_ONE, 256>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
        if (bp <= 128) return launch_fwd_rhs<T, 16, 128, 256>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
        return launch_fwd_rhs<T, 8, 256, 256>(LB, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun);
    }
}

template <typename T>
hipError_t launch_band_backward(const void* LB, int Mx, int bp, int nsys, int nrhs, void* W, hipStream_t st,
                                int sys0, int nrun) {
    if (bp > BPMAX || sys0 < 0 || nrun < 1 || sys0 + nrun > nsys) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
        if (bp == 128 && nrhs == 1)
            return launch_bwd<T, 32, 128, MODE_ONE_EXACT, 512>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        if (bp <= 128 && nrhs == 1) return launch_bwd<T, 32, 128, MODE_ONE, 512>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        if (bp <= 128 && nrhs < MULTI_RHS) return launch_bwd_rhs<T, 32, 128, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        if (bp <= 128) return launch_bwd_rhs<T, 16, 128, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        return launch_bwd_rhs<T, 16, 256, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
    } else {
        if (bp <= 128 && nrhs >= MULTI_RHS) return launch_bwd_rhs<T, 8, 128, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        if (bp == 128 && nrhs == 1)
            return launch_bwd<T, 16, 128, MODE_ONE_EXACT, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        if (bp <= 128 && nrhs == 1) return launch_bwd<T, 16, 128, MODE_ONE, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        if (bp <= 128) return launch_bwd_rhs<T, 16, 128, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
        return launch_bwd_rhs<T, 8, 256, 256>(LB, Mx, bp, nsys, nrhs, W, st, sys0, nrun);
    }
}

template hipError_t launch_band_forward<float>(const void*, int, int, int, int, const void*, void*, hipStream_t, int,
                                               int);
template hipError_t launch_band_forward<double>(const void*, int, int, int, int, const void*, void*, hipStream_t, int,
                                                int);
template hipError_t launch_band_backward<float>(const void*, int, int, int, int, void*, hipStream_t, int, int);
template hipError_t launch_band_backward<double>(const void*, int, int, int, int, void*, hipStream_t, int, int);
template size_t sweep_smem<float>(int);
template size_t sweep_smem<double>(int);

}  // namespace stfd
