// Substitution sweeps of step 3 of Algorithm FD (Sec. 4.4) for a group of up
// to 16 right-hand sides, on the matrix cores.  With the band factors
// M_x + lambda_k A_x = L_k D_k L_k^T (kernels_band.hip) the sweeps are, per
// system k and block of 16 columns c (blocks of 16 rows and columns, the
// band reaching NB = bp / 16 blocks below the diagonal):
//
//   forward   y_c = L_cc^-1 (g_c - sum_{j<c} L_cj y_j),   w_c = D_c^-1 y_c
//   backward  z_c = L_cc^-T (w_c - sum_{j>c} L_jc^T z_j)
//
// written right-looking: as soon as block c is solved, the pending sums of
// the NB blocks it couples to take its contribution, a complex 16 x 16 x 16
// product per block (four real 16x16x4 MFMAs per k-step of four).  The
// pending 16-row x 16-right-hand-side tiles live in MFMA accumulator
// registers: block j belongs to wave j mod 4 for the whole sweep, which
// holds its next S = ceil(NB / 4) blocks in order.  The diagonal solve uses
// the inverse of the unit-triangular diagonal block (computed once after the
// factorization, band_diag_inverse_kernel), so it is one more tile product.
//
// Step for block c (one workgroup barrier):
//   owner wave (c mod 4): its first tile is complete; it is multiplied by
//     L_cc^-1 (or L_cc^-T) from its accumulator registers, the result is
//     stored (forward: times D_c^-1) and written to LDS for the other waves; the owner's tiles move up one slot and the block that
//     enters the window (c + 4S forward, c - 4S backward) takes the last;
//   all waves: each pending tile j takes -= Q_jc x_c, Q_jc = L_jc (forward)
//     or L_cj^T (backward), its operands loaded from the band storage
//     straight into registers NSET - 1 steps ahead (issued as the step
//     before begins, into the register set that step has just freed).
// Every factor entry is read once for all right-hand sides of the group.
//
// Layouts: band storage LB[k][c][d] = L_k[c + d, c] (d = 0: D_k), padded
// half-bandwidth bp (multiple of 16); block inverses LI[k][b][kc][m] =
// (L_bb^-1)[m][kc] (column-major 16 x 16); right-hand sides per RHS t a
// column-major M_x x 2 n_sys block at t * M_x * 2 n_sys, real parts of system
// k in column k, imaginary parts in column n_sys + k.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace stfd {

namespace {

constexpr int TB = 16;        // block size (rows, columns, right-hand sides)
constexpr int XS = TB + 1;    // LDS row stride of the transposed tiles

}  // namespace

// ---------------------------------------------------------------------------
// Inverses of the unit lower triangular diagonal blocks, computed in FP64
// from the stored factor: LI[k][b] column m is the solution of L_bb x = e_m
// (rows and columns past M_x give the identity).  Eight blocks per workgroup,
// one thread per column.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(128) band_diag_inverse_kernel(const cplx<T>* __restrict__ LB, cplx<T>* __restrict__ LI,
                                                               int Mx, int bp, int nblk, long long nblocks) {
    __shared__ double SR[8][TB][XS], SI[8][TB][XS];
    const int q = threadIdx.x / TB, m = threadIdx.x % TB;
    const long long gb = (long long)blockIdx.x * 8 + q;
    const bool live = gb < nblocks;
    const long long sys = live ? gb / nblk : 0;
    const int b = live ? (int)(gb % nblk) : 0;
    const int bp1 = bp + 1;
    const int c = TB * b + m;
    const cplx<T>* colp = LB + ((size_t)sys * Mx + (size_t)min(c, Mx - 1)) * bp1;
#pragma unroll
    for (int r = 0; r < TB; ++r) {
        const int d = r - m;
        const bool on = live && d > 0 && c < Mx && TB * b + r < Mx;
        const cplx<T> v = on ? colp[d] : cplx<T>{T(0), T(0)};
        SR[q][r][m] = static_cast<double>(v.re);
        SI[q][r][m] = static_cast<double>(v.im);
    }
    __syncthreads();
    double xr[TB], xi[TB];
#pragma unroll
    for (int r = 0; r < TB; ++r) {
        double ar = r == m ? 1.0 : 0.0, ai = 0.0;
#pragma unroll
        for (int k = 0; k < r; ++k) {
            const double lr = SR[q][r][k], li = SI[q][r][k];
            ar -= lr * xr[k] - li * xi[k];
            ai -= lr * xi[k] + li * xr[k];
        }
        xr[r] = ar;
        xi[r] = ai;
    }
    if (live) {
        cplx<T>* dst = LI + (size_t)gb * TB * TB + (size_t)m * TB;
#pragma unroll
        for (int r = 0; r < TB; ++r) dst[r] = cplx<T>{static_cast<T>(xr[r]), static_cast<T>(xi[r])};
    }
}

// ---------------------------------------------------------------------------
// The tile sweep.  S slots per wave (ceil(NB / 4)), NSET register sets of
// prefetched factor operands.
// ---------------------------------------------------------------------------
// PAIR: two real systems A and B (lambda real, factors and right-hand sides
// real: the imaginary parts of real systems are zero, up to the rounding of
// the forward transform, and do not reach U, since the back transform weighs
// them with the zero imaginary parts of their real eigenvectors) carried in
// the real and imaginary slots of one complex sweep: every operand's real
// part is A's, its imaginary part B's, and the products drop the cross
// terms.  Both imaginary parts of the result are written as zeros.
// STAGE (the FP32 backward sweep): the factor operands of a step, block row
// c of L (16-entry pieces of the 256 columns it spans), are loaded with 16
// consecutive lanes on each piece (4 pieces per load, whole cache lines)
// and go through LDS (QB, two buffers by step parity, k XOR n swizzled so
// that both the writes and the operand reads are free of bank conflicts)
// into the MFMA layout.  Loaded in that layout directly, each load touched
// 64 columns: 25.3 ms against 18.1 ms for the same bytes in pieces
// (timing variants on synthetic storage of the L-shape N_t = 1024 shape).
template <typename T, bool FWD>
constexpr bool tile_stage() { return !FWD && sizeof(T) == 4; }

template <typename T, bool FWD, int S, int NSET, bool VT, bool PAIR>
__device__ __forceinline__ void tile_sweep_body(const cplx<T>* __restrict__ LB, const cplx<T>* __restrict__ LI,
                                                int Mx, int bp, int nsys, int nrhs, const T* __restrict__ Vin,
                                                T* __restrict__ Vout, int sys, int sysB,
                                                const int* __restrict__ reach, T (*YR)[TB][XS], T (*YI)[TB][XS],
                                                cplx<T>* __restrict__ QB) {
    constexpr bool STAGE = tile_stage<T, FWD>();
    using V4 = typename vec4<T>::type;
    const int bp1 = bp + 1;
    const int NB = bp / TB;
    const int nblk = (Mx + TB - 1) / TB;
    const int r0 = blockIdx.y * TB;
    const int nr = min(TB, nrhs - r0);
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int g = lane >> 4, n = lane & 15;
    const bool nlive = n < nr;
    const size_t rstride = (size_t)Mx * 2 * nsys;
    const size_t voff = (size_t)(r0 + (nlive ? n : 0)) * rstride;
    // (PAIR: the "imaginary" input and output are B's real parts)
    const T* vin_re = Vin + voff + (size_t)sys * Mx;
    const T* vin_im = Vin + voff + (size_t)(PAIR ? sysB : nsys + sys) * Mx;
    T* vout_re = Vout + voff + (size_t)sys * Mx;
    T* vout_im = Vout + voff + (size_t)(PAIR ? sysB : nsys + sys) * Mx;
    const cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const cplx<T>* libase = LI + (size_t)sys * nblk * TB * TB;
    const cplx<T>* baseB = LB + (size_t)sysB * Mx * bp1;
    const cplx<T>* libaseB = LI + (size_t)sysB * nblk * TB * TB;
    // factor and inverse entries by index from a workgroup-uniform base, the
    // byte offset in 32 bits (one system's band is below 4 GiB, checked by
    // the launcher): the loads take the scalar-base form, with no 64-bit
    // address arithmetic per lane.  An operand's imaginary slot is B's real
    // part of the same entry in PAIR mode.
    auto entry = [](const cplx<T>* b, uint32_t i) -> const cplx<T>* {
        return reinterpret_cast<const cplx<T>*>(reinterpret_cast<const char*>(b) + i * (uint32_t)sizeof(cplx<T>));
    };
    auto load_op = [&](const cplx<T>* a, const cplx<T>* b, uint32_t i) -> cplx<T> {
        const cplx<T>* e = entry(a, i);
        if constexpr (PAIR) return cplx<T>{e->re, entry(b, i)->re};
        else return *e;
    };

    // tile of the input vector for block j, accumulator layout.  The loads
    // are issued raw (address clamped) so that they stay in flight;
    // tile_mask zeroes the entries outside (rows past M_x, right-hand sides
    // past nr, blocks outside the matrix) where the values are used.
    auto tile_on = [&](int j, int r) {
        const int row = TB * j + mfma_row<T>(g, r);
        return nlive && j >= 0 && j < nblk && row < Mx;
    };
    auto load_tile_raw = [&](int j, V4& ar, V4& ai) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = tile_on(j, r) ? TB * j + mfma_row<T>(g, r) : 0;
            ar[r] = vin_re[rr];
            ai[r] = vin_im[rr];
        }
    };
    auto tile_mask = [&](int j, V4& ar, V4& ai) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool on = tile_on(j, r);
            ar[r] = on ? ar[r] : T(0);
            ai[r] = on ? ai[r] : T(0);
        }
    };
    // VT (FP32, M_x >= 4): the entering tile's rows 16 j + 4 g .. + 3 of
    // a lane are consecutive, one 16-byte load per part (the columns are
    // 4-byte aligned, which these loads allow) from row0c = clamp(row0, 0,
    // M_x - 4), so that the four rows read stay inside the column; row r of
    // the group is then element r + (row0 - row0c), taken where the tile is
    // used (rows that the shift pushes past the vector are past M_x)
    auto row0c_of = [&](int j) { return min(max(TB * j + 4 * g, 0), Mx - 4); };
    auto load_tile_vec = [&](int j, V4& ar, V4& ai) {
        const int r0c = row0c_of(j);
        __builtin_memcpy(&ar, vin_re + r0c, sizeof(V4));
        __builtin_memcpy(&ai, vin_im + r0c, sizeof(V4));
    };
    auto tile_take = [&](int j, V4& ar, V4& ai) {
        if constexpr (VT) {
            const int sh = TB * j + 4 * g - row0c_of(j);
            const V4 br = ar, bi = ai;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T vr = br[3], vi = bi[3];
#pragma unroll
                for (int q = 2; q >= r; --q) {
                    vr = r + sh == q ? br[q] : vr;
                    vi = r + sh == q ? bi[q] : vi;
                }
                ar[r] = vr;
                ai[r] = vi;
            }
        }
        tile_mask(j, ar, ai);
    };
    auto load_tile = [&](int j, V4& ar, V4& ai) {
        load_tile_raw(j, ar, ai);
        tile_mask(j, ar, ai);
    };
    // operand of Q_jc for k-step kk (lane: m = n, k = 4 kk + g), raw value
    // (address clamped) and whether it lies in the band
    // Factor operand of Q_jc for k-step kk (lane: m = n, k = kof(kk)):
    // forward L[16 j + m][16 c + k], backward L[16 c + k][16 j + m].  In the
    // band storage its index is linear in the blocks,
    //   forward  (16 c + k)(bp + 1) + 16 (j - c) + n - k
    //          = 16 bp c + 16 j + n + k bp,
    //   backward 16 bp j + n bp + 16 c + k,
    // and always in range except in the last block (clamped).  Entries of
    // rows past M_x are zero in the storage; only the last tile of the band
    // (d > bp there for some lanes) and columns past M_x need masking where
    // the value is used (q_on).
    // k of lane group g in k-step kk (backward, the four groups then read
    // four consecutive entries of each of the wave's 16 columns)
    auto kof = [&](int kk) { return 4 * kk + g; };
    const int qlast = Mx * bp1 - 1;
    auto q_index = [&](int j, int c, int kk) -> uint32_t {
        const int i = FWD ? TB * bp * c + TB * j + n + kof(kk) * bp
                          : TB * bp * j + n * bp + TB * c + kof(kk);
        return (uint32_t)min(max(i, 0), qlast);
    };
    auto q_on = [&](int j, int c, int kk) {
        const int d = FWD ? TB * (j - c) + n - kof(kk) : TB * (c - j) + kof(kk) - n;
        const int col = FWD ? TB * c + kof(kk) : TB * j + n;
        return d <= bp && col < Mx;
    };
    // whether block column c couples to block j (within the band and the
    // envelope of the factor: reach[b] blocks below diagonal block b; the
    // forward sweep's bound rc = min(NB, reach[c]) is read once per step)
    auto couples = [&](int j, int c, int rc) {
        return FWD ? (j > c && j < nblk && j - c <= rc)
                   : (j < c && j >= 0 && c - j <= min(NB, reach[j]));
    };
    // operand of the diagonal inverse for k-step kk: forward L_cc^-1[m][k],
    // backward L_cc^-1[k][m], with k the row that accumulator register kk
    // of the lane holds (the solve takes the owner's tile as it is, with
    // no transposition through LDS)
    auto li_addr = [&](int c, int kk) -> uint32_t {
        const int cc = min(max(c, 0), nblk - 1);
        const int m = n, k = mfma_row<T>(g, kk);
        return (uint32_t)(cc * TB * TB + (FWD ? k * TB + m : m * TB + k));
    };

    // ---- this wave's pending tiles
    V4 accR[S], accI[S];
    const int j0 = FWD ? w : nblk - 1 - ((nblk - 1 - w) & 3);   // first block of this wave (may be < 0)
#pragma unroll
    for (int t = 0; t < S; ++t) load_tile(FWD ? j0 + 4 * t : j0 - 4 * t, accR[t], accI[t]);

    // Everything step s needs from memory is loaded NSET - 1 steps ahead, at
    // the start of step s - NSET + 1 (so that the loads are in flight during
    // that step's work): the factor operands of the wave's pending tiles,
    // D of the rows of block c this wave stores (forward), and, by the
    // owner of block c only, the diagonal inverse and the tile entering
    // when c retires.  (Loaded by every wave alike, these two were three
    // fifths of the cache lines a step requested, the vector memory
    // front end the limit of the step's load issue.)
    cplx<T> qa[NSET][S][4], pa[NSET][4], da[NSET];
    V4 ea[NSET][2];
    auto fetch = [&](int s, cplx<T> (&qx)[S][4], cplx<T> (&px)[4], cplx<T>& dx, V4 (&ex)[2]) {
        const int c = FWD ? s : nblk - 1 - s;
        const int delta = FWD ? ((w - c - 1) & 3) + 1 : ((c - w - 1) & 3) + 1;
        if constexpr (STAGE) {
            // piece (jrel, nn): column 16 (c - 1 - jrel) + nn of block row
            // c, entry kq (row 16 c + kq) by lane kq of a group of 16; the
            // wave takes pieces 16 S w .. 16 S (w + 1) - 1, 4 per load, the
            // set's 4 S slots reused as a flat array
#pragma unroll
            for (int r = 0; r < 4 * S; ++r) {
                const int colidx = (w * 4 * S + r) * 4 + (lane >> 4);
                const int jb = c - 1 - (colidx >> 4), nn = colidx & 15, kq = lane & 15;
                const int i = (TB * jb + nn) * bp1 + TB * (c - jb) + kq - nn;
                qx[r >> 2][r & 3] = load_op(base, baseB, (uint32_t)min(max(i, 0), qlast));  // raw: masked where used
            }
        } else {
#pragma unroll
            for (int t = 0; t < S; ++t) {
                const int j = FWD ? c + delta + 4 * t : c - delta - 4 * t;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) qx[t][kk] = load_op(base, baseB, q_index(j, c, kk));  // raw: masked where used
            }
        }
        if ((c & 3) == w) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) px[kk] = load_op(libase, libaseB, li_addr(c, kk));
            if constexpr (VT) load_tile_vec(FWD ? c + 4 * S : c - 4 * S, ex[0], ex[1]);
            else load_tile_raw(FWD ? c + 4 * S : c - 4 * S, ex[0], ex[1]);
        }
        if (FWD) {
            const int row = min(max(TB * c + 4 * w + g, 0), Mx - 1);
            dx = load_op(base, baseB, (uint32_t)(row * bp1));
        }
    };
    // the sets go out in step order, each whole before the next: the waits
    // before a set's use count the loads issued after it, and the count on
    // entry to the loop (after these) bounds the count on every iteration.
    // Left to the scheduler, the sets' loads were interleaved, the last
    // load of set 0 came last, and every step then waited for its own
    // fresh prefetch before its first product.
#pragma unroll
    for (int u = 0; u + 1 < NSET; ++u) {
        fetch(u, qa[u], pa[u], da[u], ea[u]);
        __builtin_amdgcn_sched_barrier(0);
    }

    // one step: block c = (FWD ? s : nblk - 1 - s); steps past the end only fetch
    auto step = [&](int s, cplx<T> (&qx)[S][4], cplx<T> (&px)[4], cplx<T>& dx, V4 (&ex)[2],
                    cplx<T> (&qn)[S][4], cplx<T> (&pn)[4], cplx<T>& dn, V4 (&en)[2]) {
        // the set step s - 1 used takes step s + NSET - 1, issued before this
        // step's work so that the loads are in flight during it
        fetch(s + NSET - 1, qn, pn, dn, en);
        const int c = FWD ? s : nblk - 1 - s;
        const int par = s & 1;
        if (s < nblk) {
            const int rc = FWD ? min(NB, reach[c]) : NB;
            if constexpr (STAGE) {
                // this step's pieces of block row c to QB[par] (read after
                // the step's barrier; the buffer's previous readers, step
                // s - 2, all passed step s - 1's barrier before this)
#pragma unroll
                for (int r = 0; r < 4 * S; ++r) {
                    const int colidx = (w * 4 * S + r) * 4 + (lane >> 4);
                    const int jrel = colidx >> 4, nn = colidx & 15, kq = lane & 15;
                    QB[((par * 4 * S + jrel) * TB + nn) * TB + (kq ^ nn)] = qx[r >> 2][r & 3];
                }
            }
            if ((c & 3) == w) {
                // ---- owner: x_c = P_c acc[0], to LDS for every wave.  The
                // products' k-step kk takes, in lane group g, the tile's row
                // held in accumulator register kk (and the matching column
                // of P_c): the sum runs over all 16 rows in another order
                V4 xr = zero4<T>(), xi = zero4<T>();
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const T br = accR[0][kk], bi = accI[0][kk];
                    const cplx<T> a = px[kk];
                    if constexpr (PAIR) {
                        xr = mfma16x16x4<T>(a.re, br, xr);
                        xi = mfma16x16x4<T>(a.im, bi, xi);
                    } else {
                        xr = mfma16x16x4<T>(a.re, br, xr);
                        xr = mfma16x16x4<T>(-a.im, bi, xr);
                        xi = mfma16x16x4<T>(a.re, bi, xi);
                        xi = mfma16x16x4<T>(a.im, br, xi);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    YR[par][mfma_row<T>(g, r)][n] = xr[r];
                    YI[par][mfma_row<T>(g, r)][n] = xi[r];
                }
                // slots move up; the entering block takes the last one
#pragma unroll
                for (int t = 0; t + 1 < S; ++t) {
                    accR[t] = accR[t + 1];
                    accI[t] = accI[t + 1];
                }
                V4 er = ex[0], ei = ex[1];
                tile_take(FWD ? c + 4 * S : c - 4 * S, er, ei);
                accR[S - 1] = er;
                accI[S - 1] = ei;
            }
            __syncthreads();
            // ---- every wave: its four rows of the solved block to memory
            // (forward: times D^-1), then pending tiles -= Q_jc x_c
            {
                const int rl = 4 * w + g, row = TB * c + rl;
                T vr = YR[par][rl][n], vi = YI[par][rl][n];
                if (FWD) {
                    if constexpr (PAIR) {
                        vr = vr * cinv_fast(cplx<T>{dx.re, T(0)}).re;
                        vi = vi * cinv_fast(cplx<T>{dx.im, T(0)}).re;
                    } else {
                        const cplx<T> o = cmul(cplx<T>{vr, vi}, cinv_fast(dx));
                        vr = o.re;
                        vi = o.im;
                    }
                }
                if (nlive && row < Mx) {
                    vout_re[row] = vr;
                    vout_im[row] = vi;
                    if constexpr (PAIR) {
                        // the imaginary parts of both real systems
                        Vout[voff + (size_t)(nsys + sys) * Mx + row] = T(0);
                        Vout[voff + (size_t)(nsys + sysB) * Mx + row] = T(0);
                    }
                }
            }
            const int delta = FWD ? ((w - c - 1) & 3) + 1 : ((c - w - 1) & 3) + 1;
            // the solved block, negated once here, so that the products
            // below take the factor operands as loaded (-= Q x as += Q (-x))
            T br[4], bi[4], pi[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                pi[kk] = YI[par][kof(kk)][n];
                br[kk] = -YR[par][kof(kk)][n];
                bi[kk] = -pi[kk];
            }
#pragma unroll
            for (int t = 0; t < S; ++t) {
                const int j = FWD ? c + delta + 4 * t : c - delta - 4 * t;
                if (couples(j, c, rc)) {
                    // operands: this wave's registers, or QB (STAGE: entry
                    // k = 4 kk + g of column n of block j = c - 1 - jrel)
                    cplx<T> q[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        if constexpr (STAGE) {
                            const int jrel = c - 1 - j, k = kof(kk);
                            q[kk] = QB[((par * 4 * S + jrel) * TB + n) * TB + (k ^ n)];
                        } else {
                            q[kk] = qx[t][kk];
                        }
                    }
                    // masks only where some entry can fall outside: the
                    // last tile of the band, the last (ragged) column block
                    const bool edge = (FWD ? j - c : c - j) == NB || (FWD ? c : j) == nblk - 1;
                    if (edge) {
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            const bool on = q_on(j, c, kk);
                            q[kk].re = on ? q[kk].re : T(0);
                            q[kk].im = on ? q[kk].im : T(0);
                        }
                    }
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const cplx<T> a = q[kk];
                        // br + i bi = -x, pi = Im x: acc += Q (-x)
                        if constexpr (PAIR) {
                            accR[t] = mfma16x16x4<T>(a.re, br[kk], accR[t]);
                            accI[t] = mfma16x16x4<T>(a.im, bi[kk], accI[t]);
                        } else {
                            accR[t] = mfma16x16x4<T>(a.re, br[kk], accR[t]);
                            accR[t] = mfma16x16x4<T>(a.im, pi[kk], accR[t]);
                            accI[t] = mfma16x16x4<T>(a.re, bi[kk], accI[t]);
                            accI[t] = mfma16x16x4<T>(a.im, br[kk], accI[t]);
                        }
                    }
                }
            }
        }
    };

    for (int s0 = 0; s0 < nblk; s0 += NSET) {
#pragma unroll
        for (int u = 0; u < NSET; ++u) {
            const int v = (u + NSET - 1) % NSET;
            step(s0 + u, qa[u], pa[u], da[u], ea[u], qa[v], pa[v], da[v], ea[v]);
        }
    }
}

// Workgroups [0, ncplx): system sys0 + x, complex; workgroups past ncplx:
// the real systems sys0 + ncplx + 2 (x - ncplx) and the next one (if any, else
// the same system twice, its results written by both slots alike), paired.
template <typename T, bool FWD, int S, int NSET, bool VT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) tile_sweep_kernel(const cplx<T>* __restrict__ LB,
                                                        const cplx<T>* __restrict__ LI, int Mx, int bp, int nsys,
                                                        int nrhs, const T* __restrict__ Vin, T* __restrict__ Vout,
                                                        int sys0, int ncplx, int nrun,
                                                        const int* __restrict__ reach,
                                                        const int* __restrict__ gate) {
    if (gate && *gate) return;
    __shared__ T YR[2][TB][XS], YI[2][TB][XS];            // solved block, by step parity
    __shared__ cplx<T> QB[tile_stage<T, FWD>() ? 2 * 4 * S * TB * TB : 1];   // staged factor operands
    const int x = blockIdx.x;
    if (x < ncplx) {
        tile_sweep_body<T, FWD, S, NSET, VT, false>(LB, LI, Mx, bp, nsys, nrhs, Vin, Vout, sys0 + x, sys0 + x, reach,
                                                YR, YI, QB);
    } else {
        const int a = sys0 + ncplx + 2 * (x - ncplx);
        const int b = a + 1 < sys0 + nrun ? a + 1 : a;
        tile_sweep_body<T, FWD, S, NSET, VT, true>(LB, LI, Mx, bp, nsys, nrhs, Vin, Vout, a, b, reach, YR, YI, QB);
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_band_diag_inverse(const void* LB, void* LI, int Mx, int bp, int nsys, hipStream_t st) {
    const int nblk = (Mx + TB - 1) / TB;
    const long long nb = (long long)nsys * nblk;
    const long long grid = (nb + 7) / 8;
    hipLaunchKernelGGL(band_diag_inverse_kernel<T>, dim3((unsigned)grid), dim3(128), 0, st,
                       static_cast<const cplx<T>*>(LB), static_cast<cplx<T>*>(LI), Mx, bp, nblk, nb);
    return hipGetLastError();
}

template <typename T, bool FWD, int S>
static hipError_t launch_tile_t(const void* LB, const void* LI, const int* reach, int Mx, int bp, int nsys, int nrhs,
                                const void* Vin, void* Vout, hipStream_t st, int sys0, int nrun, int nreal) {
    // register sets (prefetch distance NSET - 1 steps): measured best at
    // 3 for the FP32 forward sweep and 2 for FP64 (whose third set costs
    // occupancy); 2 for the staged FP32 backward sweep, whose third set
    // would spill
    constexpr int NSET = (sizeof(T) == 4 && FWD) ? 3 : 2;
    const int ncplx = nrun - nreal;
    dim3 grid(ncplx + (nreal + 1) / 2, (nrhs + TB - 1) / TB);
    // the entering tile by 16-byte loads: FP32 (four consecutive rows per
    // lane) with at least four rows
    if constexpr (sizeof(T) == 4) {
        if (Mx >= 4) {
            hipLaunchKernelGGL((tile_sweep_kernel<T, FWD, S, NSET, true>), grid, dim3(256), 0, st,
                               static_cast<const cplx<T>*>(LB), static_cast<const cplx<T>*>(LI), Mx, bp, nsys, nrhs,
                               static_cast<const T*>(Vin), static_cast<T*>(Vout), sys0, ncplx, nrun, reach,
                               launch_gate());
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((tile_sweep_kernel<T, FWD, S, NSET, false>), grid, dim3(256), 0, st,
                       static_cast<const cplx<T>*>(LB), static_cast<const cplx<T>*>(LI), Mx, bp, nsys, nrhs,
                       static_cast<const T*>(Vin), static_cast<T*>(Vout), sys0, ncplx, nrun, reach, launch_gate());
    return hipGetLastError();
}

template <typename T, bool FWD>
static hipError_t launch_tile(const void* LB, const void* LI, const int* reach, int Mx, int bp, int nsys, int nrhs,
                              const void* Vin, void* Vout, hipStream_t st, int sys0, int nrun, int nreal) {
    if (bp < TB || bp % TB != 0 || bp > TILE_BPMAX || sys0 < 0 || nrun < 1 || sys0 + nrun > nsys || nrhs < 1 ||
        nreal < 0 || nreal > nrun)
        return hipErrorInvalidValue;
    // byte offsets inside one system's band and block inverses are 32-bit
    const size_t nblk = ((size_t)Mx + TB - 1) / TB;
    if ((size_t)Mx * (bp + 1) * sizeof(cplx<T>) >= (1ull << 32) || nblk * TB * TB * sizeof(cplx<T>) >= (1ull << 32))
        return hipErrorInvalidValue;
    const int slots = (bp / TB + 3) / 4;
    switch (slots) {
        case 1: return launch_tile_t<T, FWD, 1>(LB, LI, reach, Mx, bp, nsys, nrhs, Vin, Vout, st, sys0, nrun, nreal);
        case 2: return launch_tile_t<T, FWD, 2>(LB, LI, reach, Mx, bp, nsys, nrhs, Vin, Vout, st, sys0, nrun, nreal);
        case 3: return launch_tile_t<T, FWD, 3>(LB, LI, reach, Mx, bp, nsys, nrhs, Vin, Vout, st, sys0, nrun, nreal);
        default: return launch_tile_t<T, FWD, 4>(LB, LI, reach, Mx, bp, nsys, nrhs, Vin, Vout, st, sys0, nrun, nreal);
    }
}

template <typename T>
hipError_t launch_tile_forward(const void* LB, const void* LI, const int* reach, int Mx, int bp, int nsys, int nrhs,
                               const void* G, void* W, hipStream_t st, int sys0, int nrun, int nreal) {
    return launch_tile<T, true>(LB, LI, reach, Mx, bp, nsys, nrhs, G, W, st, sys0, nrun, nreal);
}

template <typename T>
hipError_t launch_tile_backward(const void* LB, const void* LI, const int* reach, int Mx, int bp, int nsys, int nrhs,
                                void* W, hipStream_t st, int sys0, int nrun, int nreal) {
    return launch_tile<T, false>(LB, LI, reach, Mx, bp, nsys, nrhs, W, W, st, sys0, nrun, nreal);
}

template hipError_t launch_band_diag_inverse<float>(const void*, void*, int, int, int, hipStream_t);
template hipError_t launch_band_diag_inverse<double>(const void*, void*, int, int, int, hipStream_t);
template hipError_t launch_tile_forward<float>(const void*, const void*, const int*, int, int, int, int, const void*,
                                               void*, hipStream_t, int, int, int);
template hipError_t launch_tile_forward<double>(const void*, const void*, const int*, int, int, int, int, const void*,
                                                void*, hipStream_t, int, int, int);
template hipError_t launch_tile_backward<float>(const void*, const void*, const int*, int, int, int, int, void*,
                                                hipStream_t, int, int, int);
template hipError_t launch_tile_backward<double>(const void*, const void*, const int*, int, int, int, int, void*,
                                                 hipStream_t, int, int, int);

}  // namespace stfd
