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

#include <algorithm>

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
// The same factorization with the active window resident in LDS.
// Panel p0 (16 columns) touches only columns [p0, p0 + bp + 16), so the
// window of bp + 16 band columns (entries d = 0..bp each, ring-indexed by
// column mod (bp + 16)) is kept in LDS for the whole factorization: the
// trailing update reads and writes it there, the columns entering the
// window are loaded into registers one panel ahead, and each finished panel
// is written to HBM once.  The panel itself is factored in registers.
// BPC bounds bp (register prefetch sizing); used where the window fits.
// ---------------------------------------------------------------------------
template <typename T, int BPC>
__global__ void __launch_bounds__(256) band_ldl_window_kernel(cplx<T>* __restrict__ LB, int Mx, int bp,
                                                              int* __restrict__ flag) {
    constexpr int EP = (16 * (BPC + 1) + 255) / 256;   // prefetched entries per thread
    constexpr int RH = (BPC + 63) / 64;                // row halves of a panel column per lane
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* Wn = reinterpret_cast<cplx<T>*>(smem_raw); // [ring][bp1], then one zero entry
    const int bp1 = bp + 1;
    const int ring = bp + 16;
    const int ZE = ring * bp1;
    const int sys = blockIdx.x;
    cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const size_t total = (size_t)Mx * bp1;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int ntile = bp / 16;
    const int tiles_total = ntile * (ntile + 1) / 2;
    const cplx<T> zero = {T(0), T(0)};

    // window columns [0, ring)
    const int wcols = min(ring, Mx);
    for (int e = tid; e < ring * bp1; e += 256) {       // values, not a choice of lvalues (that would
        const bool in = e < wcols * bp1;                 // put the operands in scratch memory)
        Wn[e] = in ? cplx<T>{base[e].re, base[e].im} : cplx<T>{0, 0};
    }
    if (tid == 0) Wn[ZE] = zero;
    // columns of entry tid + 256 j of a 16-column block (fixed for the whole run)
    int ecol[EP];
#pragma unroll
    for (int j = 0; j < EP; ++j) ecol[j] = (tid + 256 * j) / bp1;
    // registers: the block of 16 columns that enters the window next
    cplx<T> pf[EP];
    auto prefetch = [&](int c0) {
        const size_t b0 = (size_t)c0 * bp1;
#pragma unroll
        for (int j = 0; j < EP; ++j) {          // field by field: keeps pf in registers for complex double
            const cplx<T>* e = base + min(b0 + tid + 256 * j, total - 1);
            pf[j].re = e->re;
            pf[j].im = e->im;
        }
    };
    prefetch(ring);
    __syncthreads();

    int sp0 = 0;                                        // window slot of column p0
    for (int p0 = 0; p0 < Mx; p0 += 16) {
        const int nb = min(16, Mx - p0);
        cplx<T>* P = Wn + (size_t)sp0 * bp1;            // panel columns, contiguous
        // ---- factor the panel in registers, without barriers.  A lane holds
        // one row of the panel (its 16 entries): lanes 0-15 of every wave the
        // rows of the diagonal block (the same in all waves), lanes 16 .. 16 +
        // bp/4 - 1 of wave w the rows p0 + 16 + (bp/4) w + (lane - 16) below.
        // Column k: D_k and the l_jk of the block rows come from lanes k and j
        // by lane broadcasts; A[i, j] -= a_ik l_jk for j > k.
        {
            const int rw = bp >> 2;
            const bool own = lane < 16 || lane - 16 < rw;
            const int rrel = lane < 16 ? lane : 16 + rw * wave + (lane - 16);
            cplx<T> a[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int d = rrel - c;
                a[c] = Wn[own && c < nb && d >= 0 && d <= bp ? (sp0 + c) * bp1 + d : ZE];
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < nb) {
                    const cplx<T> dk = {lane_bcast(a[k].re, k), lane_bcast(a[k].im, k)};
                    const cplx<T> inv = cinv_fast(dk);
                    if (tid == 0) {
                        const T mag = fabs(dk.re) + fabs(dk.im);
                        if (!(mag > T(0)) || !isfinite(mag)) atomicOr(flag, 1);
                    }
                    const cplx<T> aik = a[k];
                    if (rrel > k) a[k] = cmul(aik, inv);
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) {
                        const T lr = lane_bcast(a[k].re, j), lim = lane_bcast(a[k].im, j);
                        a[j].re = fma(-aik.re, lr, a[j].re);
                        a[j].re = fma(aik.im, lim, a[j].re);
                        a[j].im = fma(-aik.re, lim, a[j].im);
                        a[j].im = fma(-aik.im, lr, a[j].im);
                    }
                }
                // keep each column's broadcasts next to their uses (bounded
                // scalar-register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
            const bool writer = own && (lane >= 16 || wave == 0);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int d = rrel - c;
                if (writer && c < nb && d >= 0 && d <= bp) Wn[(sp0 + c) * bp1 + d] = a[c];
            }
        }
        __syncthreads();
        // ---- trailing update in LDS on the matrix cores.  The operands of
        // every tile come from the 8 row blocks below the panel: lane (li, lk)
        // holds L[p0 + 16 + 16 m + li, p0 + 4 kk + lk] and that value times
        // D, for all m and kk, in registers.  Tile (ti, tj), ti >= tj, covers
        // rows p0 + 16 + 16 ti + (0..15) and columns p0 + 16 + 16 tj + (0..15);
        // tile number ti (ti + 1) / 2 + tj goes to wave (number mod 4).
        {
            cplx<T> lo[8][4], ld[8][4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const cplx<T> dk = Wn[k < nb ? (sp0 + k) * bp1 : ZE];
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int o = 16 + 16 * m + li - k;
                    lo[m][kk] = Wn[m < ntile && k < nb && o <= bp ? (sp0 + k) * bp1 + o : ZE];
                    ld[m][kk] = cmul(lo[m][kk], dk);
                }
            }
#pragma unroll
            for (int ti = 0; ti < 8; ++ti) {
#pragma unroll
                for (int tj = 0; tj <= ti; ++tj) {
                    if (ti < ntile && (ti * (ti + 1) / 2 + tj) % 4 == wave) {
                        int ce[4];
                        cplx<T> cv[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            // D[c' = p0 + 16 + 16 tj + mfma_row(lk, j)][r = p0 + 16 + 16 ti + li]
                            const int cl = 16 + 16 * tj + mfma_row<T>(lk, j);
                            const int d = 16 * (ti - tj) + li - mfma_row<T>(lk, j);
                            int sl = sp0 + cl;
                            sl = sl >= ring ? sl - ring : sl;
                            ce[j] = d >= 0 && d <= bp ? sl * bp1 + d : -1;
                            cv[j] = Wn[ce[j] >= 0 ? ce[j] : ZE];
                        }
                        typename vec4<T>::type accR = zero4<T>(), accI = zero4<T>();
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            const cplx<T> a = lo[tj][kk], b = ld[ti][kk];
                            accR = mfma16x16x4<T>(a.re, b.re, accR);
                            accR = mfma16x16x4<T>(-a.im, b.im, accR);
                            accI = mfma16x16x4<T>(a.re, b.im, accI);
                            accI = mfma16x16x4<T>(a.im, b.re, accI);
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (ce[j] >= 0) Wn[ce[j]] = cplx<T>{cv[j].re - accR[j], cv[j].im - accI[j]};
                    }
                }
            }
        }
        __syncthreads();
        // ---- finished panel to HBM; the block entering the window takes its slots
        {
            cplx<T>* dst = base + (size_t)p0 * bp1;
            const int ncol_in = Mx - (p0 + ring);          // columns of the entering block that exist
#pragma unroll
            for (int j = 0; j < EP; ++j) {
                const int e = tid + 256 * j;
                if (e < 16 * bp1) {
                    if (ecol[j] < nb) dst[e] = P[e];
                    const bool in = ecol[j] < ncol_in;
                    P[e].re = in ? pf[j].re : T(0);
                    P[e].im = in ? pf[j].im : T(0);
                }
            }
        }
        prefetch(p0 + ring + 16);
        __syncthreads();
        sp0 += 16;
        sp0 = sp0 >= ring ? sp0 - ring : sp0;
    }
}

// ---------------------------------------------------------------------------
// FP32 with padded half-bandwidth 128: the trailing window in registers.
// Column block B (columns 16B .. 16B + 15) lies in the trailing window of
// panels q with q < B <= q + 8; there it sits at position m = B - q - 1.  Its
// band rows 16B .. 16B + 127 (row blocks B .. B + 7) are eight 16x16 MFMA
// accumulator tiles; tile ra (row block B + ra) is owned by tile wave
// (B + ra / 2) mod 4, in that wave's slot 0 at positions 0-3 and slot 1 at
// positions 4-7, and every trailing update is subtracted from it there.  The
// shifts give every tile wave 9 of the 36 tiles a panel updates (owning
// whole blocks would give 12, 10, 8 and 6) and two tiles of every block, so
// that the update of the next block and its hand-over are spread evenly.  Row block B + 8 of the block is only touched by the
// block's own panel.
//
// Two roles share every SIMD: waves 0-3 factor the panels (a chain of lane
// broadcasts, latency-bound vector work), waves 4-7 hold the tiles and run
// the matrix cores.  Iteration q: the tile waves apply panel q - 1 to block
// q (its tiles at position 0) and hand block q over to the panel buffer,
// while the chain waves write panel q - 1 to HBM; after a barrier the chain
// waves factor panel q while the tile waves apply panel q - 1 to positions
// 1-7.  The chain waves write the factored diagonal block to PD and the rows
// below it times D to LD (double-buffered), the tile operands.
// ---------------------------------------------------------------------------
constexpr int RPS = 17;                                   // panel buffer row stride (complex)

__device__ __forceinline__ constexpr int own_shift(int ra) { return ra >> 1; }
// The tiles 2r and 2r + 1 of a block go to one wave; a tile's prefetch slot
// is ra mod 2.

__global__ void __launch_bounds__(512) band_ldl_reg_kernel(cplx<float>* __restrict__ LB, int Mx,
                                                           int* __restrict__ flag) {
    using T = float;
    using V4 = vec4<float>::type;
    constexpr int bp = 128, bp1 = 129, NROW = 144;
    constexpr int EP = (16 * bp1 + 255) / 256;            // write-out entries per chain thread
    __shared__ cplx<T> PB[2][NROW * RPS];                 // panel rows p0 + 0..143, 16 columns, by panel parity
    __shared__ cplx<T> LDB[2][128 * RPS];                 // a panel's rows 16.. times D, by panel parity
    __shared__ cplx<T> PD[16 * RPS];                      // the factored diagonal block of the last panel
    const int sys = blockIdx.x;
    cplx<T>* base = LB + (size_t)sys * Mx * bp1;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int nblk = (Mx + 15) / 16;
    const cplx<T> zero = {T(0), T(0)};

    // panel 0 straight into its buffer
    for (int e = tid; e < NROW * 16; e += 512) {
        const int r = e >> 4, c = e & 15, d = r - c;
        const bool ok = c < Mx && d >= 0 && d <= bp;
        const cplx<T>* x = base + (ok ? (size_t)c * bp1 + d : 0);
        PB[0][r * RPS + c] = cplx<T>{ok ? x->re : T(0), ok ? x->im : T(0)};
    }

    if (wave >= 4) {
        // ================= tile waves =================
        const int tw = wave - 4, ttid = tid - 256;
        // tile ra of column block B, this lane's entry j: row 16B + 16 ra + li,
        // column 16B + 4 lk + j.  Loads are issued raw (clamped address) and
        // masked where they are used, so that they stay in flight.
        auto tile_ok = [&](int B, int ra, int j) {
            return B < nblk && 16 * B + 4 * lk + j < Mx && 16 * ra + li - 4 * lk - j >= 0;
        };
        auto tile_load = [&](int B, int ra, cplx<T> (&v)[4]) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 16 * B + 4 * lk + j;
                const int d = 16 * ra + li - 4 * lk - j;
                const cplx<T>* e = base + (tile_ok(B, ra, j) ? (size_t)c * bp1 + d : 0);
                v[j].re = e->re;
                v[j].im = e->im;
            }
        };
        auto owns = [&](int B, int ra) { return ((B + own_shift(ra)) & 3) == tw; };
        // row block 8 of column block B: entry (row 128 + ttid / 16, column ttid % 16)
        const int r8r = 128 + (ttid >> 4), r8c = ttid & 15;
        auto row8_ok = [&](int B) { return B < nblk && 16 * B + r8c < Mx && r8r - r8c <= bp; };
        auto row8_load = [&](int B) -> cplx<T> {
            const cplx<T>* e = base + (row8_ok(B) ? (size_t)(16 * B + r8c) * bp1 + (r8r - r8c) : 0);
            return cplx<T>{e->re, e->im};
        };
        // C -= L_c D L_r^T on a tile: the columns are rows 16 m + li of the
        // previous panel's rows 16.. (m the block's position), the rows rows
        // 16 (m + ra) + li; operands from that panel's buffer Pp and its LD
        // (the panel's contribution is summed on its own and subtracted once,
        // so the accumulator tile rounds once per panel, not after every MFMA)
        auto tile_mfma = [&](V4& cr, V4& ci, const cplx<T>* Pp, const cplx<T>* LD, int m, int ra) {
            V4 ur = zero4<T>(), ui = zero4<T>();
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const cplx<T> x = Pp[(16 + 16 * m + li) * RPS + k], y = LD[(16 * (m + ra) + li) * RPS + k];
                ur = mfma16x16x4<T>(x.re, y.re, ur);
                ui = mfma16x16x4<T>(x.re, y.im, ui);
                ur = mfma16x16x4<T>(-x.im, y.im, ur);
                ui = mfma16x16x4<T>(x.im, y.re, ui);
            }
            cr -= ur;
            ci -= ui;
        };

        V4 accR[2][8], accI[2][8];
        cplx<T> pf[2][4];                                 // the owned tiles of the next entering block
        // prefetch this wave's tiles of block B (tiles 2r, 2r + 1) into pf
        auto prefetch = [&](int B) {
            const int r = (tw - B) & 3;
#pragma unroll
            for (int i = 0; i < 2; ++i) tile_load(B, 2 * r + i, pf[i]);
        };
#pragma unroll
        for (int ra = 0; ra < 8; ++ra) {
            int b0 = (tw - own_shift(ra)) & 3;            // this wave's blocks of tile ra: b0, b0 + 4
            b0 = b0 == 0 ? 4 : b0;
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                cplx<T> v[4];
                tile_load(b0 + 4 * sl, ra, v);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool ok = tile_ok(b0 + 4 * sl, ra, j);
                    accR[sl][ra][j] = ok ? v[j].re : T(0);
                    accI[sl][ra][j] = ok ? v[j].im : T(0);
                }
            }
        }
        prefetch(9);
        cplx<T> r8 = row8_load(1);
        __syncthreads();

        for (int q = 0; q < nblk; ++q) {
            cplx<T>* P = PB[q & 1];
            const cplx<T>* Pp = PB[(q + 1) & 1];           // panel q - 1
            const cplx<T>* LD = LDB[(q + 1) & 1];
            if (q > 0) {
                // ---- panel q - 1 on block q (position 0), then hand-over: the
                // tiles of block q into P; the block at position 4 moves to
                // slot 0, block q + 8 enters slot 1
#pragma unroll
                for (int ra = 0; ra < 8; ++ra) {
                    if (owns(q, ra)) {
                        tile_mfma(accR[0][ra], accI[0][ra], Pp, LD, 0, ra);
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            P[(16 * ra + li) * RPS + 4 * lk + j] = cplx<T>{accR[0][ra][j], accI[0][ra][j]};
                        accR[0][ra] = accR[1][ra];
                        accI[0][ra] = accI[1][ra];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const bool ok = tile_ok(q + 8, ra, j);
                            accR[1][ra][j] = ok ? pf[ra & 1][j].re : T(0);
                            accI[1][ra][j] = ok ? pf[ra & 1][j].im : T(0);
                        }
                    }
                }
                P[r8r * RPS + r8c] = cplx<T>{row8_ok(q) ? r8.re : T(0), row8_ok(q) ? r8.im : T(0)};
                prefetch(q + 9);                          // for the next hand-over
                r8 = row8_load(q + 1);
            }
            __syncthreads();
            // ---- panel q - 1 on positions 1-7 (block q + m at position m: slot m > 4)
            if (q > 0) {
#pragma unroll
                for (int m = 1; m < 8; ++m) {
                    if (q + m < nblk) {
#pragma unroll
                        for (int ra = 0; ra < 8 - m; ++ra) {
                            if (!owns(q + m, ra)) continue;
                            tile_mfma(accR[m > 4][ra], accI[m > 4][ra], Pp, LD, m, ra);
                        }
                    }
                }
            }
            __syncthreads();
        }
        return;
    }

    // ================= chain waves =================
    int ecol[EP], erow[EP];
#pragma unroll
    for (int j = 0; j < EP; ++j) {
        const int e = tid + 256 * j;
        ecol[j] = e / bp1;
        erow[j] = e - ecol[j] * bp1 + ecol[j];            // panel row of band entry (column, d)
    }
    // finished panel q to HBM: rows of the diagonal block from PD, the others from P
    auto write_out = [&](int q) {
        const cplx<T>* P = PB[q & 1];
        cplx<T>* dst = base + (size_t)16 * q * bp1;
        const int nb = min(16, Mx - 16 * q);
#pragma unroll
        for (int j = 0; j < EP; ++j) {
            const int e = tid + 256 * j;
            if (e < 16 * bp1 && ecol[j] < nb) {
                const cplx<T>* src = erow[j] < 16 ? PD + erow[j] * RPS + ecol[j] : P + erow[j] * RPS + ecol[j];
                dst[e] = cplx<T>{src->re, src->im};
            }
        }
    };
    const bool own = lane < 48;
    const int rrel = lane < 16 ? lane : 16 + 32 * wave + (lane - 16);
    __syncthreads();

    for (int q = 0; q < nblk; ++q) {
        cplx<T>* P = PB[q & 1];
        cplx<T>* LD = LDB[q & 1];
        const int nb = min(16, Mx - 16 * q);
        if (q > 0) write_out(q - 1);
        __syncthreads();
        // ---- factor panel q in registers (one row per lane: lanes 0-15 the
        // diagonal block in every wave, lanes 16-47 of wave w rows 16 + 32 w ..)
        cplx<T> a[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const cplx<T>* e = P + (own ? rrel : 0) * RPS + c;
            a[c] = cplx<T>{e->re, e->im};
        }
        int bad = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < nb) {
                const cplx<T> dk = {lane_bcast(a[k].re, k), lane_bcast(a[k].im, k)};
                const cplx<T> inv = cinv_fast(dk);
                const T mag = fabs(dk.re) + fabs(dk.im);
                bad |= int(!(mag > T(0))) | int(!isfinite(mag));
                const cplx<T> aik = a[k];
                if (rrel > k) a[k] = cmul(aik, inv);
#pragma unroll
                for (int j = k + 1; j < 16; ++j) {
                    const T lr = lane_bcast(a[k].re, j), lim = lane_bcast(a[k].im, j);
                    a[j].re = fma(-aik.re, lr, a[j].re);
                    a[j].re = fma(aik.im, lim, a[j].re);
                    a[j].im = fma(-aik.re, lim, a[j].im);
                    a[j].im = fma(-aik.im, lr, a[j].im);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (tid == 0 && bad != 0) atomicOr(flag, 1);
        // the diagonal entries D_c of this panel, from the diagonal lanes
        cplx<T> dc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) dc[c] = cplx<T>{lane_bcast(a[c].re, c), lane_bcast(a[c].im, c)};
        if (own && lane >= 16) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                P[rrel * RPS + c] = a[c];
                LD[(rrel - 16) * RPS + c] = cmul(a[c], dc[c]);
            }
        }
        if (wave == 0 && lane < 16) {
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c <= lane) PD[lane * RPS + c] = a[c];
        }
        __syncthreads();
    }
    write_out(nblk - 1);
}

// ---------------------------------------------------------------------------
// Bands up to 256 with the panel in registers and the trailing tiles
// streamed, one workgroup of 8 waves per system.  Panel q (columns p0 = 16 q
// .. p0 + 15), with nr = reach[q] row blocks below its diagonal block (the
// envelope of the factor: blocks further down are zero and stay zero):
//  1. every lane that owns a panel row holds its 16 entries in registers
//     (lanes 0-15 of every wave the rows of the diagonal block, lanes 16-47
//     of wave w the rows p0 + 16 + 32 w + (lane - 16)); the rows the previous
//     panel updated come from the hand-over buffer in LDS, the others from
//     HBM, loaded a panel ahead;
//  2. the panel is factored in registers with lane broadcasts, no barrier;
//  3. the factored panel is written to HBM once, and its rows below the
//     diagonal block (L) with D go to LDS, the operands of the update;
//  4. the trailing tiles (ti, tj), tj <= ti < nr, are dealt round-robin to
//     the 8 waves; a tile is read from HBM (the next one of the wave in
//     flight meanwhile), updated on the matrix cores, C -= L_c (L_r D)^T as
//     four real 16x16x4 MFMAs per complex k-step, and written back.  The
//     tiles of column block q + 1 (tj = 0) are the next panel: they go to
//     the hand-over buffer instead of HBM.
// LDS: L rows [256][PS], hand-over [256][PS] (complex), D [16].
// ---------------------------------------------------------------------------
constexpr int PS = 17;                                    // LDS row stride (complex) of the panel buffers

// One system; REAL: the system is real (lambda real, every imaginary part
// zero), so only the real parts are computed (a quarter of the MFMAs) and the
// stored imaginary parts stay zero.  The results are those of the complex
// form on the same system: its imaginary terms are exact zeros.
// t = ti (ti + 1) / 2 + tj with 0 <= tj <= ti (the tiles of a triangle, row
// by row): ti from the square root, corrected by one either way for the
// float's rounding.  (The counting loop it replaces took about 100 scalar
// instructions per tile near the end of a b = 256 triangle.)
__device__ __forceinline__ void tri_index(int t, int& ti, int& tj) {
    int r = (int)((__builtin_sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    r += (r + 1) * (r + 2) / 2 <= t ? 1 : 0;
    r -= r * (r + 1) / 2 > t ? 1 : 0;
    ti = r;
    tj = t - r * (r + 1) / 2;
}

template <typename T, bool REAL>
__device__ __forceinline__ void panel_factor_system(cplx<T>* __restrict__ base, int Mx, int bp,
                                                    const int* __restrict__ reach, int* __restrict__ flag,
                                                    unsigned char* smem_raw) {
    using V4 = typename vec4<T>::type;
    cplx<T>* PL = reinterpret_cast<cplx<T>*>(smem_raw);   // L of the rows below the diagonal block
    cplx<T>* NX = PL + 256 * PS;                          // hand-over: the next panel's updated rows
    cplx<T>* PD = NX + 256 * PS;                          // D of the panel
    // (complex values as 2-vectors: builtin assignment through the typed
    // pointers)
    using V2 = T __attribute__((ext_vector_type(2)));
    using LdsV2 = __attribute__((address_space(3))) V2;
    using GlbV2 = __attribute__((address_space(1))) V2;
    LdsV2* NXs = (LdsV2*)NX;
    GlbV2* gbase = (GlbV2*)base;
    const int bp1 = bp + 1;
    const int NB = bp / 16;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int lane = tid & 63;
    int li = lane & 15, lk = lane >> 4;
    const int nblk = (Mx + 15) / 16;
    const cplx<T> zero = {T(0), T(0)};
    // this lane's panel row, relative to p0
    bool own = lane < 48;
    int rrel = lane < 16 ? lane : 16 + 32 * wave + (lane - 16);
    // the lane indices again at the start of every pass, through an opaque
    // move: the lane conditions built on them (d >= 0, rrel > k, ...) are
    // then formed inside the pass, not hoisted out of the pass loop as
    // 64-bit scalar masks held across it, which the compiler spilled to
    // vector lanes by the hundreds (about 500 scalar spills; 4-5% of the
    // factor's time.  The two-panel kernel measured slower with it.)
    auto lane_indices = [&]() {
        lane = opaque_int(tid & 63);
        li = lane & 15;
        lk = lane >> 4;
        own = lane < 48;
        rrel = lane < 16 ? lane : 16 + 32 * wave + (lane - 16);
    };

    // entry (p0 + rrel, p0 + c) of the band, clamped address, and whether it exists
    auto ent_on = [&](int p0, int c, int nrow) {
        const int d = rrel - c;
        return own && rrel < nrow && d >= 0 && d <= bp && p0 + rrel < Mx && p0 + c < Mx;
    };
    // (offsets within one system fit in 32 bits: M_x (bp + 1) < 2^31, checked
    // by the launcher; 32-bit selects keep the address arithmetic branch-free)
    auto ent_off = [&](int p0, int c, int nrow, int lo) -> int {
        return ent_on(p0, c, nrow) && rrel >= lo ? (p0 + c) * bp1 + (rrel - c) : 0;
    };
    // raw loads of this lane's row of panel starting at p0 (rows lo .. nrow - 1;
    // every lane loads, the others from offset 0)
    cplx<T> pf[16];
    auto prefetch = [&](int p0, int nrow, int lo) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const cplx<T>* e = base + ent_off(p0, c, nrow, lo);
            pf[c].re = e->re;
            pf[c].im = e->im;
        }
    };
    int nr_prev = 0;                                      // row blocks the previous panel updated
    prefetch(0, nblk > 0 ? 16 + 16 * min(NB, reach[0]) : 0, 0);

    for (int q = 0; q < nblk; ++q) {
        lane_indices();
        const int p0 = 16 * q;
        const int nb = min(16, Mx - p0);
        const int nr = min(NB, reach[q]);
        const int nrow = 16 + 16 * nr;                    // rows of the panel
        // ---- 1. the panel row: hand-over buffer (rows the previous panel
        // updated) or the prefetched HBM values
        cplx<T> a[16];
        const bool from_nx = rrel < 16 * nr_prev;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const bool on = ent_on(p0, c, nrow);
            const cplx<T> x = NX[(from_nx ? rrel : 0) * PS + c];
            a[c].re = on ? (from_nx ? x.re : pf[c].re) : T(0);
            a[c].im = on ? (from_nx ? x.im : pf[c].im) : T(0);
        }
        // the next panel's rows this panel does not update: from HBM now
        if (q + 1 < nblk) {
            const int nrow1 = 16 + 16 * min(NB, reach[q + 1]);
            // rows of panel q + 1 at or beyond 16 nr (relative to its start)
            // are untouched by any earlier panel
            prefetch(p0 + 16, nrow1, 16 * nr);
        }
        // ---- 2. factor the panel in registers
        int bad = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < nb) {
                const cplx<T> dk = {lane_bcast(a[k].re, k), lane_bcast(a[k].im, k)};
                const cplx<T> inv = cinv_fast(dk);
                const T mag = fabs(dk.re) + fabs(dk.im);
                bad |= int(!(mag > T(0))) | int(!isfinite(mag));
                const cplx<T> aik = a[k];
                if constexpr (REAL) {
                    if (rrel > k) a[k].re = aik.re * inv.re;
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) a[j].re = fma(-aik.re, lane_bcast(a[k].re, j), a[j].re);
                } else {
                    if (rrel > k) a[k] = cmul(aik, inv);
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) {
                        const T lr = lane_bcast(a[k].re, j), lim = lane_bcast(a[k].im, j);
                        a[j].re = fma(-aik.re, lr, a[j].re);
                        a[j].re = fma(aik.im, lim, a[j].re);
                        a[j].im = fma(-aik.re, lim, a[j].im);
                        a[j].im = fma(-aik.im, lr, a[j].im);
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (tid == 0 && bad != 0) atomicOr(flag, 1);
        // ---- 3. write the panel out; L rows and D to LDS
        const bool writer = own && (lane >= 16 || wave == 0);
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (writer && c < nb && ent_on(p0, c, nrow)) base[(p0 + c) * bp1 + (rrel - c)] = a[c];
        if (own && lane >= 16) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                // component-wise selects (a select of whole structs becomes a
                // load through a selected address, with a[] in scratch memory)
                const bool in = rrel < nrow;
                PL[(rrel - 16) * PS + c] = cplx<T>{in ? a[c].re : T(0), in ? a[c].im : T(0)};
            }
        }
        {
            // the diagonal entry a[lane] of this lane's row, by selects (an
            // index by lane would put a[] in scratch memory)
            cplx<T> dg = a[0];
#pragma unroll
            for (int c = 1; c < 16; ++c) {
                dg.re = lane == c ? a[c].re : dg.re;
                dg.im = lane == c ? a[c].im : dg.im;
            }
            if (wave == 0 && lane < 16) PD[lane] = dg;
        }
        __syncthreads();
        // ---- 4. trailing tiles, wave w takes tiles w, w + 8, ...
        const int ntile = nr * (nr + 1) / 2;
        auto tile_ij = [](int t, int& ti, int& tj) { tri_index(t, ti, tj); };
        // element j of this lane in tile (ti, tj): row r = p0 + 16 + 16 ti + li,
        // column c' = p0 + 16 + 16 tj + mfma_row(lk, j)
        auto c_on = [&](int ti, int tj, int j) {
            const int r = p0 + 16 + 16 * ti + li, cc = p0 + 16 + 16 * tj + mfma_row<T>(lk, j);
            const int d = r - cc;
            return d >= 0 && d <= bp && r < Mx && cc < Mx;
        };
        // raw loads of tile t (t >= ntile: of the last tile, the values
        // unused; one address pattern for every call keeps the loads in
        // flight without waits)
        auto c_load = [&](int t, cplx<T> (&cv)[4]) {
            int ti, tj;
            tile_ij(min(t, ntile - 1), ti, tj);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = p0 + 16 + 16 * ti + li, cc = p0 + 16 + 16 * tj + mfma_row<T>(lk, j);
                const int off = c_on(ti, tj, j) ? cc * bp1 + (r - cc) : 0;
                const cplx<T>* e = base + off;
                cv[j].re = e->re;
                cv[j].im = e->im;
            }
        };
        auto c_update = [&](int t, const cplx<T> (&cv)[4]) {
            int ti, tj;
            tile_ij(t, ti, tj);
            // the panel's contribution is summed on its own and subtracted
            // once: C rounds once per panel, not after every MFMA
            V4 ur = zero4<T>(), ui = zero4<T>();
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                if constexpr (REAL) {
                    ur = mfma16x16x4<T>(PL[(16 * tj + li) * PS + k].re,
                                        PL[(16 * ti + li) * PS + k].re * PD[k].re, ur);
                } else {
                    const cplx<T> x = PL[(16 * tj + li) * PS + k];              // column side: L
                    const cplx<T> y = cmul(PL[(16 * ti + li) * PS + k], PD[k]);  // row side: L D
                    ur = mfma16x16x4<T>(x.re, y.re, ur);
                    ui = mfma16x16x4<T>(x.re, y.im, ui);
                    ur = mfma16x16x4<T>(-x.im, y.im, ur);
                    ui = mfma16x16x4<T>(x.im, y.re, ui);
                }
            }
            // the LDS and HBM stores through pointers of their own address
            // spaces: one store through a generic pointer for both (which
            // the compiler would otherwise make of the two branches) waits
            // on every load in flight
            if (tj == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (c_on(ti, tj, j))
                        NXs[(16 * ti + li) * PS + mfma_row<T>(lk, j)] = V2{cv[j].re - ur[j], cv[j].im - ui[j]};
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = p0 + 16 + 16 * ti + li, cc = p0 + 16 + 16 * tj + mfma_row<T>(lk, j);
                    if (c_on(ti, tj, j)) gbase[cc * bp1 + (r - cc)] = V2{cv[j].re - ur[j], cv[j].im - ui[j]};
                }
            }
        };
        {
            // NB tile buffers in straight-line code (each a fixed set of
            // registers): the loads of the wave's next NB - 1 tiles are in
            // flight while a tile is updated (FP32 3, FP64 2); the loads are
            // unconditional, only the update is skipped past the last tile
            constexpr int NB = sizeof(T) == 4 ? 4 : 3;
            cplx<T> cb[NB][4];
            int t = wave;
#pragma unroll
            for (int i = 0; i + 1 < NB; ++i) c_load(t + 8 * i, cb[i]);
            while (t < ntile) {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    c_load(t + 8 * (NB - 1), cb[(i + NB - 1) % NB]);
                    if (t < ntile) c_update(t, cb[i]);
                    t += 8;
                }
            }
        }
        nr_prev = nr;
        __syncthreads();
    }
}

// Systems [0, ncplx) complex, one per workgroup; systems [ncplx, nsys) real,
// two per workgroup one after the other (each costs about a quarter of a
// complex one), so that, e.g., 2 p + 2 systems make 2 p + 1 workgroups.
template <typename T>
__global__ void __launch_bounds__(512) band_ldl_panel_kernel(cplx<T>* __restrict__ LB, int Mx, int bp, int ncplx,
                                                            int nsys, const int* __restrict__ reach,
                                                            int* __restrict__ flag) {
    extern __shared__ unsigned char smem_raw[];
    const size_t stride = (size_t)Mx * (bp + 1);
    const int b = blockIdx.x;
    if (b < ncplx) {
        panel_factor_system<T, false>(LB + (size_t)b * stride, Mx, bp, reach, flag, smem_raw);
        return;
    }
    const int s0 = ncplx + 2 * (b - ncplx);
    panel_factor_system<T, true>(LB + (size_t)s0 * stride, Mx, bp, reach, flag, smem_raw);
    if (s0 + 1 < nsys) {
        __syncthreads();
        panel_factor_system<T, true>(LB + (size_t)(s0 + 1) * stride, Mx, bp, reach, flag, smem_raw);
    }
}

// ---------------------------------------------------------------------------
// Bands up to 256 with two 16-column panels per pass (FP32): the trailing
// tiles take the update of both panels, 32 terms, for one read and one write,
// half the tile traffic of the kernel above.  Pass Q (blocks b0 = 2Q and
// b1 = 2Q + 1, columns p0 = 32 Q .. p0 + 31, p1 = p0 + 16):
//  1. panel 0 (block b0) is factored in registers as above (its rows from
//     the hand-over NX0 or HBM), written out, its rows below the diagonal
//     block and D to LDS (PL0, PD0);
//  2. panel 1's column (block b1, rows of its band) sits in LDS (NX1: handed
//     over by the previous pass, the rest loaded from HBM a step ahead) and
//     takes panel 0's update there (tiles on the matrix cores);
//  3. panel 1 is factored in registers from NX1, written out, PL1 and PD1 to
//     LDS;
//  4. the trailing tiles right of block b1 take both panels' update, each
//     summed on its own: C - L0 D0 L0^T - L1 D1 L1^T, the roundings of two
//     passes of the one-panel kernel (whose factor this one reproduces bit
//     for bit); the tiles of blocks b0 + 2 and b0 + 3 (the next pass's
//     panels) go to NX0 and NX1 instead of HBM.
// LDS (complex, stride PS): PL0 [272], PL1 [256], NX0 [256], NX1 [272] rows,
// PD0 and PD1: 138.4 KB in FP32.
// ---------------------------------------------------------------------------
constexpr int P2_ROWS0 = 272, P2_ROWS1 = 256, P2_NX0 = 256, P2_NX1 = 272;

template <typename T>
static size_t panel2_smem() {
    return ((size_t)(P2_ROWS0 + P2_ROWS1 + P2_NX0 + P2_NX1) * PS + 32) * sizeof(cplx<T>);
}

template <typename T, bool REAL>
__device__ __forceinline__ void panel2_factor_system(cplx<T>* __restrict__ base, int Mx, int bp,
                                                     const int* __restrict__ reach, int* __restrict__ flag,
                                                     unsigned char* smem_raw) {
    using V4 = typename vec4<T>::type;
    cplx<T>* PL0 = reinterpret_cast<cplx<T>*>(smem_raw);  // panel 0's L rows below its diagonal block (row p1 + r)
    cplx<T>* PL1 = PL0 + P2_ROWS0 * PS;                   // panel 1's L rows below its diagonal block (p1 + 16 + r)
    cplx<T>* NX0 = PL1 + P2_ROWS1 * PS;                   // hand-over: the next panel 0's rows (p0 + r)
    cplx<T>* NX1 = NX0 + P2_NX0 * PS;                     // panel 1's column (p1 + r)
    cplx<T>* PD0 = NX1 + P2_NX1 * PS;
    cplx<T>* PD1 = PD0 + 16;
    using V2 = T __attribute__((ext_vector_type(2)));
    using LdsV2 = __attribute__((address_space(3))) V2;
    using GlbV2 = __attribute__((address_space(1))) V2;
    LdsV2* NX0s = (LdsV2*)NX0;
    LdsV2* NX1s = (LdsV2*)NX1;
    GlbV2* gbase = (GlbV2*)base;
    const int bp1 = bp + 1;
    const int NB = bp / 16;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int nblk = (Mx + 15) / 16;
    const bool own = lane < 48;
    const int rrel = lane < 16 ? lane : 16 + 32 * wave + (lane - 16);

    auto ent_on = [&](int p0, int c, int nrow) {
        const int d = rrel - c;
        return own && rrel < nrow && d >= 0 && d <= bp && p0 + rrel < Mx && p0 + c < Mx;
    };
    auto ent_off = [&](int p0, int c, int nrow, int lo) -> int {
        return ent_on(p0, c, nrow) && rrel >= lo ? (p0 + c) * bp1 + (rrel - c) : 0;
    };
    cplx<T> pf[16];
    auto prefetch = [&](int p0, int nrow, int lo) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const cplx<T>* e = base + ent_off(p0, c, nrow, lo);
            pf[c].re = e->re;
            pf[c].im = e->im;
        }
    };
    // factor the 16 columns of this lane's panel row in registers (lane
    // broadcasts, no barrier); returns the bad-pivot flag
    auto factor_row = [&](cplx<T> (&a)[16], int nb) {
        int bad = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < nb) {
                const cplx<T> dk = {lane_bcast(a[k].re, k), lane_bcast(a[k].im, k)};
                const cplx<T> inv = cinv_fast(dk);
                const T mag = fabs(dk.re) + fabs(dk.im);
                bad |= int(!(mag > T(0))) | int(!isfinite(mag));
                const cplx<T> aik = a[k];
                if constexpr (REAL) {
                    if (rrel > k) a[k].re = aik.re * inv.re;
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) a[j].re = fma(-aik.re, lane_bcast(a[k].re, j), a[j].re);
                } else {
                    if (rrel > k) a[k] = cmul(aik, inv);
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) {
                        const T lr = lane_bcast(a[k].re, j), lim = lane_bcast(a[k].im, j);
                        a[j].re = fma(-aik.re, lr, a[j].re);
                        a[j].re = fma(aik.im, lim, a[j].re);
                        a[j].im = fma(-aik.re, lim, a[j].im);
                        a[j].im = fma(-aik.im, lr, a[j].im);
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        return bad;
    };
    // write a factored panel out, its L rows (zero past nrow) to PL and D to PD
    auto panel_out = [&](const cplx<T> (&a)[16], int p0, int nb, int nrow, cplx<T>* PL, cplx<T>* PD) {
        const bool writer = own && (lane >= 16 || wave == 0);
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (writer && c < nb && ent_on(p0, c, nrow)) base[(p0 + c) * bp1 + (rrel - c)] = a[c];
        if (own && lane >= 16) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const bool in = rrel < nrow;
                PL[(rrel - 16) * PS + c] = cplx<T>{in ? a[c].re : T(0), in ? a[c].im : T(0)};
            }
        }
        cplx<T> dg = a[0];
#pragma unroll
        for (int c = 1; c < 16; ++c) {
            dg.re = lane == c ? a[c].re : dg.re;
            dg.im = lane == c ? a[c].im : dg.im;
        }
        if (wave == 0 && lane < 16) PD[lane] = dg;
    };
    auto tile_ij = [](int t, int& ti, int& tj) { tri_index(t, ti, tj); };
    // this lane's share of a tile update: u = sum_k x_k (y_k d_k) over the
    // panel's 16 columns (x: column-side rows, y: row-side rows of PL)
    auto tile_sum = [&](V4& ur, V4& ui, const cplx<T>* PL, const cplx<T>* PD, int xrow, int yrow) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * kk + lk;
            if constexpr (REAL) {
                ur = mfma16x16x4<T>(PL[(xrow + li) * PS + k].re, PL[(yrow + li) * PS + k].re * PD[k].re, ur);
            } else {
                const cplx<T> x = PL[(xrow + li) * PS + k];
                const cplx<T> y = cmul(PL[(yrow + li) * PS + k], PD[k]);
                ur = mfma16x16x4<T>(x.re, y.re, ur);
                ui = mfma16x16x4<T>(x.re, y.im, ui);
                ur = mfma16x16x4<T>(-x.im, y.im, ur);
                ui = mfma16x16x4<T>(x.im, y.re, ui);
            }
        }
    };

    // PL0 rows 256 .. 271 (row p1 + 256 and below: never inside panel 0's
    // band) stay zero
    for (int e = tid; e < (P2_ROWS0 - 256) * PS; e += blockDim.x) PL0[256 * PS + e] = cplx<T>{T(0), T(0)};
    int nx0 = 0, nx1 = 0;                                 // rows of NX0 / NX1 handed over
    prefetch(0, nblk > 0 ? 16 + 16 * min(NB, reach[0]) : 0, 0);

    for (int b0 = 0; b0 < nblk; b0 += 2) {
        const int b1 = b0 + 1;
        const bool has1 = b1 < nblk;
        const int p0 = 16 * b0, p1 = p0 + 16;
        const int nb0 = min(16, Mx - p0), nb1 = has1 ? min(16, Mx - p1) : 0;
        const int nr0 = min(NB, reach[b0]), nr1 = has1 ? min(NB, reach[b1]) : 0;
        const int nrow0 = 16 + 16 * nr0, nrow1 = has1 ? 16 + 16 * nr1 : 0;
        // ---- 1. panel 0 from the hand-over or the prefetched HBM rows
        cplx<T> a[16];
        {
            const bool from_nx = rrel < nx0;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const bool on = ent_on(p0, c, nrow0);
                const cplx<T> x = NX0[(from_nx ? rrel : 0) * PS + c];
                a[c].re = on ? (from_nx ? x.re : pf[c].re) : T(0);
                a[c].im = on ? (from_nx ? x.im : pf[c].im) : T(0);
            }
        }
        // panel 1's rows not handed over: from HBM now (untouched so far)
        if (has1) prefetch(p1, nrow1, nx1);
        int bad = factor_row(a, nb0);
        panel_out(a, p0, nb0, nrow0, PL0, PD0);
        // the prefetched rows of panel 1's column join the hand-over
        if (has1 && own && rrel >= nx1 && rrel < nrow1) {
#pragma unroll
            for (int c = 0; c < 16; ++c) NX1[rrel * PS + c] = pf[c];
        }
        __syncthreads();
        // ---- 2. panel 0's update of panel 1's column: tiles (ti, 0) right
        // below panel 0's diagonal block, ti < nr0, in NX1
        if (has1) {
            for (int ti = wave; ti < nr0; ti += 8) {
                V4 ur = zero4<T>(), ui = zero4<T>();
                tile_sum(ur, ui, PL0, PD0, 0, 16 * ti);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = 16 * ti + li, cc = mfma_row<T>(lk, j);     // relative to p1
                    const int d = r - cc;
                    if (d >= 0 && d <= bp && p1 + r < Mx && p1 + cc < Mx) {
                        const cplx<T> c0 = NX1[r * PS + cc];
                        NX1s[r * PS + cc] = V2{c0.re - ur[j], c0.im - ui[j]};
                    }
                }
            }
        }
        __syncthreads();
        // ---- 3. panel 1 from NX1, factored; the next panel 0's rows that
        // this pass does not update: from HBM now
        const int nt = has1 ? max(nr0 - 1, nr1) : 0;      // row blocks of the trailing update
        if (has1) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const bool on = ent_on(p1, c, nrow1);
                const cplx<T> x = NX1[(on ? rrel : 0) * PS + c];
                a[c].re = on ? x.re : T(0);
                a[c].im = on ? x.im : T(0);
            }
        }
        if (b0 + 2 < nblk) prefetch(p0 + 32, 16 + 16 * min(NB, reach[b0 + 2]), 16 * nt);
        if (has1) {
            bad |= factor_row(a, nb1);
            panel_out(a, p1, nb1, nrow1, PL1, PD1);
        }
        if (tid == 0 && bad != 0) atomicOr(flag, 1);
        __syncthreads();
        // ---- 4. trailing tiles (ti, tj), tj <= ti < nt, of the rows and
        // columns from q1 = p1 + 16 on, dealt round-robin to the waves
        const int q1 = p1 + 16;
        const int ntile = nt * (nt + 1) / 2;
        auto c_on = [&](int ti, int tj, int j) {
            const int r = q1 + 16 * ti + li, cc = q1 + 16 * tj + mfma_row<T>(lk, j);
            const int d = r - cc;
            return d >= 0 && d <= bp && r < Mx && cc < Mx;
        };
        auto c_load = [&](int t, cplx<T> (&cv)[4]) {
            int ti, tj;
            tile_ij(min(t, ntile - 1), ti, tj);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = q1 + 16 * ti + li, cc = q1 + 16 * tj + mfma_row<T>(lk, j);
                const int off = c_on(ti, tj, j) ? cc * bp1 + (r - cc) : 0;
                const cplx<T>* e = base + off;
                cv[j].re = e->re;
                cv[j].im = e->im;
            }
        };
        // each panel's update summed on its own and subtracted in panel
        // order, C - u0 - u1: the roundings of the one-panel kernel, whose
        // factor this one reproduces bit for bit
        auto c_update = [&](int t, const cplx<T> (&cv)[4]) {
            int ti, tj;
            tile_ij(t, ti, tj);
            V4 ur0 = zero4<T>(), ui0 = zero4<T>(), ur1 = zero4<T>(), ui1 = zero4<T>();
            tile_sum(ur0, ui0, PL0, PD0, 16 + 16 * tj, 16 + 16 * ti);
            tile_sum(ur1, ui1, PL1, PD1, 16 * tj, 16 * ti);
            V2 v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = V2{(cv[j].re - ur0[j]) - ur1[j], (cv[j].im - ui0[j]) - ui1[j]};
            if (tj == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (c_on(ti, tj, j)) NX0s[(16 * ti + li) * PS + mfma_row<T>(lk, j)] = v[j];
            } else if (tj == 1) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (c_on(ti, tj, j)) NX1s[(16 * (ti - 1) + li) * PS + mfma_row<T>(lk, j)] = v[j];
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = q1 + 16 * ti + li, cc = q1 + 16 * tj + mfma_row<T>(lk, j);
                    if (c_on(ti, tj, j)) gbase[cc * bp1 + (r - cc)] = v[j];
                }
            }
        };
        {
            constexpr int NBUF = 4;
            cplx<T> cb[NBUF][4];
            int t = wave;
#pragma unroll
            for (int i = 0; i + 1 < NBUF; ++i) c_load(t + 8 * i, cb[i]);
            while (t < ntile) {
#pragma unroll
                for (int i = 0; i < NBUF; ++i) {
                    c_load(t + 8 * (NBUF - 1), cb[(i + NBUF - 1) % NBUF]);
                    if (t < ntile) c_update(t, cb[i]);
                    t += 8;
                }
            }
        }
        nx0 = 16 * nt;
        nx1 = max(0, 16 * (nt - 1));
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(512) band_ldl_panel2_kernel(cplx<T>* __restrict__ LB, int Mx, int bp, int ncplx,
                                                             int nsys, const int* __restrict__ reach,
                                                             int* __restrict__ flag) {
    extern __shared__ unsigned char smem_raw[];
    const size_t stride = (size_t)Mx * (bp + 1);
    const int b = blockIdx.x;
    if (b < ncplx) {
        panel2_factor_system<T, false>(LB + (size_t)b * stride, Mx, bp, reach, flag, smem_raw);
        return;
    }
    const int s0 = ncplx + 2 * (b - ncplx);
    panel2_factor_system<T, true>(LB + (size_t)s0 * stride, Mx, bp, reach, flag, smem_raw);
    if (s0 + 1 < nsys) {
        __syncthreads();
        panel2_factor_system<T, true>(LB + (size_t)(s0 + 1) * stride, Mx, bp, reach, flag, smem_raw);
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

// LDS of the window factorization, and whether it is used for this band
template <typename T>
static size_t window_smem(int bp) { return ((size_t)(bp + 16) * (bp + 1) + 1) * sizeof(cplx<T>); }
template <typename T>
static bool use_window(int bp) { return bp <= 128 && window_smem<T>(bp) <= 150 * 1024; }

static size_t stream_smem(int bp, size_t es) { return 2 * 16 * (size_t)(bp + 1) * es; }
template <typename T>
static size_t panel_smem() { return (2 * 256 * (size_t)PS + 16) * sizeof(cplx<T>); }



template <typename T>
size_t band_ldl_smem(int bp) {
    // (the two-panel kernel, FP32 only, needs more: its launch requests it)
    return use_window<T>(bp) ? window_smem<T>(bp) : std::max(stream_smem(bp, sizeof(T)), panel_smem<T>());
}

template <typename T>
hipError_t launch_band_ldl(void* LB, int Mx, int bp, int nsys, int nreal, const int* reach, int* flag,
                           int kernel, hipStream_t st) {
    if (nreal < 0 || nreal > nsys) return hipErrorInvalidValue;
    // the panel kernel takes the trailing real systems in pairs
    const int ncplx = nsys - nreal;
    const int nwg = ncplx + (nreal + 1) / 2;
    if constexpr (sizeof(T) == 4) {
        // FP32: the two-panel kernel is also the automatic choice where the
        // one-panel kernel would be
        if (kernel == FACTOR_PANEL2 || (kernel == FACTOR_AUTO && !use_window<T>(bp) && bp != 128)) {
            if (bp > 256 || bp % 16 != 0 || (size_t)Mx * (bp + 1) >= ((size_t)1 << 31)) return hipErrorInvalidValue;
            const size_t smem = panel2_smem<T>();
            hipError_t e = hipFuncSetAttribute((const void*)band_ldl_panel2_kernel<T>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(band_ldl_panel2_kernel<T>, dim3(nwg), dim3(512), smem, st, static_cast<cplx<T>*>(LB),
                               Mx, bp, ncplx, nsys, reach, flag);
            return hipGetLastError();
        }
    } else {
        if (kernel == FACTOR_PANEL2) return hipErrorInvalidValue;   // its LDS does not fit in FP64
    }
    if (kernel == FACTOR_PANEL || (kernel == FACTOR_AUTO && !use_window<T>(bp) && !(sizeof(T) == 4 && bp == 128))) {
        if (bp > 256 || bp % 16 != 0 || (size_t)Mx * (bp + 1) >= ((size_t)1 << 31)) return hipErrorInvalidValue;
        const size_t smem = panel_smem<T>();
        hipError_t e = hipFuncSetAttribute((const void*)band_ldl_panel_kernel<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(band_ldl_panel_kernel<T>, dim3(nwg), dim3(512), smem, st, static_cast<cplx<T>*>(LB), Mx, bp,
                           ncplx, nsys, reach, flag);
        return hipGetLastError();
    }
    if (kernel == FACTOR_STREAM) {
        const size_t smem = stream_smem(bp, sizeof(T));
        hipError_t e = hipFuncSetAttribute((const void*)band_ldl_kernel<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(band_ldl_kernel<T>, dim3(nsys), dim3(256), smem, st, static_cast<cplx<T>*>(LB), Mx, bp,
                           flag);
        return hipGetLastError();
    }
    const size_t smem = use_window<T>(bp) ? window_smem<T>(bp) : stream_smem(bp, sizeof(T));
    if constexpr (sizeof(T) == 4) {
        if (bp == 128) {
            hipLaunchKernelGGL(band_ldl_reg_kernel, dim3(nsys), dim3(512), 0, st, static_cast<cplx<float>*>(LB), Mx,
                               flag);
            return hipGetLastError();
        }
    }
    if (use_window<T>(bp)) {
        hipError_t e = hipFuncSetAttribute((const void*)band_ldl_window_kernel<T, 128>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((band_ldl_window_kernel<T, 128>), dim3(nsys), dim3(256), smem, st,
                           static_cast<cplx<T>*>(LB), Mx, bp, flag);
        return hipGetLastError();
    }
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
template hipError_t launch_band_ldl<float>(void*, int, int, int, int, const int*, int*, int, hipStream_t);
template hipError_t launch_band_ldl<double>(void*, int, int, int, int, const int*, int*, int, hipStream_t);
template size_t band_ldl_smem<float>(int);
template size_t band_ldl_smem<double>(int);

}  // namespace stfd
