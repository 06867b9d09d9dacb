// Dense transforms of Algorithm FD (steps 2 and 4, Sec. 4.4) and the FP64
// residual of the refinement, as matrix-core (MFMA) GEMMs, plus the sparse
// spatial operator and small helpers.
//
// Every GEMM here has the shape  C (M x N) = A (M x K) * B (K x N)  with
//   A column-major (the space-time block, M = M_x rows, i fastest),
//   B row-major and shared by the batch (the small time-side factor),
//   C column-major,
// batched over right-hand sides.  M is large (1e4..1e5) and N, K <= 2 N_t.
// A 64 x 64 output tile per workgroup, 4 waves of 32 x 32, K in steps of 16
// staged through LDS; each wave issues 16x16x4 MFMAs with the B tile as the
// first operand so that the output lane index runs along M (coalesced
// column-major stores).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace stfd {

constexpr int BN = 64, BK = 16;

// TM 16-row MFMA tiles per wave along M: the workgroup tile is (32 TM) x 64
// (TM = 2: 64 x 64, TM = 4: 128 x 64).  NFAST: blockIdx.x runs over the N
// tiles (the workgroups that share an A panel run side by side) instead of
// the M tiles.
template <typename TA, typename TC, int EPI, int TM, bool NFAST>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    if (g.gate && *g.gate) return;
    constexpr int BMT = 32 * TM;
    constexpr int RA = BMT / 64;                 // A rows per thread and k
    __shared__ TC As[BK][BMT];
    __shared__ TC Bs[BK][BN];
    __shared__ double red[8];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m0 = (NFAST ? blockIdx.y : blockIdx.x) * BMT, n0 = (NFAST ? blockIdx.x : blockIdx.y) * BN;
    const int batch = blockIdx.z;
    const TA* A = static_cast<const TA*>(g.A) + (size_t)batch * g.strideA;
    const TC* B = static_cast<const TC*>(g.B);
    const int wm = (wave & 1) * (16 * TM), wn = (wave >> 1) * 32;
    const int li = lane & 15, lk = lane >> 4;

    typename vec4<TC>::type acc[2][TM];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < TM; ++b) acc[a][b] = zero4<TC>();

    // global -> registers for the K step at k0 (A coalesced along m, B along
    // n); the next step's loads are in flight while this one computes
    TC ra[4][RA], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = tid & 63, k = (tid >> 6) + 4 * i;
            const int gk = k0 + k;
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const int gm = m0 + m + 64 * r;
                ra[i][r] = gm < g.M && gk < g.K ? static_cast<TC>(A[(size_t)gm + (size_t)gk * g.lda]) : TC(0);
            }
            const int gn = n0 + m;
            rb[i] = gn < g.N && gk < g.K ? B[(size_t)gk * g.ldb + gn] : TC(0);
        }
    };
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = tid & 63, k = (tid >> 6) + 4 * i;
#pragma unroll
            for (int r = 0; r < RA; ++r) As[k][m + 64 * r] = ra[i][r];
            Bs[k][m] = rb[i];
        }
        __syncthreads();
        if (k0 + BK < g.K) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int k = 4 * kk + lk;
            TC bf[2], af[TM];
#pragma unroll
            for (int t = 0; t < 2; ++t) bf[t] = Bs[k][wn + 16 * t + li];
#pragma unroll
            for (int t = 0; t < TM; ++t) af[t] = As[k][wm + 16 * t + li];
#pragma unroll
            for (int tn = 0; tn < 2; ++tn)
#pragma unroll
                for (int tm = 0; tm < TM; ++tm) acc[tn][tm] = mfma16x16x4<TC>(bf[tn], af[tm], acc[tn][tm]);
        }
        __syncthreads();
    }

    // epilogue: acc[tn][tm][j] = C[m = m0 + wm + 16 tm + li][n = n0 + wn + 16 tn + mfma_row(lk, j)]
    double s_r = 0.0, s_f = 0.0;
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = m0 + wm + 16 * tm + li;
                const int n = n0 + wn + 16 * tn + mfma_row<TC>(lk, j);
                if (m >= g.M || n >= g.N) continue;
                const size_t off = (size_t)batch * g.strideC + (size_t)m + (size_t)n * g.ldc;
                const TC v = acc[tn][tm][j];
                if (EPI == EPI_STORE_F32) {
                    static_cast<float*>(g.C)[off] = static_cast<float>(v);
                } else if (EPI == EPI_STORE_F64) {
                    static_cast<double*>(g.C)[off] = static_cast<double>(v);
                } else if (EPI == EPI_ADD_F64) {
                    static_cast<double*>(g.C)[off] += g.alpha * static_cast<double>(v);
                } else {   // EPI_RESID: C = F - A B, sums of squares of C and F
                    const size_t foff = (size_t)batch * g.strideF + (size_t)m + (size_t)n * g.ldc;
                    const double f = static_cast<const double*>(g.F)[foff];
                    const double r = f - static_cast<double>(v);
                    static_cast<double*>(g.C)[off] = r;
                    s_r += r * r;
                    s_f += f * f;
                }
            }
    if (EPI == EPI_RESID) {
        const double tr = block_sum(s_r, red);
        const double tf = block_sum(s_f, red);
        if (tid == 0) {
            const size_t blocks = (size_t)gridDim.x * gridDim.y;
            const size_t idx = (size_t)batch * blocks + (size_t)blockIdx.y * gridDim.x + blockIdx.x;
            // (the partials of a RHS are summed in full, in any block order)
            g.partial[2 * idx] = tr;
            g.partial[2 * idx + 1] = tf;
        }
    }
}

// ---------------------------------------------------------------------------
// FP64-accumulating GEMMs with a 128 x 128 workgroup tile: 4 waves of 64 x 64
// (4 x 4 FP64 16x16x4 MFMA tiles each, 128 accumulator registers), K in
// steps of 16 through a double-buffered LDS (one barrier per step), the next
// step's tiles loaded into registers while the current one is on the matrix
// cores.  Against the 64 x 64 tile it halves the bytes per flop that every
// workgroup pulls through L2 (the small time-side factor B, re-read for
// every row panel, is the larger share).
//
// Tile order: workgroup i runs on XCD i mod 8; each XCD gets a contiguous
// range of the logical tiles.  Within a right-hand side the logical tiles
// run through groups of GM row panels: down the GM panels of one N tile,
// then the next N tile.  The 64 workgroups an XCD holds at once (32 CUs, two
// each) so cover about 8 row panels x 8 N tiles and share their A panels and
// B slabs in that XCD's L2: A and B each come from HBM about once per group
// instead of once per tile (rocprofv3 FETCH_SIZE of the 64 x 64 kernel,
// whose neighbouring tiles sit on different XCDs: 6.9x the algorithmic
// bytes for the residual GEMM, 20x for the forward transform).
// ---------------------------------------------------------------------------
constexpr int WBM = 128, WBN = 128, WPAD = 2, NXCD = 8, WGM = 8;

__host__ __device__ inline unsigned wide_tiles(int M, int N) {
    return (unsigned)((M + WBM - 1) / WBM) * (unsigned)((N + WBN - 1) / WBN);
}

template <typename TA, int EPI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) gemm_wide_kernel(GemmArgs g) {
    if (g.gate && *g.gate) return;
    __shared__ double As[2][BK][WBM + WPAD];
    __shared__ double Bs[2][BK][WBN + WPAD];
    __shared__ double red[8];
    const unsigned per = wide_tiles(g.M, g.N);
    const unsigned total = per * (unsigned)g.batch;
    const unsigned per_xcd = (total + NXCD - 1) / NXCD;
    const unsigned logical = (blockIdx.x % NXCD) * per_xcd + blockIdx.x / NXCD;
    if (logical >= total) return;
    const int batch = (int)(logical / per);
    const unsigned tile = logical % per;
    const int nt = (g.N + WBN - 1) / WBN, mt = (g.M + WBM - 1) / WBM;
    const int group = (int)(tile / (WGM * nt)), first_m = group * WGM;
    const int gsz = min(mt - first_m, WGM);
    const int in_group = (int)(tile % (WGM * nt));
    const int m0 = (first_m + in_group % gsz) * WBM, n0 = (in_group / gsz) * WBN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const TA* A = static_cast<const TA*>(g.A) + (size_t)batch * g.strideA;
    const double* B = static_cast<const double*>(g.B);

    typename vec4<double>::type acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = zero4<double>();

    // global -> registers: thread t loads rows / columns (t & 127) of k rows
    // (t >> 7) + 2 i.  Rows of A past M and columns of B past N are loaded
    // clamped (copies of the last one) and never masked: they only reach
    // rows and columns of C that are not stored.  Full K steps read at
    // loop-invariant 32-bit byte offsets from the step's first column of A
    // and row of B (workgroup-uniform pointers; the launcher checks that the
    // offsets fit); the last, partial step clamps k and zeroes the entries
    // past K.
    const int lr = tid & 127, lh = tid >> 7;
    const int gm = min(m0 + lr, g.M - 1), gn = min(n0 + lr, g.N - 1);
    uint32_t aoff[8], boff[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        aoff[i] = (uint32_t)(((lh + 2 * i) * (uint32_t)g.lda + gm) * sizeof(TA));
        boff[i] = (uint32_t)(((lh + 2 * i) * (uint32_t)g.ldb + gn) * sizeof(double));
    }
    TA ra[8];
    double rb[8];
    auto load = [&](int k0) {
        const char* Ak = reinterpret_cast<const char*>(A + (size_t)k0 * g.lda);
        const char* Bk = reinterpret_cast<const char*>(B + (size_t)k0 * g.ldb);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            ra[i] = *reinterpret_cast<const TA*>(Ak + aoff[i]);
            rb[i] = *reinterpret_cast<const double*>(Bk + boff[i]);
        }
    };
    auto load_tail = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int gk = min(k0 + lh + 2 * i, g.K - 1);
            ra[i] = A[(size_t)gm + (size_t)gk * g.lda];
            rb[i] = B[(size_t)gk * g.ldb + gn];
        }
    };
    auto load_any = [&](int k0) {
        if (k0 + BK <= g.K) load(k0);
        else load_tail(k0);
    };
    auto stash = [&](int buf, int k0) {
        const bool tail = k0 + BK > g.K;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = lh + 2 * i;
            const bool k_in = !tail || k0 + k < g.K;
            As[buf][k][lr] = k_in ? static_cast<double>(ra[i]) : 0.0;
            Bs[buf][k][lr] = k_in ? rb[i] : 0.0;
        }
    };
    // one k-step of 4: 16 MFMAs of the wave's 4 x 4 tiles
    auto mfma_k = [&](int buf, int kk) {
        const int k = 4 * kk + lk;
        double bf[4], af[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            bf[t] = Bs[buf][k][wn + 16 * t + li];
            af[t] = As[buf][k][wm + 16 * t + li];
        }
#pragma unroll
        for (int tn = 0; tn < 4; ++tn)
#pragma unroll
            for (int tm = 0; tm < 4; ++tm) acc[tn][tm] = mfma16x16x4<double>(bf[tn], af[tm], acc[tn][tm]);
    };
    load_any(0);
    stash(0, 0);
    __syncthreads();
    int buf = 0;
    int k0 = 0;
    // Steps whose next step is full, branch-free: the 64 MFMAs of the step
    // interleaved with the next step's 16 global loads (first half) and its
    // 16 LDS writes (second half, once the loads have had half a step), and
    // the LDS reads of the operands spread in between (scheduling groups),
    // so that the matrix cores keep issuing while the memory work goes on.
    // Against loads, MFMAs and LDS writes in three blocks this takes the
    // residual GEMM of the L-shape N_t = 1024 solve from 58 to 46 ms.
    for (; k0 + 2 * BK <= g.K; k0 += BK) {
        load(k0 + BK);
        mfma_k(buf, 0);
        mfma_k(buf, 1);
        mfma_k(buf, 2);
        stash(buf ^ 1, k0 + BK);
        mfma_k(buf, 3);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // global load
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);   // LDS write
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
        }
        __syncthreads();
        buf ^= 1;
    }
    // the last one or two steps (the next one partial, or none)
    for (; k0 < g.K; k0 += BK) {
        const bool more = k0 + BK < g.K;
        if (more) load_any(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) mfma_k(buf, kk);
        if (more) stash(buf ^ 1, k0 + BK);
        __syncthreads();
        buf ^= 1;
    }

    // epilogue: acc[tn][tm][j] = C[m = m0 + wm + 16 tm + li][n = n0 + wn + 16 tn + mfma_row(lk, j)]
    double s_r = 0.0, s_f = 0.0;
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
        for (int tm = 0; tm < 4; ++tm)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = m0 + wm + 16 * tm + li;
                const int n = n0 + wn + 16 * tn + mfma_row<double>(lk, j);
                if (m >= g.M || n >= g.N) continue;
                const size_t off = (size_t)batch * g.strideC + (size_t)m + (size_t)n * g.ldc;
                const double v = acc[tn][tm][j];
                if (EPI == EPI_STORE_F32) {
                    static_cast<float*>(g.C)[off] = static_cast<float>(v);
                } else if (EPI == EPI_STORE_F64) {
                    static_cast<double*>(g.C)[off] = v;
                } else if (EPI == EPI_ADD_F64) {
                    static_cast<double*>(g.C)[off] += g.alpha * v;
                } else {   // EPI_RESID: C = F - A B, sums of squares of C and F
                    const size_t foff = (size_t)batch * g.strideF + (size_t)m + (size_t)n * g.ldc;
                    const double f = static_cast<const double*>(g.F)[foff];
                    const double r = f - v;
                    static_cast<double*>(g.C)[off] = r;
                    s_r += r * r;
                    s_f += f * f;
                }
            }
    if (EPI == EPI_RESID) {
        const double tr = block_sum(s_r, red);
        const double tf = block_sum(s_f, red);
        if (tid == 0) {
            // (the partials of a RHS are summed in full, in any block order)
            const size_t idx = (size_t)batch * per + tile;
            g.partial[2 * idx] = tr;
            g.partial[2 * idx + 1] = tf;
        }
    }
}

template <typename TA, int EPI>
static hipError_t launch_gemm_wide(const GemmArgs& g, hipStream_t st) {
    // the loads of a K step sit at 32-bit byte offsets from its first column
    // of A and row of B
    if (((uint64_t)BK * g.lda + g.M) * sizeof(TA) >= (1ull << 32) ||
        ((uint64_t)BK * g.ldb + g.N) * sizeof(double) >= (1ull << 32))
        return hipErrorInvalidValue;
    const unsigned total = wide_tiles(g.M, g.N) * (unsigned)g.batch;
    const unsigned grid = NXCD * ((total + NXCD - 1) / NXCD);
    hipLaunchKernelGGL((gemm_wide_kernel<TA, EPI>), dim3(grid), dim3(256), 0, st, g);
    return hipGetLastError();
}

template <typename TA, typename TC, int EPI, int TM, bool NFAST>
static hipError_t launch_gemm_v(const GemmArgs& g, hipStream_t st) {
    const unsigned mt = (g.M + 32 * TM - 1) / (32 * TM), nt = (g.N + BN - 1) / BN;
    dim3 grid(NFAST ? nt : mt, NFAST ? mt : nt, g.batch);
    hipLaunchKernelGGL((gemm_kernel<TA, TC, EPI, TM, NFAST>), grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

// variant by the tile height (bm = 64 or 128) and the grid order
template <typename TA, typename TC, int EPI>
static hipError_t launch_gemm_t(const GemmArgs& g0, hipStream_t st) {
    GemmArgs g = g0;
    g.gate = launch_gate();
    if constexpr (sizeof(TC) == 8) {
        // the residual always takes the 128 x 128 tile (its partials are
        // counted for it); the others where chosen (bm = 0)
        if (EPI == EPI_RESID || g.bm == 0) return launch_gemm_wide<TA, EPI>(g, st);
    }
    if (g.bm == 0) g.bm = 64;
    if (g.bm == 128)
        return g.nfast ? launch_gemm_v<TA, TC, EPI, 4, true>(g, st) : launch_gemm_v<TA, TC, EPI, 4, false>(g, st);
    return g.nfast ? launch_gemm_v<TA, TC, EPI, 2, true>(g, st) : launch_gemm_v<TA, TC, EPI, 2, false>(g, st);
}

hipError_t launch_gemm(GemmKind kind, const GemmArgs& g, hipStream_t st) {
    switch (kind) {
        case GEMM_D_D_STORE_D: return launch_gemm_t<double, double, EPI_STORE_F64>(g, st);
        case GEMM_D_D_STORE_F: return launch_gemm_t<double, double, EPI_STORE_F32>(g, st);
        case GEMM_D_F_STORE_F: return launch_gemm_t<double, float, EPI_STORE_F32>(g, st);
        case GEMM_F_F_STORE_F: return launch_gemm_t<float, float, EPI_STORE_F32>(g, st);
        case GEMM_F_F_ADD_D: return launch_gemm_t<float, float, EPI_ADD_F64>(g, st);
        case GEMM_D_D_ADD_D: return launch_gemm_t<double, double, EPI_ADD_F64>(g, st);
        case GEMM_D_D_RESID: return launch_gemm_t<double, double, EPI_RESID>(g, st);
        case GEMM_F_D_STORE_F: return launch_gemm_t<float, double, EPI_STORE_F32>(g, st);
        case GEMM_F_D_ADD_D: return launch_gemm_t<float, double, EPI_ADD_F64>(g, st);
    }
    return hipErrorInvalidValue;
}

size_t gemm_resid_partials(int M, int N, int batch) {
    return (size_t)wide_tiles(M, N) * batch;
}

// ---------------------------------------------------------------------------
// Spatial operator for the residual: P[:, j] = M_x U[:, j] and
// P[:, N_t + j] = A_x U[:, j] (CSR, FP64), for every RHS.
// ---------------------------------------------------------------------------
// P = [M_x U | A_x U] per right-hand side.  A thread takes one row and KC
// time columns: the row's CSR entries (up to NNZ of them in registers, a
// longer row loops over the rest) are read once and serve both products;
// for a fixed time column the lanes of a wave read consecutive rows of U.
// KC = 64: the CSR arrays (6.8 MB at M_x = 48641) are read once per 64
// time columns of a right-hand side (16 measured 8.6 ms against 7.7 ms at
// the L-shape N_t = 1024 shape, 16 right-hand sides).
constexpr int SPATIAL_KC = 64;

template <int NNZ>
__global__ void __launch_bounds__(256) spatial_apply_kernel(int Mx, int Nt, int nrhs, const int* __restrict__ rowptr,
                                                            const int* __restrict__ col,
                                                            const double* __restrict__ valM,
                                                            const double* __restrict__ valA,
                                                            const double* __restrict__ U, double* __restrict__ P,
                                                            const int* __restrict__ gate) {
    if (gate && *gate) return;
    // workgroup w (a 1D grid of 8 per_xcd) runs on XCD w mod 8: each XCD
    // takes a contiguous range of the (row block, time chunk, RHS) blocks,
    // row blocks fastest, so that the neighbouring row blocks whose rows a
    // stencil reads share its L2
    const unsigned gx = (Mx + 255) / 256, gy = (Nt + SPATIAL_KC - 1) / SPATIAL_KC;
    const unsigned total = gx * gy * (unsigned)nrhs;
    const unsigned per_xcd = gridDim.x / 8;
    const unsigned logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (logical >= total) return;
    const int i = (int)(logical % gx) * blockDim.x + threadIdx.x;
    const int k0 = (int)((logical / gx) % gy) * SPATIAL_KC;
    const int batch = (int)(logical / (gx * gy));
    if (i >= Mx) return;
    const int e0 = rowptr[i], n = rowptr[i + 1] - e0;
    int c[NNZ];
    double vm[NNZ], va[NNZ];
#pragma unroll
    for (int e = 0; e < NNZ; ++e) {
        const bool on = e < n;
        c[e] = on ? col[e0 + e] : i;
        vm[e] = on ? valM[e0 + e] : 0.0;
        va[e] = on ? valA[e0 + e] : 0.0;
    }
    const double* u = U + (size_t)batch * Mx * Nt;
    double* pb = P + (size_t)batch * Mx * 2 * Nt;
    const int k1 = min(k0 + SPATIAL_KC, Nt);
    for (int k = k0; k < k1; ++k) {
        const double* uk = u + (size_t)k * Mx;
        double sm = 0.0, sa = 0.0;
#pragma unroll
        for (int e = 0; e < NNZ; ++e) {
            const double x = uk[c[e]];
            sm += vm[e] * x;
            sa += va[e] * x;
        }
        for (int e = NNZ; e < n; ++e) {
            const double x = uk[col[e0 + e]];
            sm += valM[e0 + e] * x;
            sa += valA[e0 + e] * x;
        }
        pb[(size_t)k * Mx + i] = sm;
        pb[(size_t)(Nt + k) * Mx + i] = sa;
    }
}

hipError_t launch_spatial_apply(int Mx, int Nt, int nrhs, const int* rowptr, const int* col, const double* valM,
                                const double* valA, const double* U, double* P, hipStream_t st) {
    // (8 per_xcd workgroups: those past the blocks return)
    const unsigned gx = (Mx + 255) / 256, gy = (Nt + SPATIAL_KC - 1) / SPATIAL_KC;
    const unsigned total = gx * gy * (unsigned)nrhs;
    hipLaunchKernelGGL(spatial_apply_kernel<8>, dim3(8 * ((total + 7) / 8)), dim3(256), 0, st, Mx, Nt, nrhs, rowptr,
                       col, valM, valA, U, P, launch_gate());
    return hipGetLastError();
}

// Residual of the spatial systems of step 3 of Algorithm FD, for the
// refinement of the spatial solves inside an application: R = G - (M_x +
// lambda_k A_x) Z for every system k and right-hand side, the CSR products and
// the subtraction in FP64 from FP64 G and Z, R rounded to the working
// precision (the band factors solve it).  Layout of G, Z, R per RHS:
// column-major M_x x 2 n_sys, real parts of system k in column k, imaginary
// parts in column n_sys + k.  A thread takes one row and RESID_KS systems:
// the row's CSR entries (up to NNZ in registers) are read once for all of
// them (one system per thread read them once per system: 8 thousand times
// at the L-shape N_t = 1024 shape with 16 right-hand sides).  grid.y runs
// over the groups of systems, grid.z over the right-hand sides.
constexpr int RESID_KS = 32;

template <typename TR, int NNZ>
__global__ void __launch_bounds__(256) spatial_resid_kernel(int Mx, int nsys, const int* __restrict__ rowptr,
                                                            const int* __restrict__ col,
                                                            const double* __restrict__ valM,
                                                            const double* __restrict__ valA,
                                                            const double* __restrict__ lam,
                                                            const double* __restrict__ G,
                                                            const double* __restrict__ Z, TR* __restrict__ R,
                                                            const int* __restrict__ gate) {
    if (gate && *gate) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Mx) return;
    const int e0 = rowptr[i], n = rowptr[i + 1] - e0;
    int c[NNZ];
    double vm[NNZ], va[NNZ];
#pragma unroll
    for (int e = 0; e < NNZ; ++e) {
        const bool on = e < n;
        c[e] = on ? col[e0 + e] : i;
        vm[e] = on ? valM[e0 + e] : 0.0;
        va[e] = on ? valA[e0 + e] : 0.0;
    }
    const size_t rhs = (size_t)blockIdx.z * 2 * nsys * Mx;
    const int k0 = blockIdx.y * RESID_KS, k1 = min(k0 + RESID_KS, nsys);
    for (int k = k0; k < k1; ++k) {
        const size_t cr = rhs + (size_t)k * Mx, ci = rhs + (size_t)(nsys + k) * Mx;
        const double lr = lam[2 * k], li = lam[2 * k + 1];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int e = 0; e < NNZ; ++e) {
            const double mr = vm[e] + lr * va[e], mi = li * va[e];
            const double xr = Z[cr + c[e]], xi = Z[ci + c[e]];
            sr += mr * xr - mi * xi;
            si += mr * xi + mi * xr;
        }
        for (int e = NNZ; e < n; ++e) {
            const int j = col[e0 + e];
            const double mr = valM[e0 + e] + lr * valA[e0 + e], mi = li * valA[e0 + e];
            const double xr = Z[cr + j], xi = Z[ci + j];
            sr += mr * xr - mi * xi;
            si += mr * xi + mi * xr;
        }
        R[cr + i] = static_cast<TR>(G[cr + i] - sr);
        R[ci + i] = static_cast<TR>(G[ci + i] - si);
    }
}

template <typename TR>
hipError_t launch_spatial_resid(int Mx, int nsys, int nrhs, const int* rowptr, const int* col, const double* valM,
                                const double* valA, const double* lam, const double* G, const double* Z, void* R,
                                hipStream_t st) {
    dim3 grid((Mx + 255) / 256, (nsys + RESID_KS - 1) / RESID_KS, nrhs);
    hipLaunchKernelGGL((spatial_resid_kernel<TR, 8>), grid, dim3(256), 0, st, Mx, nsys, rowptr, col, valM, valA,
                       lam, G, Z, static_cast<TR*>(R), launch_gate());
    return hipGetLastError();
}

// y = x (ACC = false) or y += x (ACC = true), elementwise, x converted to the
// type of y; four elements per thread and step (n need not be a multiple)
template <typename TY, typename TX, bool ACC>
__global__ void __launch_bounds__(256) convert_kernel(TY* __restrict__ y, const TX* __restrict__ x, size_t n,
                                                      const int* __restrict__ gate) {
    if (gate && *gate) return;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += 4 * stride) {
        TX v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = i + u * stride < n ? x[i + u * stride] : TX(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * stride < n) y[i + u * stride] = ACC ? y[i + u * stride] + static_cast<TY>(v[u]) : static_cast<TY>(v[u]);
    }
}

template <typename TY, typename TX, bool ACC>
hipError_t launch_convert(void* y, const void* x, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 1023) / 1024, 32768);
    hipLaunchKernelGGL((convert_kernel<TY, TX, ACC>), dim3((unsigned)blocks), dim3(256), 0, st, static_cast<TY*>(y),
                       static_cast<const TX*>(x), n, launch_gate());
    return hipGetLastError();
}

template hipError_t launch_spatial_resid<float>(int, int, int, const int*, const int*, const double*, const double*,
                                                const double*, const double*, const double*, void*, hipStream_t);
template hipError_t launch_spatial_resid<double>(int, int, int, const int*, const int*, const double*,
                                                 const double*, const double*, const double*, const double*, void*,
                                                 hipStream_t);
template hipError_t launch_convert<float, double, false>(void*, const void*, size_t, hipStream_t);
template hipError_t launch_convert<double, float, false>(void*, const void*, size_t, hipStream_t);
template hipError_t launch_convert<double, float, true>(void*, const void*, size_t, hipStream_t);
template hipError_t launch_convert<double, double, true>(void*, const void*, size_t, hipStream_t);

// Bartels-Stewart with the complex Schur form (Alg. BSc, Sec. 4.3), step 3:
// once z_k is solved, the right-hand sides of the systems still to come take
// its coupling, g_i -= S[i][k] A_x z_k for i < k.  A thread takes one row:
// v = (A_x z_k)[row] (complex, from the CSR row), then the k updates of that
// row (for a fixed i the lanes of a wave touch consecutive rows).  G per RHS:
// column-major Mx x 2 nsys, real parts in column i, imaginary in nsys + i.
__global__ void __launch_bounds__(256) bs_update_kernel(int Mx, int nsys, int k, const int* __restrict__ rowptr,
                                                        const int* __restrict__ col,
                                                        const double* __restrict__ valA,
                                                        const double* __restrict__ S, double* __restrict__ G) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Mx) return;
    double* Gb = G + (size_t)blockIdx.y * 2 * nsys * Mx;
    const double* zr = Gb + (size_t)k * Mx;
    const double* zi = Gb + (size_t)(nsys + k) * Mx;
    double vr = 0.0, vi = 0.0;
    for (int e = rowptr[m]; e < rowptr[m + 1]; ++e) {
        const double a = valA[e];
        vr += a * zr[col[e]];
        vi += a * zi[col[e]];
    }
    for (int i = 0; i < k; ++i) {
        const double sr = S[2 * ((size_t)i * nsys + k)], si = S[2 * ((size_t)i * nsys + k) + 1];
        Gb[(size_t)i * Mx + m] -= sr * vr - si * vi;
        Gb[(size_t)(nsys + i) * Mx + m] -= sr * vi + si * vr;
    }
}

hipError_t launch_bs_update(int Mx, int nsys, int nrhs, int k, const int* rowptr, const int* col,
                            const double* valA, const double* S, double* G, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    dim3 grid((Mx + 255) / 256, nrhs);
    hipLaunchKernelGGL(bs_update_kernel, grid, dim3(256), 0, st, Mx, nsys, k, rowptr, col, valA, S, G);
    return hipGetLastError();
}

// fixed-order reduction of the residual GEMM partial sums: norms[2 r] =
// ||R_r||^2, norms[2 r + 1] = ||F_r||^2
__global__ void reduce_partials_kernel(const double* __restrict__ partial, size_t blocks, double* __restrict__ norms,
                                       const int* __restrict__ gate) {
    if (gate && *gate) return;
    __shared__ double red[8];
    const int batch = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (size_t q = threadIdx.x; q < blocks; q += blockDim.x) {
        a += partial[2 * ((size_t)batch * blocks + q)];
        b += partial[2 * ((size_t)batch * blocks + q) + 1];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        norms[2 * batch] = a;
        norms[2 * batch + 1] = b;
    }
}

hipError_t launch_reduce_partials(const double* partial, size_t blocks, int nrhs, double* norms, hipStream_t st) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(nrhs), dim3(256), 0, st, partial, blocks, norms, launch_gate());
    return hipGetLastError();
}

__global__ void fill_zero_kernel(double* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_fill_zero(double* p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gate of a refinement round and the device-side convergence check
// ---------------------------------------------------------------------------
static thread_local const int* g_launch_gate = nullptr;

void set_launch_gate(const int* gate) { g_launch_gate = gate; }
const int* launch_gate() { return g_launch_gate; }

__global__ void refine_check_kernel(const double* __restrict__ norms, int nrhs, double rtol,
                                    const int* __restrict__ pivot_flag, int max_apps, int* __restrict__ ctl,
                                    double* __restrict__ hist) {
    if (ctl[0]) return;
    if (threadIdx.x != 0) return;
    double rel = 0.0;
    bool finite = true;
    for (int q = 0; q < nrhs; ++q) {
        const double rr = norms[2 * q], ff = norms[2 * q + 1];
        if (!isfinite(rr)) finite = false;
        rel = fmax(rel, ff > 0.0 ? sqrt(rr / ff) : sqrt(rr));
    }
    const int a = ctl[1];
    hist[a] = rel;
    ctl[1] = a + 1;
    int status = 0;
    if (pivot_flag && *pivot_flag) status = 2;
    else if (!finite) status = 4;
    else if (rel <= rtol) status = 1;
    else if (a + 1 >= max_apps) status = 3;
    if (status) {
        ctl[2] = status;
        ctl[0] = 1;
    }
}

hipError_t launch_refine_check(const double* norms, int nrhs, double rtol, const int* pivot_flag, int max_apps,
                               int* ctl, double* hist, hipStream_t st) {
    hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(64), 0, st, norms, nrhs, rtol, pivot_flag, max_apps, ctl,
                       hist);
    return hipGetLastError();
}

__global__ void reset_ints_kernel(int* __restrict__ p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t launch_reset_ints(int* p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_ints_kernel, dim3(1), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace stfd
