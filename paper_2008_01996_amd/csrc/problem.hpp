// The problem handle behind the C-ABI (internal to the library): setup
// data, device buffers of the transforms and band factors, work buffers and
// the per-stage event timing.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "host_internal.hpp"

struct stfd_problem {
    const stfd_space* space = nullptr;
    stfd_opts opts{};
    int Nt = 0, Mx = 0, b = 0, bp = 0, nsys = 0, npair = 0, nreal = 0;
    int method = STFD_METHOD_FD;
    stfd_setup_report rep{};
    std::vector<double> lam_sys;   // 2 nsys (re, im)
    bool factored = false;
    // device data
    int* d_rowptr = nullptr;
    int* d_col = nullptr;
    int* d_reach = nullptr;     // envelope of the factor per 16-column block (space's block_reach)
    double* d_valM = nullptr;
    double* d_valA = nullptr;
    double* d_lam = nullptr;
    double* d_W1 = nullptr;     // Nt x 2Nt  FP64: [Re | Im] of A_t^-1 conj(U_t) Sigma^-1
    float* d_W1f = nullptr;     // FP32 copy (first forward GEMM in FP32)
    void* d_W2 = nullptr;       // 2Nt x 2nsys  [[Re, Im], [-Im, Re]] of V_t^T[:, sys], working precision
    void* d_Xb = nullptr;       // 2nsys x Nt   [Re; -Im] of c_k x_k^T, working precision
    double* d_W2d = nullptr;    // FP64 copies for FP64 transforms in the FP32 form
    double* d_Wfwd = nullptr;   // Nt x 2nsys FP64: W1 W2, the forward transform as one product
    bool fwd_merged = false;    // forward transform: one FP64 GEMM with d_Wfwd (else W1, then W2)
    double* d_Xbd = nullptr;
    double* d_Bres = nullptr;   // 2Nt x Nt     [A_t^T; M_t^T]
    double* d_S = nullptr;      // Alg. BSc: Nt x Nt upper-triangular Schur factor, complex interleaved
    void* d_LB = nullptr;       // band factors
    void* d_LI = nullptr;       // inverses of their 16 x 16 diagonal blocks (tile sweeps)
    int tile_min_rhs = 0;       // tile sweeps from this many right-hand sides on (0: never)
    int gemm_bm[2] = {64, 128}; // GEMM tile rows on FP32 / FP64 matrix cores
    int gemm_bn64 = 128;        // GEMM tile columns on FP64 matrix cores (128: the 128 x 128 tile)
    int gemm_nfast = 0;         // GEMM grid order
    int factor_kernel = 0;      // band factor kernel (stfd_tuning.factor_kernel)
    int factor_pack_real = 1;   // real systems two to a workgroup (stfd_tuning.factor_pack_real)
    int sweep_pack_real = 1;    // the same for the tile sweeps (stfd_tuning.sweep_pack_real)
    int* d_flag = nullptr;
    // work buffers, sized for nrhs_cap right-hand sides
    int nrhs_cap = 0;
    void* d_T1 = nullptr;       // Mx x 2Nt per RHS (FP32 or FP64)
    void* d_G = nullptr;        // Mx x 2nsys per RHS
    double* d_Gs = nullptr;     // Mx x 2nsys per RHS, FP64: G kept for the inner refinement
    double* d_Z64 = nullptr;    // Mx x 2nsys per RHS, FP64: the spatial solutions summed over the inner refinement
    double* d_P = nullptr;      // Mx x 2Nt per RHS
    double* d_R = nullptr;      // Mx x Nt per RHS
    double* d_part = nullptr;
    double* d_norms = nullptr;
    // refinement control on the device (captured rounds): ctl = {done,
    // applications, status, spare}, hist = residual after each application;
    // pinned host mirrors of both
    int* d_ctl = nullptr;
    double* d_hist = nullptr;
    int* h_ctl = nullptr;
    double* h_hist = nullptr;
    // captured refinement rounds (first: applied to F; next: to the
    // residual), valid for (g_F, g_U, g_nrhs)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t g_first = nullptr, g_next = nullptr;
    const double* g_F = nullptr;
    double* g_U = nullptr;
    int g_nrhs = 0;
    int last_apps = 0;          // applications the last solve needed (rounds launched ahead)
    // per-stage event timing
    struct ProfRec {
        int stage;
        hipEvent_t a, b;
    };
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;    // all events ever created
    size_t ev_used = 0;                 // events handed out since the last drain
    std::vector<ProfRec> prof_recs;
    double prof_ms[STFD_NSTAGE] = {};
    long long prof_cnt[STFD_NSTAGE] = {};
};
