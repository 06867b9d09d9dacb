// The K_h residual of the refinement without any device allocation: the
// work memory of stfd_kh_residual (the spatial products [M_x U | A_x U] and
// the per-workgroup partial norms) comes from a fixed array in device memory
// instead of the problem's work buffers.
//
// The array is file-scope device memory; each GPU the library runs on holds
// its own copy until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in symbol): on the first
// call on a device, with that device current, its device address is looked
// up once and kept per device, and every launch uses that address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host_internal.hpp"
#include "kernels.hpp"
#include "problem.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(128) << 20;      // 128 MiB per device
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mutex;
void* g_scratch[MAX_DEVICES] = {};

// device address of this device's scratch array (looked up once per device)
int scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return stfd::fail(STFD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return stfd::fail(STFD_EINVAL, "kh_residual_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return stfd::fail(STFD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return STFD_OK;
}

}  // namespace

extern "C" size_t stfd_kh_residual_noalloc_max_bytes(void) { return SCRATCH_BYTES; }

extern "C" int stfd_kh_residual_noalloc(stfd_problem* p, int nrhs, const double* F_dev, const double* U_dev,
                                        double* R_dev, double* norms_dev, void* hip_stream) {
    if (!p || nrhs < 1 || !F_dev || !U_dev || !R_dev)
        return stfd::fail(STFD_EINVAL, "kh_residual_noalloc: bad arguments");
    const size_t Mx = p->Mx, Nt = p->Nt;
    const size_t parts = stfd::gemm_resid_partials(p->Mx, p->Nt, nrhs);
    const size_t need = (Mx * 2 * Nt * nrhs + 2 * parts) * sizeof(double);
    if (need > SCRATCH_BYTES)
        return stfd::fail(STFD_EINVAL, "kh_residual_noalloc: needs " + std::to_string(need) +
                                           " bytes of work memory, more than its fixed " +
                                           std::to_string(SCRATCH_BYTES));
    void* base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double* P = static_cast<double*>(base);                 // [M_x U | A_x U] per RHS
    double* part = P + Mx * 2 * Nt * nrhs;                  // partial sums of squares
    hipError_t e = stfd::launch_spatial_apply(p->Mx, p->Nt, nrhs, p->d_rowptr, p->d_col, p->d_valM, p->d_valA, U_dev,
                                              P, st);
    if (e != hipSuccess) return stfd::fail(STFD_EHIP, std::string("spatial operator: ") + hipGetErrorString(e));
    stfd::GemmArgs g{};
    g.A = P; g.B = p->d_Bres; g.C = R_dev; g.F = F_dev; g.partial = part;
    g.M = p->Mx; g.N = p->Nt; g.K = 2 * p->Nt;
    g.lda = Mx; g.ldb = Nt; g.ldc = Mx;
    g.strideA = (long long)(Mx * 2 * Nt); g.strideC = (long long)(Mx * Nt); g.strideF = (long long)(Mx * Nt);
    g.batch = nrhs;
    e = stfd::launch_gemm(stfd::GEMM_D_D_RESID, g, st);
    if (e != hipSuccess) return stfd::fail(STFD_EHIP, std::string("residual: ") + hipGetErrorString(e));
    if (norms_dev) {
        e = stfd::launch_reduce_partials(part, stfd::gemm_resid_partials(p->Mx, p->Nt, 1), nrhs, norms_dev, st);
        if (e != hipSuccess) return stfd::fail(STFD_EHIP, std::string("residual norms: ") + hipGetErrorString(e));
    }
    stfd::clear_error();
    return STFD_OK;
}
