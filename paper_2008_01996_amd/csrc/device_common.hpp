// Device helpers for gfx950 (CDNA4): complex arithmetic on real pairs and the
// 16x16x4 matrix-core (MFMA) instructions in FP32 and FP64.
//
// MFMA 16x16x4 operand layout (wave of 64 lanes, one 16x16 output block):
//   A operand: lane l holds A[m = l % 16][k = l / 16]
//   B operand: lane l holds B[k = l / 16][n = l % 16]
//   D output : lane l, register j holds D[m][n = l % 16] with
//              m = 4 * (l / 16) + j   for the FP32 instruction,
//              m = (l / 16) + 4 * j   for the FP64 instruction
//   (mfma_row<T> below; both measured on gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace stfd {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename T>
__device__ __forceinline__ cplx<T> cinv(cplx<T> a) {
    // 1/a with a scaling that avoids overflow in |a|^2
    const T s = fabs(a.re) > fabs(a.im) ? fabs(a.re) : fabs(a.im);
    const T ar = a.re / s, ai = a.im / s;
    const T d = (ar * ar + ai * ai) * s;
    return {ar / d, -ai / d};
}

// 1/a from the hardware reciprocal (1 ulp) in FP32; the scaled division in FP64
template <typename T>
__device__ __forceinline__ cplx<T> cinv_fast(cplx<T> a) {
    if constexpr (sizeof(T) == 4) {
        const float s = __builtin_amdgcn_rcpf(a.re * a.re + a.im * a.im);
        return {a.re * s, -a.im * s};
    } else {
        return cinv(a);
    }
}

template <typename T>
struct vec4;
template <>
struct vec4<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct vec4<double> {
    typedef double type __attribute__((ext_vector_type(4)));
};

template <typename T>
__device__ __forceinline__ typename vec4<T>::type mfma16x16x4(T a, T b, typename vec4<T>::type c);

template <>
__device__ __forceinline__ vec4<float>::type mfma16x16x4<float>(float a, float b, vec4<float>::type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <>
__device__ __forceinline__ vec4<double>::type mfma16x16x4<double>(double a, double b, vec4<double>::type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// output row m of register j in lane group g = l / 16
template <typename T>
__device__ __forceinline__ int mfma_row(int g, int j);
template <>
__device__ __forceinline__ int mfma_row<float>(int g, int j) { return 4 * g + j; }
template <>
__device__ __forceinline__ int mfma_row<double>(int g, int j) { return g + 4 * j; }

template <typename T>
__device__ __forceinline__ typename vec4<T>::type zero4() {
    typename vec4<T>::type z;
    z[0] = z[1] = z[2] = z[3] = T(0);
    return z;
}

// value of lane l (uniform) broadcast to the whole wave through a scalar
// register (v_readlane), without an LDS round trip
// x through an opaque register move: what the compiler computes from the
// result cannot be hoisted out of the loop the move sits in
__device__ __forceinline__ int opaque_int(int x) {
    int r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
__device__ __forceinline__ float lane_bcast(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_bcast(double v, int l) {
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x & 0xffffffffull), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// lane k of this lane's group of G consecutive lanes (64 / G groups per wave)
template <int G, typename T>
__device__ __forceinline__ T group_bcast(T v, int k, int grp) {
    T r = lane_bcast(v, k);
#pragma unroll
    for (int g = 1; g < 64 / G; ++g) {
        const T o = lane_bcast(v, g * G + k);
        if (grp == g) r = o;
    }
    return r;
}

// acc += a * b for complex values given as real pairs, in fused multiply-adds
template <typename T>
__device__ __forceinline__ void cmac(T& accr, T& acci, T ar, T ai, T br, T bi) {
    accr = fma(ar, br, accr);
    accr = fma(-ai, bi, accr);
    acci = fma(ar, bi, acci);
    acci = fma(ai, br, acci);
}

// Orders one wave's LDS accesses across its lanes for the compiler (values a
// lane stores are read by other lanes of the same wave afterwards).  The
// hardware runs the LDS instructions of a wave in issue order, so no wait or
// workgroup barrier is needed.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// block-wide sum of one double per thread (blockDim.x a multiple of 64, <= 1024)
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += scratch[w];
    }
    __syncthreads();
    return s;
}

}  // namespace stfd
