// Shared host/device helpers of the RBF-FD library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rbffd.h"

struct rbf_ctx {
    int device;
    hipStream_t stream;
    // autotuned plan of the batched form (size-class packing), see batched.hip
    int plan_valid;
    int plan_chunk;
    int plan_waves_per_cu;
    // surrogate network parameters (device, owned), see mlp.hip
    void* mlp_params;
    size_t mlp_bytes;
};

#define RBF_HIP_CHECK(expr)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return RBF_EHIP;                \
    } while (0)

#define RBF_LAUNCH_CHECK()                                    \
    do {                                                      \
        hipError_t e_ = hipGetLastError();                    \
        if (e_ != hipSuccess) return RBF_EHIP;                \
    } while (0)

static inline size_t rbf_align(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int WAVE = 64;

__host__ __device__ constexpr int binom(int n, int k) {
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// number of monomials of total degree <= P in D variables
__host__ __device__ constexpr int n_mono(int D, int P) { return binom(P + D, D); }

// ---------------------------------------------------------------- device side
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ double readlane_d(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int lane);
template <>
__device__ __forceinline__ double readlane_t<double>(double v, int lane) { return readlane_d(v, lane); }
template <>
__device__ __forceinline__ float readlane_t<float>(float v, int lane) { return readlane_f(v, lane); }

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// first set lane of a wave-uniform 64-bit mask (mask != 0)
__device__ __forceinline__ int first_lane(uint64_t m) { return __builtin_ctzll(m); }
