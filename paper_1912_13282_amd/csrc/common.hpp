// Shared host/device helpers of the RBF-FD library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/rbffd.h"

struct rbf_ctx {
    int device;
    hipStream_t stream;
    // plan of each size class of the batched form (chunk, waves per CU), see
    // batched.hip; plan_valid == 0: the defaults
    int plan_valid;
    int plan_chunk[RBF_BATCHED_CLASSES];
    int plan_waves_per_cu[RBF_BATCHED_CLASSES];
    // surrogate network parameters (device, owned), see mlp.hip
    void* mlp_params;
    size_t mlp_bytes;
};

// resolves the device address of the no-allocation selection scratch (knn.hip)
rbf_status rbf_select_scratch_init(int device);

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

// The operators selected in op_mask (the RBF_OP_* bits, LAP .. DZZ) fill the
// right-hand-side slots 0..R-1 in bit order; *opc receives one 4-bit code per
// slot (the operator's bit index).  Returns R, or -1 for an empty mask, an
// unknown bit, more than four operators, or an operator along z in 2D.
inline int op_slots(unsigned op_mask, int d, unsigned* opc) {
    const unsigned zops = RBF_OP_DZ | RBF_OP_DXZ | RBF_OP_DYZ | RBF_OP_DZZ;
    if (op_mask == 0 || (op_mask & ~0x3FFu) || (d == 2 && (op_mask & zops))) return -1;
    unsigned c = 0;
    int R = 0;
    for (int b = 0; b < 10; ++b) {
        if (!(op_mask & (1u << b))) continue;
        if (R == 4) return -1;
        c |= (unsigned)b << (4 * R);
        ++R;
    }
    *opc = c;
    return R;
}

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

// DPP move of a double (each 32-bit half with the same control); rows outside
// row_mask keep their own value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Wave-wide maximum through DPP (quad xor 1, xor 2, half-row mirror, row mirror,
// row broadcast 15 / 31); the total ends in lane 63 and is returned uniformly.
__device__ __forceinline__ double wave_max_dpp_d(double v) {
    v = fmax(v, dpp_d<0xB1, 0xF>(v));
    v = fmax(v, dpp_d<0x4E, 0xF>(v));
    v = fmax(v, dpp_d<0x141, 0xF>(v));
    v = fmax(v, dpp_d<0x140, 0xF>(v));
    v = fmax(v, dpp_d<0x142, 0xA>(v));
    v = fmax(v, dpp_d<0x143, 0xC>(v));
    return readlane_d(v, 63);
}
__device__ __forceinline__ float wave_max_dpp_f(float v) {
    v = fmaxf(v, dpp_f<0xB1, 0xF>(v));
    v = fmaxf(v, dpp_f<0x4E, 0xF>(v));
    v = fmaxf(v, dpp_f<0x141, 0xF>(v));
    v = fmaxf(v, dpp_f<0x140, 0xF>(v));
    v = fmaxf(v, dpp_f<0x142, 0xA>(v));
    v = fmaxf(v, dpp_f<0x143, 0xC>(v));
    return readlane_f(v, 63);
}
// Wave-wide maximum of an int through DPP; INT_MIN fills the lanes a stage does
// not reach, so every stage folds into one v_max_i32 with a DPP operand.  Lane 63
// ends with the total, returned uniformly.  (Non-negative floats compare like
// their bit patterns, which makes this the pivot search on magnitudes.)
__device__ __forceinline__ int wave_max_dpp_i(int v) {
    constexpr int LO = -2147483647 - 1;
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0xB1, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x4E, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x141, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x140, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x142, 0xA, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// Wave-wide sum through DPP in a fixed order (deterministic); uniform result.
__device__ __forceinline__ double wave_sum_dpp_d(double v) {
    v += dpp_d<0xB1, 0xF>(v);
    v += dpp_d<0x4E, 0xF>(v);
    v += dpp_d<0x141, 0xF>(v);
    v += dpp_d<0x140, 0xF>(v);
    // rows now hold their row sums; combine the four rows in a fixed order
    double r0 = readlane_d(v, 0), r1 = readlane_d(v, 16), r2 = readlane_d(v, 32), r3 = readlane_d(v, 48);
    return (r0 + r1) + (r2 + r3);
}

// LDS visibility of this wave's own stores to its other lanes (LDS operations of
// one wavefront execute in order; the fences stop the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of lane ^ M (M a compile-time mask of the low lane bits).  Masks inside
// a row of 16 lanes are DPP moves: 1, 2, 3 quad permutations, 7 the half-row
// mirror, 15 the row mirror, 8 a row rotation, 4 = 3 then 7; the others cross
// rows and go through the LDS permute.  The partner lane must be active.
template <int M>
__device__ __forceinline__ unsigned lane_xor_u32(unsigned v) {
    const int x = (int)v;
    if constexpr (M == 1) return (unsigned)__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false);
    else if constexpr (M == 2) return (unsigned)__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false);
    else if constexpr (M == 3) return (unsigned)__builtin_amdgcn_update_dpp(x, x, 0x1B, 0xF, 0xF, false);
    else if constexpr (M == 4) {
        const int a = __builtin_amdgcn_update_dpp(x, x, 0x1B, 0xF, 0xF, false);
        return (unsigned)__builtin_amdgcn_update_dpp(a, a, 0x141, 0xF, 0xF, false);
    } else if constexpr (M == 7) return (unsigned)__builtin_amdgcn_update_dpp(x, x, 0x141, 0xF, 0xF, false);
    else if constexpr (M == 8) return (unsigned)__builtin_amdgcn_update_dpp(x, x, 0x128, 0xF, 0xF, false);
    else if constexpr (M == 15) return (unsigned)__builtin_amdgcn_update_dpp(x, x, 0x140, 0xF, 0xF, false);
    else return (unsigned)__shfl_xor(x, M);
}

// lanes where pred holds (wave64), without materialising pred in a register
__device__ __forceinline__ uint64_t ballot64(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

// first set lane of a wave-uniform 64-bit mask (mask != 0)
__device__ __forceinline__ int first_lane(uint64_t m) { return __builtin_ctzll(m); }
