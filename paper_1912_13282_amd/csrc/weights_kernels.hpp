// Kernels of the RBF-FD weight computation and their per-size-class registry.
// Every (dimension, degree, system-size class) is instantiated in a translation
// unit of its own (wcls_*.hip) so that the heavily unrolled classes compile in
// parallel; each registers its launcher at load time.
#pragma once

#include "weights_f64.hpp"
#include "weights_ir.hpp"
#include "weights_gj.hpp"
#include "weights_irgj.hpp"

namespace rbf {

template <int MAXM>
constexpr int waves_per_block() { return MAXM <= 64 ? 4 : 1; }

// Plain FP64 solve.  With fallback_pass set, only stencils whose status is
// FALLBACK (left by the refined form) are solved; they keep status FALLBACK.
template <int D, int P, int MAXM>
__device__ __forceinline__ void stencil_f64_any(const StencilArgs& a, int64_t node, double* lds) {
    if constexpr (MAXM <= 64) stencil_f64_gj<D, P, MAXM>(a, node, lds);
    else stencil_f64<D, P, MAXM>(a, node, lds);
}

template <int D, int P, int MAXM>
constexpr int f64_lds_doubles() {
    return MAXM <= 64 ? GjLds<D, P, MAXM>::TOTAL : n_mono(D, P) * (MAXM - n_mono(D, P));
}

template <int D, int P, int MAXM>
__global__ __launch_bounds__(MAXM <= 64 ? 256 : 64, MAXM <= 64 ? 3 : 1) void k_weights_f64(StencilArgs a, int64_t N, int fallback_pass) {
    constexpr int WPB = waves_per_block<MAXM>();
    __shared__ __attribute__((aligned(16))) double lds[WPB][f64_lds_doubles<D, P, MAXM>()];
    const int wv = threadIdx.x / WAVE;
    const int64_t node = (int64_t)blockIdx.x * WPB + wv;
    if (node >= N) return;
    // one body for both uses (a second call site would duplicate the unrolled code)
    if (fallback_pass && a.status[node] != RBF_ST_FALLBACK) return;
    stencil_f64_any<D, P, MAXM>(a, node, lds[wv]);
    if (fallback_pass && lane_id() == 0 && a.status[node] == RBF_ST_OK) a.status[node] = RBF_ST_FALLBACK;
}

// FP32 LU + FP64 refinement; stencils not accepted are marked FALLBACK.
template <int D, int P, int MAXM>
constexpr int ir_lds_doubles() {
    if constexpr (MAXM <= 64) return IrLds<D, P, MAXM>::TOTAL;
    else return 2;
}

template <int D, int P, int MAXM>
__global__ __launch_bounds__(MAXM <= 64 ? 256 : 64, MAXM <= 64 ? 3 : 1) void k_weights_ir(StencilArgs a, int64_t N, int max_refine,
                                                                      double refine_tol) {
    constexpr int WPB = waves_per_block<MAXM>();
    __shared__ __attribute__((aligned(16))) double lds[WPB][ir_lds_doubles<D, P, MAXM>()];
    const int wv = threadIdx.x / WAVE;
    const int64_t node = (int64_t)blockIdx.x * WPB + wv;
    if (node >= N) return;
    if constexpr (MAXM <= 64) stencil_ir_gj<D, P, MAXM>(a, node, lds[wv], max_refine, refine_tol);
}

using LaunchFn = hipError_t (*)(const StencilArgs&, int64_t, int, int, double, hipStream_t);

template <int D, int P, int MAXM>
hipError_t launch_class(const StencilArgs& a, int64_t N, int precision, int max_refine, double refine_tol,
                        hipStream_t s) {
    constexpr int WPB = waves_per_block<MAXM>();
    dim3 grid((unsigned)((N + WPB - 1) / WPB)), block(64 * WPB);
    if (precision == RBF_PREC_F64 || MAXM > 64) {
        // the refined form keeps FP64 rows in registers and exists for n + m <= 64 only
        hipLaunchKernelGGL((k_weights_f64<D, P, MAXM>), grid, block, 0, s, a, N, 0);
    } else {
        hipLaunchKernelGGL((k_weights_ir<D, P, MAXM>), grid, block, 0, s, a, N, max_refine, refine_tol);
        hipLaunchKernelGGL((k_weights_f64<D, P, MAXM>), grid, block, 0, s, a, N, 1);
    }
    return hipGetLastError();
}

struct ClassEntry {
    int d, P, maxm;
    LaunchFn fn;
};

// registry shared by all translation units (defined in weights.hip)
void register_class(const ClassEntry& e);

struct ClassRegistrar {
    explicit ClassRegistrar(const ClassEntry& e) { register_class(e); }
};

}  // namespace rbf

#define RBF_WEIGHTS_CLASS(D, P, MX)                                                                  \
    namespace {                                                                                      \
    const rbf::ClassRegistrar rbf_reg_##D##_##P##_##MX(rbf::ClassEntry{D, P, MX, &rbf::launch_class<D, P, MX>}); \
    }
