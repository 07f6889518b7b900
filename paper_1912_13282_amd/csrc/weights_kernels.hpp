// Kernels of the RBF-FD weight computation and their per-size-class registry.
// A class is the register-array size MAXM (system size n + m <= MAXM); every
// class is instantiated in a translation unit of its own (wcls_*.hip) so the
// unrolled solvers compile in parallel, and registers its launcher at load time.
#pragma once

#include "wsolve.hpp"
#include "wsolve_pair.hpp"
#include "wsolve_quad.hpp"

namespace rbf {

// Plain FP64 solve.  With select != 0 only the stencils whose status equals
// select (FALLBACK left by the refined form, SURROGATE_REJECTED left by the
// surrogate) are solved, and a successful solve keeps that status.
template <int MAXM>
__global__ __launch_bounds__(256, 3) void k_weights_f64(StencilArgs a, int64_t N, int select) {
    static_assert(MAXM <= 64, "one row per lane");
    __shared__ __attribute__((aligned(16))) double lds[4][RowLds<MAXM>::TOTAL];
    const int wv = threadIdx.x / WAVE;
    const int64_t node = (int64_t)blockIdx.x * 4 + wv;
    if (node >= N) return;
    // one call site: a second one would duplicate the unrolled solver
    if (select && a.status[node] != select) return;
    stencil_f64_rows<MAXM, false>(a, node, node_degree(a, node), lds[wv]);
    if (select && lane_id() == 0 && a.status[node] == RBF_ST_OK) a.status[node] = (int8_t)select;
}

// Plain FP64 solve of systems above 64 unknowns: one stencil per 4-wave workgroup.
template <int MAXM>
__global__ __launch_bounds__(256, 3) void k_weights_quad(StencilArgs a, int64_t N, int select) {
    static_assert(MAXM > 64 && MAXM <= 128, "two row groups of 64, two column halves");
    __shared__ __attribute__((aligned(16))) double lds[QuadLds<MAXM / 2>::TOTAL];
    const int64_t node = blockIdx.x;
    if (node >= N) return;
    if (select && a.status[node] != select) return;  // uniform
    stencil_f64_quad<MAXM / 2>(a, node, node_degree(a, node), lds);
    if (select && threadIdx.x == 0 && a.status[node] == RBF_ST_OK) a.status[node] = (int8_t)select;
}

// FP32 Gauss-Jordan + FP64 refinement; stencils not accepted are marked FALLBACK.
template <int MAXM>
__global__ __launch_bounds__(256, 3) void k_weights_ir(StencilArgs a, int64_t N, int max_refine, double refine_tol) {
    static_assert(MAXM <= 64, "the refined form keeps one row per lane");
    __shared__ __attribute__((aligned(16))) double lds[4][RowLds<MAXM>::TOTAL];
    const int wv = threadIdx.x / WAVE;
    const int64_t node = (int64_t)blockIdx.x * 4 + wv;
    if (node >= N) return;
    stencil_ir_rows<MAXM, false>(a, node, node_degree(a, node), lds[wv], max_refine, refine_tol);
}

// FP32 Gauss-Jordan + FP64 refinement of systems above 64 unknowns: one stencil
// per wavefront, two rows per lane; stencils not accepted are marked FALLBACK.
template <int MAXM>
__global__ __launch_bounds__(256, 1) void k_weights_ir_pair(StencilArgs a, int64_t N, int max_refine,
                                                             double refine_tol) {
    __shared__ __attribute__((aligned(16))) double lds[4][PairLds<MAXM>::TOTAL];
    const int wv = threadIdx.x / WAVE;
    const int64_t node = (int64_t)blockIdx.x * 4 + wv;
    if (node >= N) return;
    stencil_ir_pair<MAXM>(a, node, node_degree(a, node), lds[wv], max_refine, refine_tol);
}

using LaunchFn = hipError_t (*)(const StencilArgs&, int64_t, int, int, double, hipStream_t);

template <int MAXM>
hipError_t launch_class(const StencilArgs& a, int64_t N, int precision, int max_refine, double refine_tol,
                        hipStream_t s) {
    if constexpr (MAXM > 64) {
        if (precision == RBF_PREC_F32_IR && MAXM <= PAIR_MAXM) {
            hipLaunchKernelGGL((k_weights_ir_pair<MAXM>), dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, a, N,
                               max_refine, refine_tol);
            hipLaunchKernelGGL((k_weights_quad<MAXM>), dim3((unsigned)N), dim3(256), 0, s, a, N, RBF_ST_FALLBACK);
        } else {
            // no refined form in this class: float64 directly (the refined form
            // reports FALLBACK)
            hipLaunchKernelGGL((k_weights_quad<MAXM>), dim3((unsigned)N), dim3(256), 0, s, a, N, 0);
        }
    } else {
        const dim3 grid((unsigned)((N + 3) / 4)), block(256);
        if (precision == RBF_PREC_F64) {
            hipLaunchKernelGGL((k_weights_f64<MAXM>), grid, block, 0, s, a, N, 0);
        } else {
            hipLaunchKernelGGL((k_weights_ir<MAXM>), grid, block, 0, s, a, N, max_refine, refine_tol);
            hipLaunchKernelGGL((k_weights_f64<MAXM>), grid, block, 0, s, a, N, RBF_ST_FALLBACK);
        }
    }
    return hipGetLastError();
}

// plain FP64 solve of the stencils whose status equals select
template <int MAXM>
hipError_t launch_select(const StencilArgs& a, int64_t N, int select, hipStream_t s) {
    if constexpr (MAXM > 64)
        hipLaunchKernelGGL((k_weights_quad<MAXM>), dim3((unsigned)N), dim3(256), 0, s, a, N, select);
    else
        hipLaunchKernelGGL((k_weights_f64<MAXM>), dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, a, N, select);
    return hipGetLastError();
}

using SelectFn = hipError_t (*)(const StencilArgs&, int64_t, int, hipStream_t);

struct ClassEntry {
    int maxm;
    LaunchFn fn;
    SelectFn fallback;
};

// registry shared by all translation units (defined in weights.hip)
void register_class(const ClassEntry& e);
// smallest compiled class holding systems of M unknowns, or NULL
const ClassEntry* find_class(int M);

struct ClassRegistrar {
    explicit ClassRegistrar(const ClassEntry& e) { register_class(e); }
};

}  // namespace rbf

#define RBF_WEIGHTS_CLASS(MX) \
    namespace {               \
    const rbf::ClassRegistrar rbf_reg_##MX(rbf::ClassEntry{MX, &rbf::launch_class<MX>, &rbf::launch_select<MX>}); \
    }
