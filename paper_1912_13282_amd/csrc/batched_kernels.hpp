// Batched persistent RBF-FD weights: shared types and the per-size-class
// persistent kernel.
//
// The stencils of every domain of a batch are sorted into size classes by
// n + m (MAXM = 24, 32, 48, 64, 128); dimension and degree stay runtime values
// inside a class.  Each class runs ONE persistent launch: a fixed grid of
// single-wave workgroups (four-wave workgroups above 64 unknowns) that take
// `chunk` items at a time from the class's atomic counter until the class's
// range of the work list is drained, so uneven stencils balance dynamically.  Classes are separate kernels because a
// GPU kernel's register budget is the maximum over all the code it contains:
// one kernel for every size would run the 24-unknown systems at the occupancy
// of the 128-unknown solver.
#pragma once

#include "wsolve.hpp"
#include "wsolve_quad.hpp"

namespace rbf {

constexpr int BMAX_DOMS = 16;
constexpr int NBCLS = 5;      // size classes
constexpr int BREJECT = NBCLS;  // class index of invalid stencils (bad size / degree)
__host__ __device__ constexpr int bcls_maxm(int c) { return c == 0 ? 24 : c == 1 ? 32 : c == 2 ? 48 : c == 3 ? 64 : 128; }
constexpr int NCOUNTERS = 2 * NBCLS;  // one work counter per class and pass

struct BDom {
    StencilArgs a;         // a.d is the domain's dimension, a.P its uniform degree
    const int8_t* degree;  // per-node degree, or NULL
    int64_t first;         // first global item of this domain
};

struct BParams {
    int n_doms;
    int64_t total;
    BDom dom[BMAX_DOMS];
};

__device__ __forceinline__ int find_dom(const BParams& bp, int64_t g) {
    int d = 0;
    for (int k = 1; k < bp.n_doms; ++k)
        if (g >= bp.dom[k].first) d = k;
    return d;
}


// Persistent solve of size class `cls` (items starts[cls] .. starts[cls+1]).
// select != 0: only items whose status equals select are solved (the FP64 pass
// over the refined form's fallbacks) and keep that status.
template <int PREC, int MAXM>
__global__ __launch_bounds__(64, MAXM <= 32 ? 4 : (MAXM <= 48 ? 3 : 2)) void k_bclass(
    const BParams* __restrict__ bpp, const uint64_t* __restrict__ items, const int64_t* __restrict__ starts,
    unsigned long long* __restrict__ counter, int cls, int chunk, int max_refine, double refine_tol, int select) {
    static_assert(MAXM <= 64, "one row per lane");
    __shared__ __attribute__((aligned(16))) double lds[RowLds<MAXM>::TOTAL];
    const BParams& bp = *bpp;
    const int64_t beg = starts[cls], end = starts[cls + 1];
    for (;;) {
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(counter, (unsigned long long)chunk);
        base = (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(base & 0xFFFFFFFFull)) |
               ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32);
        const int64_t t0 = beg + (int64_t)base;
        if (t0 >= end) break;  // every wave leaves once the class is drained
        const int64_t t1 = (t0 + chunk < end) ? t0 + chunk : end;
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t g = (int64_t)items[t];
            const BDom& D = bp.dom[find_dom(bp, g)];
            const int64_t node = g - D.first;
            if (select && D.a.status[node] != select) continue;
            const int P = D.degree ? (int)D.degree[node] : D.a.P;
            if constexpr (PREC == RBF_PREC_F64) {
                stencil_f64_rows<MAXM, true>(D.a, node, P, lds);
            } else {
                stencil_ir_rows<MAXM, true>(D.a, node, P, lds, max_refine, refine_tol);
            }
            if (select && lane_id() == 0 && D.a.status[node] == RBF_ST_OK) D.a.status[node] = (int8_t)select;
        }
    }
}

// Persistent solve of the class above 64 unknowns: 4-wave workgroups, one
// stencil at a time per workgroup (float64; the refined form reports FALLBACK).
template <int PREC, int MAXM>
__global__ __launch_bounds__(256, 2) void k_bclass_quad(const BParams* __restrict__ bpp,
                                                        const uint64_t* __restrict__ items,
                                                        const int64_t* __restrict__ starts,
                                                        unsigned long long* __restrict__ counter, int cls, int chunk,
                                                        int select) {
    static_assert(MAXM > 64 && MAXM <= 128, "two row groups of 64, two column halves");
    __shared__ __attribute__((aligned(16))) double lds[QuadLds<MAXM / 2>::TOTAL];
    __shared__ unsigned long long grab;
    const BParams& bp = *bpp;
    const int64_t beg = starts[cls], end = starts[cls + 1];
    for (;;) {
        if (threadIdx.x == 0) grab = atomicAdd(counter, (unsigned long long)chunk);
        __syncthreads();
        const int64_t t0 = beg + (int64_t)grab;
        __syncthreads();  // every thread has read grab before it is written again
        if (t0 >= end) break;  // uniform: the whole workgroup leaves once the class is drained
        const int64_t t1 = (t0 + chunk < end) ? t0 + chunk : end;
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t g = (int64_t)items[t];
            const BDom& D = bp.dom[find_dom(bp, g)];
            const int64_t node = g - D.first;
            if (select && D.a.status[node] != select) continue;
            const int P = D.degree ? (int)D.degree[node] : D.a.P;
            stencil_f64_quad<MAXM / 2>(D.a, node, P, lds);
            if (threadIdx.x == 0 && D.a.status[node] == RBF_ST_OK) {
                if (PREC == RBF_PREC_F32_IR) D.a.status[node] = RBF_ST_FALLBACK;
                else if (select) D.a.status[node] = (int8_t)select;
            }
        }
    }
}

using BLaunchFn = hipError_t (*)(const BParams* bp, const uint64_t* items, const int64_t* starts,
                                 unsigned long long* counter, int cls, int precision, int chunk, int grid,
                                 int max_refine, double refine_tol, int select, hipStream_t s);

template <int MAXM>
hipError_t launch_bclass(const BParams* bp, const uint64_t* items, const int64_t* starts, unsigned long long* counter,
                         int cls, int precision, int chunk, int grid, int max_refine, double refine_tol, int select,
                         hipStream_t s) {
    if constexpr (MAXM > 64) {
        const int g4 = grid / 4 > 0 ? grid / 4 : 1;  // grid counts waves; a workgroup here is four
        if (precision == RBF_PREC_F32_IR)
            hipLaunchKernelGGL((k_bclass_quad<RBF_PREC_F32_IR, MAXM>), dim3(g4), dim3(256), 0, s, bp, items, starts,
                               counter, cls, chunk, select);
        else
            hipLaunchKernelGGL((k_bclass_quad<RBF_PREC_F64, MAXM>), dim3(g4), dim3(256), 0, s, bp, items, starts,
                               counter, cls, chunk, select);
    } else if (precision == RBF_PREC_F64) {
        hipLaunchKernelGGL((k_bclass<RBF_PREC_F64, MAXM>), dim3(grid), dim3(64), 0, s, bp, items, starts, counter, cls,
                           chunk, max_refine, refine_tol, select);
    } else {
        hipLaunchKernelGGL((k_bclass<RBF_PREC_F32_IR, MAXM>), dim3(grid), dim3(64), 0, s, bp, items, starts, counter,
                           cls, chunk, max_refine, refine_tol, select);
    }
    return hipGetLastError();
}

// registry of the compiled classes (defined in batched.hip)
void register_bclass(int maxm, BLaunchFn fn);

struct BClassRegistrar {
    BClassRegistrar(int maxm, BLaunchFn fn) { register_bclass(maxm, fn); }
};

}  // namespace rbf

#define RBF_BATCHED_CLASS(MX) \
    namespace {               \
    const rbf::BClassRegistrar rbf_breg_##MX(MX, &rbf::launch_bclass<MX>); \
    }
