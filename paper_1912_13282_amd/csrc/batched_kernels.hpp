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
#include "wsolve_pair.hpp"
#include "wsolve_quad.hpp"

namespace rbf {

constexpr int BMAX_DOMS = 16;
constexpr int NBCLS = RBF_BATCHED_CLASSES;  // size classes
constexpr int BREJECT = NBCLS;  // class index of invalid stencils (bad size / degree)
__host__ __device__ constexpr int bcls_maxm(int c) {
    return c == 0 ? 24 : c == 1 ? 32 : c == 2 ? 48 : c == 3 ? 64 : c == 4 ? 80 : c == 5 ? 100 : c == 6 ? 108 : 128;
}
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


// The persistent loops call the solvers through these non-inlined functions:
// register allocation across a loop around a fully unrolled solver spills
// heavily, while a call keeps the solver's allocation separate.  The stencil
// arguments are re-made uniform (scalar registers) inside the callee, and each
// callee owns its LDS.
template <typename T>
__device__ __forceinline__ T* rfl_ptr(T* p) {
    const uint64_t v = (uint64_t)p;
    return (T*)((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v & 0xFFFFFFFFu)) |
                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32));
}
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t rfl64(int64_t v) {
    return (int64_t)((uint64_t)(uint32_t)rfl((int)(v & 0xFFFFFFFF)) | ((uint64_t)(uint32_t)rfl((int)(v >> 32)) << 32));
}
__device__ __forceinline__ double rfld(double v) { return __hiloint2double(rfl(__double2hiint(v)), rfl(__double2loint(v))); }

__device__ __forceinline__ StencilArgs uniform_args(const StencilArgs& a0) {
    StencilArgs a;
    a.X = rfl_ptr(a0.X);
    a.N = rfl64(a0.N);
    a.d = rfl(a0.d);
    a.P = rfl(a0.P);
    a.offsets = rfl_ptr(a0.offsets);
    a.idx = rfl_ptr(a0.idx);
    a.nnz = rfl64(a0.nnz);
    a.n_max = rfl(a0.n_max);
    a.op_mask = (unsigned)rfl((int)a0.op_mask);
    a.opc = (unsigned)rfl((int)a0.opc);
    a.phs_power = rfl(a0.phs_power);
    a.scale_mode = rfl(a0.scale_mode);
    a.repro_tol = rfld(a0.repro_tol);
    a.w = rfl_ptr(a0.w);
    a.status = rfl_ptr(a0.status);
    return a;
}

template <int PREC, int MAXM>
__device__ __attribute__((noinline)) void solve_item_rows(StencilArgs a0, int64_t node, int P, int max_refine,
                                                          double refine_tol) {
    __shared__ __attribute__((aligned(16))) double lds[RowLds<MAXM>::TOTAL];
    const StencilArgs a = uniform_args(a0);
    if constexpr (PREC == RBF_PREC_F64)
        stencil_f64_rows<MAXM, true>(a, rfl64(node), rfl(P), lds);
    else
        stencil_ir_rows<MAXM, true>(a, rfl64(node), rfl(P), lds, rfl(max_refine), rfld(refine_tol));
}

template <int MAXM>
__device__ __attribute__((noinline)) void solve_item_pair(StencilArgs a0, int64_t node, int P, int max_refine,
                                                          double refine_tol) {
    __shared__ __attribute__((aligned(16))) double lds[PairLds<MAXM>::TOTAL];
    stencil_ir_pair<MAXM>(uniform_args(a0), rfl64(node), rfl(P), lds, rfl(max_refine), rfld(refine_tol));
}

template <int H>
__device__ __attribute__((noinline)) void solve_item_quad(StencilArgs a0, int64_t node, int P) {
    __shared__ __attribute__((aligned(16))) double lds[QuadLds<H>::TOTAL];
    stencil_f64_quad<H>(uniform_args(a0), rfl64(node), rfl(P), lds);
}

// Persistent solve of size class `cls` (items starts[cls] .. starts[cls+1]).
// select != 0: only items whose status equals select are solved (the FP64 pass
// over the refined form's fallbacks) and keep that status.
template <int PREC, int MAXM>
__global__ __launch_bounds__(64, MAXM <= 32 ? 4 : (MAXM <= 48 ? 3 : 2)) void k_bclass(
    const BParams* __restrict__ bpp, const uint64_t* __restrict__ items, const int64_t* __restrict__ starts,
    unsigned long long* __restrict__ counter, int cls, int chunk, int max_refine, double refine_tol, int select) {
    static_assert(MAXM <= 64, "one row per lane");
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
            solve_item_rows<PREC, MAXM>(D.a, node, P, max_refine, refine_tol);
            if (select && lane_id() == 0 && D.a.status[node] == RBF_ST_OK) D.a.status[node] = (int8_t)select;
        }
    }
}

// Persistent FP32 + FP64-refinement solve of a class above 64 unknowns: one
// stencil per wave (two float rows per lane); rejected stencils are marked
// FALLBACK for the float64 pass.
template <int MAXM>
__global__ __launch_bounds__(64, 1) void k_bclass_pair(const BParams* __restrict__ bpp,
                                                       const uint64_t* __restrict__ items,
                                                       const int64_t* __restrict__ starts,
                                                       unsigned long long* __restrict__ counter, int cls, int chunk,
                                                       int max_refine, double refine_tol) {
    static_assert(MAXM > 64 && MAXM <= PAIR_MAXM, "two float rows per lane");
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
            const int P = D.degree ? (int)D.degree[node] : D.a.P;
            solve_item_pair<MAXM>(D.a, node, P, max_refine, refine_tol);
        }
    }
}

// Persistent float64 solve of a class above 64 unknowns: 4-wave workgroups, one
// stencil at a time per workgroup (the refined form of a class without a
// refined solver reports FALLBACK).
template <int PREC, int MAXM>
__global__ __launch_bounds__(256, 3) void k_bclass_quad(const BParams* __restrict__ bpp,
                                                        const uint64_t* __restrict__ items,
                                                        const int64_t* __restrict__ starts,
                                                        unsigned long long* __restrict__ counter, int cls, int chunk,
                                                        int select) {
    static_assert(MAXM > 64 && MAXM <= 128, "two row groups of 64, two column halves");
    __shared__ unsigned long long grab;
    const BParams& bp = *bpp;
    const int64_t beg = starts[cls], end = starts[cls + 1];
    for (;;) {
        if (threadIdx.x == 0) grab = atomicAdd(counter, (unsigned long long)chunk);
        __syncthreads();
        // uniform by construction; readfirstlane lets the compiler know, so every
        // value derived from the item stays in scalar registers
        const unsigned long long gv = grab;
        const int64_t t0 = beg + (int64_t)((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                               (int)(gv & 0xFFFFFFFFull)) |
                                           ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                                (int)(gv >> 32)) << 32));
        __syncthreads();  // every thread has read grab before it is written again
        if (t0 >= end) break;  // uniform: the whole workgroup leaves once the class is drained
        const int64_t t1 = (t0 + chunk < end) ? t0 + chunk : end;
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t g = (int64_t)items[t];
            const BDom& D = bp.dom[find_dom(bp, g)];
            const int64_t node = g - D.first;
            if (select && D.a.status[node] != select) continue;
            const int P = D.degree ? (int)D.degree[node] : D.a.P;
            solve_item_quad<MAXM / 2>(D.a, node, P);
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
        if (precision == RBF_PREC_F32_IR) {
            if constexpr (MAXM <= PAIR_MAXM)
                hipLaunchKernelGGL((k_bclass_pair<MAXM>), dim3(grid), dim3(64), 0, s, bp, items, starts, counter, cls,
                                   chunk, max_refine, refine_tol);
            else
                hipLaunchKernelGGL((k_bclass_quad<RBF_PREC_F32_IR, MAXM>), dim3(g4), dim3(256), 0, s, bp, items,
                                   starts, counter, cls, chunk, select);
        } else
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
