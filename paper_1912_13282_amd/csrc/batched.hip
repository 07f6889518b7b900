// Batched persistent RBF-FD weights: stencils of several node sets, mixed
// dimension (2D/3D), augmentation degree (2..4) and size, in one persistent
// launch per size class and precision.
//
//   k_bclassify : size class of every stencil (smallest MAXM >= n + m) and its
//                 rank inside the class
//   k_bscan     : class offsets (one block); resets the work counters
//   k_bscatter  : class-sorted work list of (domain, node) items
//   k_bclass    : per class, a fixed grid of single-wave workgroups pulling
//                 chunks of the class's range from an atomic counter
//                 (batched_kernels.hpp, instantiated in bcls_*.hip)
//   k_breject   : NaN weights and BADSIZE for invalid stencils
// The FP32+refinement form adds one FP64 pass per class over its fallbacks.
// The plan (chunk, waves per CU) comes from rbf_autotune_batched, which times
// candidate plans on the caller's batch.
#include "batched_kernels.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

namespace rbf {

static BLaunchFn g_bclass[NBCLS];

void register_bclass(int maxm, BLaunchFn fn) {
    for (int c = 0; c < NBCLS; ++c)
        if (bcls_maxm(c) == maxm) g_bclass[c] = fn;
}

__global__ __launch_bounds__(64) void k_bzero(int* __restrict__ counts) {
    if (threadIdx.x <= BREJECT) counts[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_bclassify(const BParams* __restrict__ bpp, int* __restrict__ counts,
                                                   uint32_t* __restrict__ cls_rank) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const BParams& bp = *bpp;
    if (g >= bp.total) return;
    const BDom& D = bp.dom[find_dom(bp, g)];
    const int64_t i = g - D.first;
    const int P = D.degree ? (int)D.degree[i] : D.a.P;
    const int64_t off = D.a.offsets[i];
    const int64_t n = D.a.offsets[i + 1] - off;
    int c = BREJECT;
    if (P >= 0 && P <= 4 && n >= 1 && n <= D.a.n_max && off >= 0 && off + n <= D.a.nnz) {
        const int M = (int)n + binom(P + D.a.d, D.a.d);
        for (int k = NBCLS - 1; k >= 0; --k)
            if (M <= bcls_maxm(k)) c = k;
    }
    const int r = atomicAdd(&counts[c], 1);
    cls_rank[2 * g] = (uint32_t)c;
    cls_rank[2 * g + 1] = (uint32_t)r;
}

__global__ __launch_bounds__(64) void k_bscan(const int* __restrict__ counts, int64_t* __restrict__ starts,
                                              unsigned long long* __restrict__ counters) {
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int c = 0; c <= BREJECT; ++c) {
            starts[c] = s;
            s += counts[c];
        }
        starts[BREJECT + 1] = s;
    }
    if (threadIdx.x < NCOUNTERS) counters[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_bscatter(const BParams* __restrict__ bpp, const uint32_t* __restrict__ cls_rank,
                                                  const int64_t* __restrict__ starts, uint64_t* __restrict__ items) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= bpp->total) return;
    const uint32_t c = cls_rank[2 * g], r = cls_rank[2 * g + 1];
    items[starts[c] + r] = (uint64_t)g;
}

// invalid stencils: one wave per item, NaN weights inside the valid part of the arrays
__global__ __launch_bounds__(256) void k_breject(const BParams* __restrict__ bpp, const uint64_t* __restrict__ items,
                                                 const int64_t* __restrict__ starts) {
    const BParams& bp = *bpp;
    const int64_t beg = starts[BREJECT], end = starts[BREJECT + 1];
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t t = beg + (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; t < end; t += nw) {
        const int64_t g = (int64_t)items[t];
        const BDom& D = bp.dom[find_dom(bp, g)];
        const int64_t node = g - D.first;
        const int64_t off = D.a.offsets[node];
        const int64_t n = D.a.offsets[node + 1] - off;
        reject_stencil(D.a, node, off, (n < 0 || off < 0 || off + n > D.a.nnz) ? 0 : n, RBF_ST_BADSIZE);
    }
}

struct BLayout {
    size_t params, counts, starts, counter, cls_rank, items, total;
};

BLayout blayout(int64_t total) {
    BLayout L;
    size_t o = 0;
    L.params = o;
    o += rbf_align(sizeof(BParams));
    L.counts = o;
    o += rbf_align(sizeof(int) * (BREJECT + 1));
    L.starts = o;
    o += rbf_align(sizeof(int64_t) * (BREJECT + 2));
    L.counter = o;
    o += rbf_align(sizeof(unsigned long long) * NCOUNTERS);
    L.cls_rank = o;
    o += rbf_align(sizeof(uint32_t) * 2 * total);
    L.items = o;
    o += rbf_align(sizeof(uint64_t) * total);
    L.total = o;
    return L;
}

rbf_status check_doms(const rbf_domain_desc* doms, int n_doms, int64_t* total) {
    if (!doms || n_doms < 1 || n_doms > BMAX_DOMS) return RBF_EINVAL;
    int64_t t = 0;
    for (int k = 0; k < n_doms; ++k) {
        const rbf_domain_desc& D = doms[k];
        if (!D.X || !D.offsets || !D.idx || !D.w || !D.status || D.N < 1 || D.nnz < 1 || D.n_max < 1) return RBF_EINVAL;
        if (D.d != 2 && D.d != 3) return RBF_EDIM;
        unsigned opc;
        if (op_slots(D.op_mask, D.d, &opc) < 0) return RBF_EINVAL;
        if (!D.degree && (D.degree_uniform < 0 || D.degree_uniform > 4)) return RBF_EUNSUPPORTED;
        if (D.n_max > D.N) return RBF_ETOOFEW;
        t += D.N;
    }
    *total = t;
    return RBF_OK;
}

// Enqueue the batched computation with a given plan.
rbf_status run_batched(rbf_ctx* ctx, const rbf_domain_desc* doms, int n_doms, const rbf_options& o, void* ws,
                       size_t ws_bytes, int chunk, int waves_per_cu) {
    int64_t total = 0;
    rbf_status st = check_doms(doms, n_doms, &total);
    if (st != RBF_OK) return st;
    BLayout L = blayout(total);
    if (!ws || ws_bytes < L.total) return RBF_EWORKSPACE;
    char* w = (char*)ws;
    BParams bp;
    memset(&bp, 0, sizeof(bp));
    bp.n_doms = n_doms;
    bp.total = total;
    int64_t first = 0;
    for (int k = 0; k < n_doms; ++k) {
        const rbf_domain_desc& D = doms[k];
        BDom& B = bp.dom[k];
        B.a.X = D.X;
        B.a.N = D.N;
        B.a.offsets = D.offsets;
        B.a.idx = D.idx;
        B.a.nnz = D.nnz;
        B.a.n_max = D.n_max;
        unsigned opc = 0;
        const int R = op_slots(D.op_mask, D.d, &opc);  // validated by check_doms
        B.a.op_mask = (1u << R) - 1u;
        B.a.opc = opc;
        B.a.phs_power = o.phs_power;
        B.a.scale_mode = o.scale_mode;
        B.a.repro_tol = o.repro_tol;
        B.a.w = D.w;
        B.a.status = D.status;
        B.a.d = D.d;
        B.a.P = D.degree_uniform;
        B.degree = D.degree;
        B.first = first;
        first += D.N;
    }
    hipStream_t s = ctx->stream;
    BParams* dbp = (BParams*)(w + L.params);
    int* counts = (int*)(w + L.counts);
    int64_t* starts = (int64_t*)(w + L.starts);
    unsigned long long* counter = (unsigned long long*)(w + L.counter);
    uint32_t* cls_rank = (uint32_t*)(w + L.cls_rank);
    uint64_t* items = (uint64_t*)(w + L.items);
    RBF_HIP_CHECK(hipMemcpyAsync(dbp, &bp, sizeof(bp), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bzero, dim3(1), dim3(64), 0, s, counts);
    const unsigned nb = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_bclassify, dim3(nb), dim3(256), 0, s, dbp, counts, cls_rank);
    hipLaunchKernelGGL(k_bscan, dim3(1), dim3(64), 0, s, counts, starts, counter);
    hipLaunchKernelGGL(k_bscatter, dim3(nb), dim3(256), 0, s, dbp, cls_rank, starts, items);
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) return RBF_EHIP;
    const int grid = cus * waves_per_cu;
    for (int c = 0; c < NBCLS; ++c) {
        if (!g_bclass[c]) return RBF_EUNSUPPORTED;
        if (g_bclass[c](dbp, items, starts, counter + c, c, o.precision, chunk, grid, o.max_refine, o.refine_tol, 0,
                        s) != hipSuccess)
            return RBF_EHIP;
    }
    if (o.precision == RBF_PREC_F32_IR)
        for (int c = 0; c < NBCLS; ++c)
            if (bcls_maxm(c) <= 64 &&
                g_bclass[c](dbp, items, starts, counter + NBCLS + c, c, RBF_PREC_F64, chunk, grid, 0, 0.0,
                            RBF_ST_FALLBACK, s) != hipSuccess)
                return RBF_EHIP;
    hipLaunchKernelGGL(k_breject, dim3(64), dim3(256), 0, s, dbp, items, starts);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}

}  // namespace rbf

extern "C" rbf_status rbf_batched_workspace(const rbf_domain_desc* doms, int n_doms, size_t* bytes) {
    if (!bytes) return RBF_EINVAL;
    int64_t total = 0;
    rbf_status st = rbf::check_doms(doms, n_doms, &total);
    if (st != RBF_OK) return st;
    *bytes = rbf::blayout(total).total;
    return RBF_OK;
}

extern "C" rbf_status rbf_compute_weights_batched(rbf_ctx* ctx, const rbf_domain_desc* doms, int n_doms,
                                                  const rbf_options* opt, void* workspace, size_t ws_bytes) {
    if (!ctx) return RBF_EINVAL;
    rbf_options o;
    rbf_options_default(&o);
    if (opt) o = *opt;
    if (o.precision != RBF_PREC_F64 && o.precision != RBF_PREC_F32_IR) return RBF_EINVAL;
    if ((o.phs_power != 3 && o.phs_power != 5) || o.max_refine < 0 || !(o.refine_tol >= 0.0)) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    const int chunk = ctx->plan_valid ? ctx->plan_chunk : 4;
    const int wpc = ctx->plan_valid ? ctx->plan_waves_per_cu : 8;
    return rbf::run_batched(ctx, doms, n_doms, o, workspace, ws_bytes, chunk, wpc);
}

extern "C" rbf_status rbf_set_plan(rbf_ctx* ctx, const rbf_plan* plan) {
    if (!ctx) return RBF_EINVAL;
    if (!plan) {
        ctx->plan_valid = 0;
        return RBF_OK;
    }
    if (plan->chunk < 1 || plan->chunk > 4096 || plan->waves_per_cu < 1 || plan->waves_per_cu > 64) return RBF_EINVAL;
    ctx->plan_valid = 1;
    ctx->plan_chunk = plan->chunk;
    ctx->plan_waves_per_cu = plan->waves_per_cu;
    return RBF_OK;
}

extern "C" rbf_status rbf_get_plan(const rbf_ctx* ctx, rbf_plan* plan) {
    if (!ctx || !plan) return RBF_EINVAL;
    plan->chunk = ctx->plan_valid ? ctx->plan_chunk : 4;
    plan->waves_per_cu = ctx->plan_valid ? ctx->plan_waves_per_cu : 8;
    plan->ms = 0.0f;
    return RBF_OK;
}

// Plan search: every (chunk, waves per CU) candidate runs the whole batch once
// (after one warm-up run) and is timed with HIP events on the context stream;
// the fastest becomes the context's plan.  This call synchronises.  With a
// cache path, a plan stored there for the same device and batch signature is
// reused without timing, and a newly tuned plan is appended.
extern "C" rbf_status rbf_autotune_batched(rbf_ctx* ctx, const rbf_domain_desc* doms, int n_doms,
                                           const rbf_options* opt, void* workspace, size_t ws_bytes,
                                           const char* cache_path, rbf_plan* best_out) {
    if (!ctx) return RBF_EINVAL;
    rbf_options o;
    rbf_options_default(&o);
    if (opt) o = *opt;
    int64_t total = 0;
    rbf_status st = rbf::check_doms(doms, n_doms, &total);
    if (st != RBF_OK) return st;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    RBF_HIP_CHECK(hipGetDeviceProperties(&prop, ctx->device));
    // batch signature: device, precision, domain sizes and shapes
    std::string key = std::string(prop.gcnArchName) + "|p" + std::to_string(o.precision);
    for (int k = 0; k < n_doms; ++k)
        key += "|" + std::to_string(doms[k].d) + ":" + std::to_string(doms[k].N) + ":" + std::to_string(doms[k].nnz) +
               ":" + std::to_string(doms[k].degree ? -1 : doms[k].degree_uniform) + ":" + std::to_string(doms[k].n_max);
    if (cache_path) {
        FILE* f = fopen(cache_path, "r");
        if (f) {
            char line[1024];
            while (fgets(line, sizeof(line), f)) {
                char k[900];
                int c = 0, w = 0;
                float ms = 0;
                if (sscanf(line, "%899s %d %d %f", k, &c, &w, &ms) == 4 && key == k && c >= 1 && w >= 1) {
                    fclose(f);
                    rbf_plan p{c, w, ms};
                    rbf_set_plan(ctx, &p);
                    if (best_out) *best_out = p;
                    return RBF_OK;
                }
            }
            fclose(f);
        }
    }
    const int chunks[] = {1, 2, 4, 8, 16};
    const int waves[] = {4, 8, 12, 16};
    hipEvent_t e0, e1;
    RBF_HIP_CHECK(hipEventCreate(&e0));
    RBF_HIP_CHECK(hipEventCreate(&e1));
    rbf_plan best{4, 8, 1e30f};
    st = rbf::run_batched(ctx, doms, n_doms, o, workspace, ws_bytes, 4, 8);  // warm-up
    if (st == RBF_OK) {
        for (int c : chunks)
            for (int w : waves) {
                if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = RBF_EHIP; break; }
                st = rbf::run_batched(ctx, doms, n_doms, o, workspace, ws_bytes, c, w);
                if (st != RBF_OK) break;
                if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    st = RBF_EHIP;
                    break;
                }
                float ms = 0;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = RBF_EHIP; break; }
                if (ms < best.ms) best = rbf_plan{c, w, ms};
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RBF_OK) return st;
    rbf_set_plan(ctx, &best);
    if (best_out) *best_out = best;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d %.4f\n", key.c_str(), best.chunk, best.waves_per_cu, best.ms);
            fclose(f);
        }
    }
    return RBF_OK;
}
