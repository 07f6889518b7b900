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

// The ranks come from one atomic per class present in a wavefront (the lanes of
// a class take consecutive ranks after the wave's base), not one per stencil:
// with a handful of classes, per-stencil atomics on the same few counters
// serialise.
__global__ __launch_bounds__(256) void k_bclassify(const BParams* __restrict__ bpp, int* __restrict__ counts,
                                                   uint32_t* __restrict__ cls_rank) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const BParams& bp = *bpp;
    const bool in = g < bp.total;
    int c = BREJECT;
    if (in) {
        const BDom& D = bp.dom[find_dom(bp, g)];
        const int64_t i = g - D.first;
        const int P = D.degree ? (int)D.degree[i] : D.a.P;
        const int64_t off = D.a.offsets[i];
        const int64_t n = D.a.offsets[i + 1] - off;
        if (P >= 0 && P <= 4 && n >= 1 && n <= D.a.n_max && off >= 0 && off + n <= D.a.nnz) {
            const int M = (int)n + binom(P + D.a.d, D.a.d);
            for (int k = NBCLS - 1; k >= 0; --k)
                if (M <= bcls_maxm(k)) c = k;
        }
    }
    const int lane = lane_id();
    uint64_t rem = ballot64(in);
    int r = 0;
    while (rem) {  // wave-uniform: one pass per class present
        const int leader = first_lane(rem);
        const int cl = __builtin_amdgcn_readlane(c, leader);
        const uint64_t same = ballot64(in && c == cl);
        int base = 0;
        if (lane == leader) base = atomicAdd(&counts[cl], __builtin_popcountll(same));
        base = __builtin_amdgcn_readlane(base, leader);
        if (in && c == cl)
            r = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(same >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)same, 0u));
        rem &= ~same;
    }
    if (!in) return;
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

// Enqueue the batched computation with the given per-class plans.  With ev
// (NBCLS + 1 events) the launches of class c (its solve and, for the refined
// form, its float64 fallback pass) are bracketed by ev[c] and ev[c + 1].
rbf_status run_batched(rbf_ctx* ctx, const rbf_domain_desc* doms, int n_doms, const rbf_options& o, void* ws,
                       size_t ws_bytes, const int* chunk, const int* waves_per_cu, hipEvent_t* ev = nullptr) {
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
    if (ev && hipEventRecord(ev[0], s) != hipSuccess) return RBF_EHIP;
    for (int c = 0; c < NBCLS; ++c) {
        if (!g_bclass[c]) return RBF_EUNSUPPORTED;
        const int grid = cus * waves_per_cu[c];
        if (g_bclass[c](dbp, items, starts, counter + c, c, o.precision, chunk[c], grid, o.max_refine, o.refine_tol,
                        0, s) != hipSuccess)
            return RBF_EHIP;
        // the refined form's float64 pass over this class's fallbacks
        if (o.precision == RBF_PREC_F32_IR && bcls_maxm(c) <= PAIR_MAXM &&
            g_bclass[c](dbp, items, starts, counter + NBCLS + c, c, RBF_PREC_F64, chunk[c], grid, 0, 0.0,
                        RBF_ST_FALLBACK, s) != hipSuccess)
            return RBF_EHIP;
        if (ev && hipEventRecord(ev[c + 1], s) != hipSuccess) return RBF_EHIP;
    }
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

// the context's plan of every class (the defaults where none is set)
static void ctx_plans(const rbf_ctx* ctx, int* chunk, int* wpc) {
    for (int c = 0; c < rbf::NBCLS; ++c) {
        chunk[c] = ctx->plan_valid ? ctx->plan_chunk[c] : 4;
        wpc[c] = ctx->plan_valid ? ctx->plan_waves_per_cu[c] : 8;
    }
}

extern "C" rbf_status rbf_batched_class_size(int cls, int* maxm) {
    if (!maxm || cls < 0 || cls >= rbf::NBCLS) return RBF_EINVAL;
    *maxm = rbf::bcls_maxm(cls);
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
    int chunk[rbf::NBCLS], wpc[rbf::NBCLS];
    ctx_plans(ctx, chunk, wpc);
    return rbf::run_batched(ctx, doms, n_doms, o, workspace, ws_bytes, chunk, wpc);
}

extern "C" rbf_status rbf_set_plan(rbf_ctx* ctx, const rbf_plan* plans) {
    if (!ctx) return RBF_EINVAL;
    if (!plans) {
        ctx->plan_valid = 0;
        return RBF_OK;
    }
    for (int c = 0; c < rbf::NBCLS; ++c)
        if (plans[c].chunk < 1 || plans[c].chunk > 4096 || plans[c].waves_per_cu < 1 || plans[c].waves_per_cu > 64)
            return RBF_EINVAL;
    for (int c = 0; c < rbf::NBCLS; ++c) {
        ctx->plan_chunk[c] = plans[c].chunk;
        ctx->plan_waves_per_cu[c] = plans[c].waves_per_cu;
    }
    ctx->plan_valid = 1;
    return RBF_OK;
}

extern "C" rbf_status rbf_get_plan(const rbf_ctx* ctx, rbf_plan* plans) {
    if (!ctx || !plans) return RBF_EINVAL;
    int chunk[rbf::NBCLS], wpc[rbf::NBCLS];
    ctx_plans(ctx, chunk, wpc);
    for (int c = 0; c < rbf::NBCLS; ++c) plans[c] = rbf_plan{chunk[c], wpc[c], 0.0f};
    return RBF_OK;
}

// Plan search: every (chunk, waves per CU) candidate runs the whole batch once
// (after one warm-up run) with all classes on that candidate; each class's
// launches are timed separately with HIP events on the context stream, and each
// class keeps its fastest candidate.  This call synchronises.  With a cache
// path, plans stored there for the same signature (device, solver options,
// batch shape) are reused without timing, and newly tuned plans are appended.
extern "C" rbf_status rbf_autotune_batched(rbf_ctx* ctx, const rbf_domain_desc* doms, int n_doms,
                                           const rbf_options* opt, void* workspace, size_t ws_bytes,
                                           const char* cache_path, rbf_plan* best_out) {
    using rbf::NBCLS;
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
    // signature: device, solver options, domain shapes
    char opts[256];
    snprintf(opts, sizeof(opts), "|p%d|k%d|r%d|t%.17g|s%d|q%.17g", o.precision, o.phs_power, o.max_refine,
             o.refine_tol, o.scale_mode, o.repro_tol);
    std::string key = std::string(prop.gcnArchName) + opts;
    for (int k = 0; k < n_doms; ++k)
        key += "|" + std::to_string(doms[k].d) + ":" + std::to_string(doms[k].N) + ":" + std::to_string(doms[k].nnz) +
               ":" + std::to_string(doms[k].degree ? -1 : doms[k].degree_uniform) + ":" +
               std::to_string(doms[k].n_max) + ":" + std::to_string(doms[k].op_mask);
    for (char& ch : key)
        if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
    rbf_plan best[NBCLS];
    if (cache_path) {
        FILE* f = fopen(cache_path, "r");
        if (f) {
            char buf[4096];
            while (fgets(buf, sizeof(buf), f)) {
                char* save = nullptr;
                char* tok = strtok_r(buf, " \n", &save);
                if (!tok || key != tok) continue;
                int v[2 * NBCLS];
                bool okl = true;
                for (int i = 0; i < 2 * NBCLS && okl; ++i) {
                    tok = strtok_r(nullptr, " \n", &save);
                    okl = tok && sscanf(tok, "%d", &v[i]) == 1 && v[i] >= 1;
                }
                if (!okl) continue;
                for (int c = 0; c < NBCLS; ++c) best[c] = rbf_plan{v[2 * c], v[2 * c + 1], 0.0f};
                fclose(f);
                st = rbf_set_plan(ctx, best);
                if (st == RBF_OK && best_out)
                    for (int c = 0; c < NBCLS; ++c) best_out[c] = best[c];
                return st;
            }
            fclose(f);
        }
    }
    const int chunks[] = {1, 2, 4, 8, 16};
    const int waves[] = {4, 8, 12, 16};
    hipEvent_t ev[NBCLS + 1];
    for (int c = 0; c <= NBCLS; ++c) RBF_HIP_CHECK(hipEventCreate(&ev[c]));
    for (int c = 0; c < NBCLS; ++c) best[c] = rbf_plan{4, 8, 1e30f};
    int cc[NBCLS], ww[NBCLS];
    ctx_plans(ctx, cc, ww);
    for (int c = 0; c < NBCLS; ++c) cc[c] = 4, ww[c] = 8;
    st = rbf::run_batched(ctx, doms, n_doms, o, workspace, ws_bytes, cc, ww);  // warm-up
    float total_ms = 0.0f;
    if (st == RBF_OK) {
        for (int ch : chunks)
            for (int w : waves) {
                for (int c = 0; c < NBCLS; ++c) cc[c] = ch, ww[c] = w;
                st = rbf::run_batched(ctx, doms, n_doms, o, workspace, ws_bytes, cc, ww, ev);
                if (st != RBF_OK) break;
                if (hipEventSynchronize(ev[NBCLS]) != hipSuccess) {
                    st = RBF_EHIP;
                    break;
                }
                for (int c = 0; c < NBCLS && st == RBF_OK; ++c) {
                    float ms = 0;
                    if (hipEventElapsedTime(&ms, ev[c], ev[c + 1]) != hipSuccess) st = RBF_EHIP;
                    else if (ms < best[c].ms) best[c] = rbf_plan{ch, w, ms};
                }
                if (st != RBF_OK) break;
            }
    }
    for (int c = 0; c <= NBCLS; ++c) (void)hipEventDestroy(ev[c]);
    if (st != RBF_OK) return st;
    for (int c = 0; c < NBCLS; ++c) total_ms += best[c].ms;
    st = rbf_set_plan(ctx, best);
    if (st != RBF_OK) return st;
    if (best_out)
        for (int c = 0; c < NBCLS; ++c) best_out[c] = best[c];
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s", key.c_str());
            for (int c = 0; c < NBCLS; ++c) fprintf(f, " %d %d", best[c].chunk, best[c].waves_per_cu);
            fprintf(f, " %.4f\n", total_ms);
            fclose(f);
        }
    }
    return RBF_OK;
}
