// Host entry point of the RBF-FD weight computation (eq. rbf-system-aug) and the
// registry of compiled size classes (instantiated in wcls_*.hip).
#include "weights_kernels.hpp"

#include <math.h>

#include <vector>

namespace rbf {

static std::vector<ClassEntry>& registry() {
    static std::vector<ClassEntry> r;
    return r;
}

void register_class(const ClassEntry& e) { registry().push_back(e); }

const ClassEntry* find_class(int M) {
    const ClassEntry* best = nullptr;
    for (const auto& c : registry())
        if (c.maxm >= M && (!best || c.maxm < best->maxm)) best = &c;
    return best;
}

}  // namespace rbf

__global__ __launch_bounds__(256) void k_mark_fallback(int8_t* __restrict__ status, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N && status[i] == RBF_ST_OK) status[i] = RBF_ST_FALLBACK;
}

extern "C" rbf_status rbf_options_default(rbf_options* opt) {
    if (!opt) return RBF_EINVAL;
    opt->precision = RBF_PREC_F64;
    opt->max_refine = 10;
    opt->phs_power = 3;
    opt->scale_mode = 0;
    opt->repro_tol = 1e-8;
    opt->refine_tol = 0.0;
    opt->surrogate_tol = 1e-6;
    opt->surrogate_corr_tol = 0.25;
    return RBF_OK;
}

extern "C" rbf_status rbf_compute_weights(rbf_ctx* ctx, const double* X, int64_t N, int d, const int64_t* offsets,
                                          const int32_t* idx, int64_t nnz, int n_max, const int8_t* degree,
                                          int degree_max, unsigned op_mask, const rbf_options* opt, double* w,
                                          int8_t* status) {
    if (!ctx || !X || !offsets || !idx || !w || N < 1 || nnz < 1) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    unsigned opc;
    const int R = op_slots(op_mask, d, &opc);
    if (R < 0) return RBF_EINVAL;
    if (degree_max < 0 || degree_max > 4 || n_max < 1) return RBF_EINVAL;
    if (n_max > N) return RBF_ETOOFEW;
    rbf_options o;
    rbf_options_default(&o);
    if (opt) o = *opt;
    if (o.phs_power != 3 && o.phs_power != 5) return RBF_EINVAL;
    if (o.precision != RBF_PREC_F64 && o.precision != RBF_PREC_F32_IR) return RBF_EINVAL;
    if (o.precision == RBF_PREC_F32_IR && !status) return RBF_EINVAL;  // the fallback list lives in status
    if (o.max_refine < 0 || o.scale_mode < 0 || o.scale_mode > 1 || !(o.refine_tol >= 0.0)) return RBF_EINVAL;
    const int m = n_mono(d, degree_max);
    const rbf::ClassEntry* c = rbf::find_class(n_max + m);
    if (!c) return RBF_EUNSUPPORTED;
    // the refined form exists for every class up to rbf::PAIR_MAXM unknowns; larger
    // systems are solved in float64
    const int prec = (c->maxm > rbf::PAIR_MAXM) ? RBF_PREC_F64 : o.precision;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    rbf::StencilArgs a;
    a.X = X;
    a.N = N;
    a.d = d;
    a.P = degree_max;
    a.degree = degree;
    a.offsets = offsets;
    a.idx = idx;
    a.nnz = nnz;
    a.n_max = n_max;
    a.op_mask = (1u << R) - 1u;
    a.opc = opc;
    a.phs_power = o.phs_power;
    a.scale_mode = o.scale_mode;
    a.repro_tol = o.repro_tol;
    a.w = w;
    a.status = status;
    if (c->fn(a, N, prec, o.max_refine, o.refine_tol, ctx->stream) != hipSuccess) return RBF_EHIP;
    if (prec != o.precision) {
        // mark every valid stencil of the float64 solve as FALLBACK (float64 used)
        hipLaunchKernelGGL(k_mark_fallback, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, ctx->stream, status, N);
        RBF_LAUNCH_CHECK();
    }
    return RBF_OK;
}
