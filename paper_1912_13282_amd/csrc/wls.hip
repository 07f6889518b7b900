// Generalized weighted least squares weights (Sec. 2.2.1): one stencil per
// wavefront, stencil node j in lane j.
//
// With B the monomials of degree <= P at the scaled offsets and W the diagonal
// of weight-function values, the weights are w = W y with y the minimum-norm
// solution of (W B)^T y = (L b)(0), eq. (wbsys).  The kernel factors W B = Q R
// by Householder reflections (lane j holds row j of W B in registers; each
// reflection costs one wave reduction per remaining column), solves
// R^T z = (L b)(0) by forward substitution and forms y = Q [z; 0] by applying
// the reflections in reverse.  Every reduction is a fixed DPP butterfly, so
// the result does not depend on timing.  The weights then pass the same float64
// reproduction test as the RBF-FD weights (B^T w = (L b)(0) on a test
// polynomial) and are scaled back by s^-2 (Laplacian) or s^-1.
#include "wsolve.hpp"

using namespace rbf;

namespace {

// Reproduction test of the weights held by lane j (node j): the test polynomial
// of the RBF-FD check, sum_j w_j p(x_j) against (L p)(0), relative to sum |w_j p(x_j)|.
__device__ __forceinline__ bool wls_repro(const StencilArgs& a, int n, int m, const FrameG<1>& F,
                                          const double (&sol)[1][NR]) {
    const int lane = lane_id();
    double pv = 0.0;
    if (lane < n)
        for (int l = 0; l < m; ++l) pv += check_coef(l) * mono(a.d, l, F.xh[0]);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const double v = (lane < n) ? sol[0][q] * pv : 0.0;
        const double s = wave_sum_dpp_d(v);
        const double ab = wave_sum_dpp_d(fabs(v));
        if (!(a.op_mask & (1u << q))) continue;
        double lp = 0.0;
        for (int l = 0; l < m; ++l) lp += check_coef(l) * mono_lop(a.d, l, slot_op(a.opc, q));
        // multiplicative form: weights that are exactly zero (a Laplacian of degree <= 1) pass
        ok = ok && (fabs(s - lp) <= a.repro_tol * (ab + fabs(lp)));
    }
    return ok;
}

// per-wave LDS: the reflections' v_kk and beta and the diagonal R_kk (wave-uniform
// scalars; in registers they would take 6 MM VGPRs and halve the occupancy)
template <int MM>
struct WlsLds {
    double vkk[MM], bet[MM], rkk[MM];
};

template <int MM>
__device__ __forceinline__ void stencil_wls(const StencilArgs& a, int64_t node, int wkind, double inv_sigma2,
                                            WlsLds<MM>& L) {
    const int lane = lane_id();
    const int64_t off = a.offsets[node];
    const int64_t n64 = a.offsets[node + 1] - off;
    const int m = (a.P >= 0 && a.P <= 4) ? binom(a.P + a.d, a.d) : 1 << 20;
    if (n64 < 1 || n64 > a.n_max || n64 > WAVE || m > MM || off < 0 || off + n64 > a.nnz) {
        reject_stencil(a, node, off, (n64 < 0 || off < 0 || off + n64 > a.nnz) ? 0 : n64, RBF_ST_BADSIZE);
        return;
    }
    const int n = (int)n64;
    FrameG<1> F;
    if (!load_frame_g<1>(a, off, n, 0, F)) {  // lane j: node j
        reject_stencil(a, node, off, n, RBF_ST_BADSIZE);
        return;
    }
    const bool act = lane < n;
    const double r2 = F.xh[0][0] * F.xh[0][0] + F.xh[0][1] * F.xh[0][1] + F.xh[0][2] * F.xh[0][2];
    const double om = act ? (wkind == RBF_WLS_GAUSSIAN ? exp(-r2 * inv_sigma2) : 1.0) : 0.0;
    // row j of W B
    double A[MM];
#pragma unroll
    for (int l = 0; l < MM; ++l) A[l] = (act && l < m) ? om * mono(a.d, l, F.xh[0]) : 0.0;

    // Householder QR; reflection k: v = (0.., A_kk - alpha, A_{k+1,k}, ..), beta = 2 / v^T v
    double rmax = 0.0, rmin = INFINITY;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        if (k < m) {
            const double akk = readlane_d(A[k], k);
            const double sig = wave_sum_dpp_d(lane > k ? A[k] * A[k] : 0.0);
            const double nrm = sqrt(akk * akk + sig);
            const double alpha = akk > 0.0 ? -nrm : nrm;
            const double vk = akk - alpha;
            const double vtv = vk * vk + sig;
            const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
            const double vj = lane > k ? A[k] : (lane == k ? vk : 0.0);
#pragma unroll
            for (int c = k + 1; c < MM; ++c) {
                if (c < m) {
                    const double dot = wave_sum_dpp_d(vj * A[c]);
                    A[c] -= beta * dot * vj;
                }
            }
            if (lane == k) A[k] = alpha;  // R_kk; the lanes below keep v in column k
            if (lane == 0) {
                L.vkk[k] = vk;
                L.bet[k] = beta;
                L.rkk[k] = alpha;
            }
            rmax = fmax(rmax, fabs(alpha));
            rmin = fmin(rmin, fabs(alpha));
        }
    }
    wave_lds_sync();
    // full column rank: every |R_kk| above a relative floor (n >= m needed)
    const bool ok = n >= m && rmin > 1e-13 * rmax;

    // R^T z = (L b)(0) by forward substitution (z_k kept in lane k), then
    // y = Q [z; 0] by the reflections in reverse order; the operators advance
    // together so that their reduction chains overlap
    double zl[NR], y[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) zl[q] = 0.0;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        if (k < m) {
            const double rk = L.rkk[k];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (!(a.op_mask & (1u << q))) continue;
                const double acc = wave_sum_dpp_d(lane < k ? A[k] * zl[q] : 0.0);  // sum_{i<k} R_ik z_i
                const double zk = (mono_lop(a.d, k, slot_op(a.opc, q)) - acc) / rk;
                if (lane == k) zl[q] = zk;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) y[q] = lane < m ? zl[q] : 0.0;
#pragma unroll
    for (int k = MM - 1; k >= 0; --k) {
        if (k < m) {
            const double vj = lane > k ? A[k] : (lane == k ? L.vkk[k] : 0.0);
            const double bk = L.bet[k];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (!(a.op_mask & (1u << q))) continue;
                const double dot = wave_sum_dpp_d(vj * y[q]);
                y[q] -= bk * dot * vj;
            }
        }
    }
    double sol[1][NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) sol[0][q] = (ok && (a.op_mask & (1u << q))) ? om * y[q] : 0.0;
    const bool good = ok && wls_repro(a, n, m, F, sol);
    store_weights<1>(a, node, off, n, 0, F, sol, good, (int8_t)RBF_ST_OK);
}

template <int MM>
__global__ __launch_bounds__(256) void k_wls(StencilArgs a, int64_t N, int wkind, double inv_sigma2) {
    __shared__ WlsLds<MM> lds[4];
    const int wv = threadIdx.x / WAVE;
    const int64_t node = (int64_t)blockIdx.x * 4 + wv;
    if (node >= N) return;
    stencil_wls<MM>(a, node, wkind, inv_sigma2, lds[wv]);
}

}  // namespace

extern "C" rbf_status rbf_compute_weights_wls(rbf_ctx* ctx, const double* X, int64_t N, int d,
                                              const int64_t* offsets, const int32_t* idx, int64_t nnz, int n_max,
                                              int degree, unsigned op_mask, int weight_fn, double sigma,
                                              const rbf_options* opt, double* w, int8_t* status) {
    if (!ctx || !X || !offsets || !idx || !w || N < 1 || nnz < 1) return RBF_EINVAL;
    if (d != 2 && d != 3) return RBF_EDIM;
    unsigned opc;
    const int R = op_slots(op_mask, d, &opc);
    if (R < 0) return RBF_EINVAL;
    if (degree < 0 || degree > 4 || n_max < 1) return RBF_EINVAL;
    if (n_max > N) return RBF_ETOOFEW;
    if (n_max > WAVE) return RBF_EUNSUPPORTED;
    if (weight_fn != RBF_WLS_UNIT && weight_fn != RBF_WLS_GAUSSIAN) return RBF_EINVAL;
    if (weight_fn == RBF_WLS_GAUSSIAN && !(sigma > 0.0)) return RBF_EINVAL;
    rbf_options o;
    rbf_options_default(&o);
    if (opt) o = *opt;
    if (o.scale_mode < 0 || o.scale_mode > 1 || !(o.repro_tol > 0.0)) return RBF_EINVAL;
    RBF_HIP_CHECK(hipSetDevice(ctx->device));
    StencilArgs a;
    a.X = X;
    a.N = N;
    a.d = d;
    a.P = degree;
    a.offsets = offsets;
    a.idx = idx;
    a.nnz = nnz;
    a.n_max = n_max;
    a.op_mask = (1u << R) - 1u;
    a.opc = opc;
    a.phs_power = 3;  // unused by this engine
    a.scale_mode = o.scale_mode;
    a.repro_tol = o.repro_tol;
    a.w = w;
    a.status = status;
    const int m = n_mono(d, degree);
    const double is2 = weight_fn == RBF_WLS_GAUSSIAN ? 1.0 / (sigma * sigma) : 0.0;
    const dim3 grid((unsigned)((N + 3) / 4)), block(256);
    if (m <= 10)
        hipLaunchKernelGGL((k_wls<10>), grid, block, 0, ctx->stream, a, N, weight_fn, is2);
    else if (m <= 20)
        hipLaunchKernelGGL((k_wls<20>), grid, block, 0, ctx->stream, a, N, weight_fn, is2);
    else
        hipLaunchKernelGGL((k_wls<35>), grid, block, 0, ctx->stream, a, N, weight_fn, is2);
    RBF_LAUNCH_CHECK();
    return RBF_OK;
}
