// Mixed-precision RBF-FD weights: float32 LU of the augmented system with
// float64 residuals and iterative refinement (stopping test of LAPACK dsgesv).
// FP64 is used only for the assembled matrix, the residuals, the accumulated
// solution and the reproduction check.  A stencil that is not accepted after
// max_refine corrections gets status FALLBACK and is recomputed by the FP64 path.
#pragma once

#include "weights_f64.hpp"

namespace rbf {

// Reproduction check only (no store); see check_and_store.
template <int D, int P, int MAXM>
__device__ __forceinline__ bool repro_ok(const StencilArgs& a, int n, const Frame<D, P, MAXM>& F,
                                         const double (&sol)[(MAXM + 63) / 64][1 + D]) {
    constexpr int m = n_mono(D, P);
    constexpr int RPL = (MAXM + 63) / 64;
    constexpr int NR = 1 + D;
    constexpr Mono<D, P> MO{};
    const int lane = lane_id();
    double S[NR], A[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) S[q] = A[q] = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int j = lane + 64 * t - m;
        if (j >= 0 && j < n) {
            double qv[m];
            monomials<D, P>(F.xh[t], qv);
            double pv = 0.0;
#pragma unroll
            for (int l = 0; l < m; ++l) pv += check_coef(l) * qv[l];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                double v = sol[t][q] * pv;
                S[q] += v;
                A[q] += fabs(v);
            }
        }
    }
    bool ok = true;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (!(a.op_mask & (1u << q))) continue;
        double s = wave_sum_dpp_d(S[q]);
        double ab = wave_sum_dpp_d(A[q]);
        double lp = 0.0;
#pragma unroll
        for (int l = 0; l < m; ++l) lp += check_coef(l) * MO.lq(l, q);
        ok = ok && (fabs(s - lp) / (ab + fabs(lp)) <= a.repro_tol);
    }
    return ok;
}

// Forward substitution with the unit-lower factor kept in row[t][k] (k < step[t]).
template <int NR, int MAXM>
__device__ __forceinline__ void forward_l(int M, const float (&row)[(MAXM + 63) / 64][MAXM],
                                          float (&b)[(MAXM + 63) / 64][NR], const int (&step)[(MAXM + 63) / 64]) {
    constexpr int RPL = (MAXM + 63) / 64;
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        if (k < M) {
            int p = 0, ps = 0;
            uint64_t b0 = __ballot(step[0] == k);
            if (b0) {
                p = first_lane(b0);
            } else if constexpr (RPL == 2) {
                p = first_lane(__ballot(step[RPL - 1] == k));
                ps = 1;
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const float y = readlane_f(ps == 0 ? b[0][q] : b[RPL - 1][q], p);
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const float l = (step[t] > k) ? row[t][k] : 0.0f;
                    b[t][q] = fmaf(-l, y, b[t][q]);
                }
            }
        }
    }
}

// Back substitution with the upper factor (columns > step[t] of row[t]).
template <int NR, int MAXM>
__device__ __forceinline__ void backward_u(int M, const float (&row)[(MAXM + 63) / 64][MAXM],
                                           float (&b)[(MAXM + 63) / 64][NR], const int (&step)[(MAXM + 63) / 64],
                                           const float (&invd)[(MAXM + 63) / 64], float (&x)[(MAXM + 63) / 64][NR]) {
    constexpr int RPL = (MAXM + 63) / 64;
    const int lane = lane_id();
#pragma unroll
    for (int t = 0; t < RPL; ++t)
#pragma unroll
        for (int q = 0; q < NR; ++q) x[t][q] = 0.0f;
#pragma unroll
    for (int k = MAXM - 1; k >= 0; --k) {
        if (k < M) {
            int p = 0, ps = 0;
            uint64_t b0 = __ballot(step[0] == k);
            if (b0) {
                p = first_lane(b0);
            } else if constexpr (RPL == 2) {
                p = first_lane(__ballot(step[RPL - 1] == k));
                ps = 1;
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const float y = (ps == 0) ? b[0][q] * invd[0] : b[RPL - 1][q] * invd[RPL - 1];
                const float xv = readlane_f(y, p);
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const float u = (step[t] < k && step[t] >= 0) ? row[t][k] : 0.0f;
                    b[t][q] = fmaf(-u, xv, b[t][q]);
                }
                if (lane == (k & 63)) x[k >> 6][q] = xv;
            }
        }
    }
}

template <int D, int P, int MAXM>
__device__ __forceinline__ void stencil_ir(const StencilArgs& a, int64_t node, double* qt, int max_refine) {
    if constexpr (MAXM > 64) {
        // not instantiated: the launcher sends n + m > 64 to the FP64 kernel
        return;
    } else {
    constexpr int m = n_mono(D, P);
    constexpr int RPL = (MAXM + 63) / 64;
    constexpr int NR = 1 + D;
    const int lane = lane_id();
    const int64_t off = a.offsets[node];
    const int64_t n64 = a.offsets[node + 1] - off;
    if (n64 < 1 || n64 > a.n_max || n64 + m > MAXM) {
        reject_stencil(a, node, off, n64 < 0 ? 0 : n64, RBF_ST_BADSIZE);
        return;
    }
    const int n = (int)n64;
    const int M = n + m;
    Frame<D, P, MAXM> F;
    if (!load_frame<D, P, MAXM>(a, off, n, F)) {
        reject_stencil(a, node, off, n, RBF_ST_BADSIZE);
        return;
    }
    double K[RPL][MAXM];
    double B[RPL][NR];
    assemble_rows<D, P, MAXM>(F, n, a.phs_power, qt, K, B);

    // ||K||_inf
    double rs = 0.0;
#pragma unroll
    for (int c = 0; c < MAXM; ++c) rs += fabs(K[0][c]);
    const int r0 = lane;
    const double knorm = wave_max_d((r0 < M) ? rs : 0.0);

    float L[RPL][MAXM];
    float b[RPL][NR];
#pragma unroll
    for (int c = 0; c < MAXM; ++c) L[0][c] = (float)K[0][c];
#pragma unroll
    for (int q = 0; q < NR; ++q) b[0][q] = (float)B[0][q];
    int step[RPL];
    float invd[RPL];
    bool ok = lu_rows<float, NR, MAXM>(M, L, b, step, invd, true);
    bool accepted = false;
    double x[RPL][NR];
    if (ok) {
        float xs[RPL][NR];
        backward_u<NR, MAXM>(M, L, b, step, invd, xs);
#pragma unroll
        for (int q = 0; q < NR; ++q) x[0][q] = (double)xs[0][q];
        const double tolc = sqrt((double)M) * 0x1p-53 * knorm;
        for (int it = 0; it <= max_refine; ++it) {
            // r = B - K x in float64 (x of unknown c lives in lane c)
            double r[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) r[q] = B[0][q];
#pragma unroll
            for (int c = 0; c < MAXM; ++c) {
                if (c < M) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) r[q] = fma(-K[0][c], readlane_d(x[0][q], c), r[q]);
                }
            }
            if (it >= 1) {
                bool conv = true;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const double rn = wave_max_d((r0 < M) ? fabs(r[q]) : 0.0);
                    const double xn = wave_max_d((r0 < M) ? fabs(x[0][q]) : 0.0);
                    conv = conv && (rn <= tolc * xn);
                }
                if (conv) {
                    accepted = true;
                    break;
                }
            }
            if (it == max_refine) break;
            float rb[RPL][NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) rb[0][q] = (float)r[q];
            forward_l<NR, MAXM>(M, L, rb, step);
            float dx[RPL][NR];
            backward_u<NR, MAXM>(M, L, rb, step, invd, dx);
#pragma unroll
            for (int q = 0; q < NR; ++q) x[0][q] += (double)dx[0][q];
        }
    }
    if (accepted) accepted = repro_ok<D, P, MAXM>(a, n, F, x);
    if (!accepted) {
        if (a.status && lane == 0) a.status[node] = (int8_t)RBF_ST_FALLBACK;
        return;
    }
    check_and_store<D, P, MAXM>(a, node, off, n, F, x, true, (int8_t)RBF_ST_REFINED);
    }
}

}  // namespace rbf
