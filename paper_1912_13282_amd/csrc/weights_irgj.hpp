// Mixed-precision RBF-FD weights, one stencil per wavefront: float32
// Gauss-Jordan with partial pivoting, float64 residuals and iterative refinement.
//
// The float32 elimination keeps each row's multipliers in the columns it has
// eliminated, so a correction K d = r is one replay of the recorded row
// operations on r (a sequence of broadcast + FMA per pivot) followed by the
// diagonal scaling.  The residual r = B - K x is formed in float64 with K
// recomputed from the scaled offsets (kept in LDS since assembly): FP64 is used
// only for the residual, the accumulated solution and the reproduction check.
// Acceptance: every right-hand side satisfies
//     max|r| <= tol * ||K||_inf * max|x|,   tol = max(sqrt(M) 2^-53, refine_tol)
// after at least one correction; otherwise the stencil is marked FALLBACK.
#pragma once

#include "weights_gj.hpp"

namespace rbf {

template <int D, int P, int MAXM>
struct IrLds {
    using G = GjLds<D, P, MAXM>;
    static constexpr int NR = 1 + D;
    static constexpr int QT = G::QT + (G::QT & 1);   // Q^T (kept for the residuals)
    static constexpr int XH = G::XH;                  // scaled offsets (kept)
    static constexpr int X64 = MAXM * NR;             // float64 solution broadcast
    static constexpr int PRWF = ((MAXM + NR + 3) / 4) * 4 + 4;   // float pivot row (see gauss_jordan)
    static constexpr int F32 = 2 * PRWF + MAXM * NR;            // two float pivot rows + float solution
    static constexpr int TOTAL = QT + XH + X64 + (F32 + 1) / 2;  // in doubles
};

// Replay of the recorded float32 elimination on the right-hand sides b (one per
// row lane): returns the solution component of unknown `step` in this lane.
template <int NR, int MAXM>
__device__ __forceinline__ void gj_replay(const float (&row)[MAXM], float (&b)[NR], int mystep, float invd) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        const int p = first_lane(__ballot(mystep == k));
        const float l = (lane == p) ? 0.0f : row[k];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const float y = readlane_f(b[q], p);
            b[q] = fmaf(-l, y, b[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) b[q] *= invd;
}

template <int D, int P, int MAXM>
__device__ __forceinline__ void stencil_ir_gj(const StencilArgs& a, int64_t node, double* lds, int max_refine,
                                              double refine_tol) {
    static_assert(MAXM <= 64, "one row per lane");
    using L = IrLds<D, P, MAXM>;
    using G = GjLds<D, P, MAXM>;
    constexpr int m = n_mono(D, P);
    constexpr int NR = 1 + D;
    constexpr int QW = MAXM - m;
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
    double* qt = lds;                 // m * QW
    double* xh = lds + L::QT;         // QW * 4
    double* x64 = xh + L::XH;         // MAXM * NR
    float* f32 = reinterpret_cast<float*>(x64 + L::X64);
    float* prow = f32;
    float* sol32 = f32 + 2 * L::PRWF;

    // assemble (entries computed in float64, rounded once); Q^T and the scaled
    // offsets stay in LDS for the float64 residuals
    double B[NR];
    float row[MAXM];
    static_assert(G::A >= G::QT, "layout");
    assemble_rows_lds<D, P, MAXM, float>(F, n, a.phs_power, lds, row, B);
    if (G::A != L::QT) {
        // move the offsets from the assembly layout to this one (only the n used entries)
        wave_lds_sync();
        double2 t0 = make_double2(0, 0), t1 = make_double2(0, 0);
        const int j = lane - m;
        if (j >= 0 && j < n) {
            t0 = *reinterpret_cast<const double2*>(lds + G::A + 4 * j);
            t1 = *reinterpret_cast<const double2*>(lds + G::A + 4 * j + 2);
        }
        wave_lds_sync();
        if (j >= 0 && j < n) {
            *reinterpret_cast<double2*>(xh + 4 * j) = t0;
            *reinterpret_cast<double2*>(xh + 4 * j + 2) = t1;
        }
    }
    float b32[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) b32[q] = (float)B[q];

    float s32[NR];
    int mystep;
    float invd;
    const bool ok32 = gauss_jordan<float, NR, MAXM>(row, b32, prow, sol32, s32, true, mystep, invd);

    bool accepted = false;
    double x[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) x[q] = (double)s32[q];
    if (ok32) {
        const double tolc0 = sqrt((double)M) * 0x1p-53;
        const double tolc = refine_tol > tolc0 ? refine_tol : tolc0;
        double knorm = 0.0;
        for (int it = 0; it <= max_refine; ++it) {
            // broadcast x (unknown r lives in lane r) through LDS
            if (lane < MAXM)
#pragma unroll
                for (int q = 0; q < NR; ++q) x64[lane * NR + q] = x[q];
            wave_lds_sync();
            // r = B - K x in float64, K recomputed for this lane's row
            double r[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) r[q] = B[q];
            double rowabs = 0.0;
            const int j = lane - m;
            const bool wrow = (j >= 0 && j < n);
            if (wrow) {
                // Q row of this node: column j of Q^T, kept in LDS since assembly
#pragma unroll 4
                for (int c = 0; c < m; ++c) {
                    const double qv = qt[c * QW + j];
#pragma unroll
                    for (int q = 0; q < NR; ++q) r[q] = fma(-qv, x64[c * NR + q], r[q]);
                    rowabs += fabs(qv);
                }
            }
#pragma unroll 2
            for (int c = m; c < MAXM; ++c) {
                const int k = c - m;
                double kv;
                if (wrow) {
                    const double2 p01 = *reinterpret_cast<const double2*>(xh + 4 * k);
                    const double2 p2 = *reinterpret_cast<const double2*>(xh + 4 * k + 2);
                    const double dx = F.xh[0][0] - p01.x, dy = F.xh[0][1] - p01.y;
                    double r2 = dx * dx + dy * dy;
                    if (D == 3) {
                        const double dz = F.xh[0][2] - p2.x;
                        r2 += dz * dz;
                    }
                    kv = (k < n) ? phs_from_r2(r2, a.phs_power) : 0.0;
                } else if (lane < m) {
                    kv = (k < n) ? qt[lane * QW + k] : 0.0;
                } else {
                    kv = 0.0;  // padding rows are never part of the residual
                }
#pragma unroll
                for (int q = 0; q < NR; ++q) r[q] = fma(-kv, x64[c * NR + q], r[q]);
                rowabs += fabs(kv);
            }
            const bool live = lane < M;
            if (it == 0) knorm = wave_max_dpp_d(live ? rowabs : 0.0);
            if (it >= 1) {
                bool conv = true;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const double rn = wave_max_dpp_d(live ? fabs(r[q]) : 0.0);
                    const double xn = wave_max_dpp_d(live ? fabs(x[q]) : 0.0);
                    conv = conv && (rn <= tolc * knorm * xn);
                }
                if (conv) {
                    accepted = true;
                    break;
                }
            }
            if (it == max_refine) break;
            // correction: replay the float32 elimination on r, then permute to unknown order
            float rb[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q) rb[q] = live ? (float)r[q] : 0.0f;
            gj_replay<NR, MAXM>(row, rb, mystep, invd);
            wave_lds_sync();
            if (mystep >= 0)
#pragma unroll
                for (int q = 0; q < NR; ++q) sol32[mystep * NR + q] = rb[q];
            wave_lds_sync();
            if (lane < MAXM)
#pragma unroll
                for (int q = 0; q < NR; ++q) x[q] += (double)sol32[lane * NR + q];
            wave_lds_sync();
        }
    }
    double sol[1][NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) sol[0][q] = x[q];
    if (accepted) accepted = repro_ok<D, P, MAXM>(a, n, F, sol);
    if (!accepted) {
        if (a.status && lane == 0) a.status[node] = (int8_t)RBF_ST_FALLBACK;
        return;
    }
    check_and_store<D, P, MAXM>(a, node, off, n, F, sol, true, (int8_t)RBF_ST_REFINED);
}

}  // namespace rbf
