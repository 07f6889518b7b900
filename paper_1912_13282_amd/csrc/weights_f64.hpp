// Plain FP64 RBF-FD weights of one stencil per wavefront (LU with partial pivoting).
#pragma once

#include "weights_core.hpp"

namespace rbf {

// Assemble the rows of K' held by this lane (see weights_core.hpp) in float64.
// row[t][c] is column c of row r = lane + 64 t; rhs[t][q] the q-th operator's
// right-hand side (q = 0: Laplacian, q = 1..D: d/dx_q).  qt is this wave's LDS
// scratch of m * (MAXM - m) doubles (Q transposed for the polynomial rows).
template <int D, int P, int MAXM>
__device__ __forceinline__ void assemble_rows(const Frame<D, P, MAXM>& F, int n, int kpow, double* qt,
                                              double (&row)[(MAXM + 63) / 64][MAXM],
                                              double (&rhs)[(MAXM + 63) / 64][1 + D]) {
    constexpr int m = n_mono(D, P);
    constexpr int RPL = (MAXM + 63) / 64;
    constexpr int NR = 1 + D;
    constexpr int QW = MAXM - m;
    constexpr Mono<D, P> MO{};
    const int lane = lane_id();
    const int M = n + m;

    // polynomial columns (c < m) of the weight rows, and Q^T into LDS
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        const int j = r - m;
        double q[m];
        monomials<D, P>(F.xh[t], q);
        const bool wrow = (j >= 0 && j < n);
#pragma unroll
        for (int c = 0; c < m; ++c) {
            row[t][c] = wrow ? q[c] : 0.0;
            if (wrow) qt[c * QW + j] = q[c];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // RBF columns c = m + k: A for weight rows, Q^T for polynomial rows, identity for padding
#pragma unroll
    for (int c = m; c < MAXM; ++c) {
        const int k = c - m;
        double xk[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) xk[q] = (q < D) ? readlane_d(F.xh[c >> 6][q], c & 63) : 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int r = lane + 64 * t;
            const int j = r - m;
            double v;
            if (j >= 0 && j < n) {
                double dx = F.xh[t][0] - xk[0], dy = F.xh[t][1] - xk[1];
                double r2 = dx * dx + dy * dy;
                if (D == 3) {
                    double dz = F.xh[t][2] - xk[2];
                    r2 += dz * dz;
                }
                v = (k < n) ? phs_from_r2(r2, kpow) : 0.0;
            } else if (r < m) {
                v = (k < n) ? qt[r * QW + k] : 0.0;
            } else {
                v = (r == c) ? 1.0 : 0.0;  // padding row (or a row beyond MAXM: never read)
            }
            row[t][c] = v;
        }
    }

    // right-hand sides
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        const int j = r - m;
#pragma unroll
        for (int q = 0; q < NR; ++q) rhs[t][q] = 0.0;
        if (j >= 0 && j < n) {
            double r2 = F.xh[t][0] * F.xh[t][0] + F.xh[t][1] * F.xh[t][1] + F.xh[t][2] * F.xh[t][2];
            double rr = sqrt(r2);
            double pw = (kpow == 5) ? r2 * rr : rr;  // ||x_j||^(k-2)
            rhs[t][0] = (double)(kpow * (kpow + D - 2)) * pw;
#pragma unroll
            for (int q = 1; q < NR; ++q) rhs[t][q] = -(double)kpow * pw * F.xh[t][q - 1];
        } else if (r < m) {
#pragma unroll
            for (int l = 0; l < m; ++l)
                if (r == l) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) rhs[t][q] = MO.lq(l, q);
                }
        }
    }
    (void)M;
}

// FP64 reproduction check of the weights held by this lane's weight rows and the
// output write.  sol[t][q] is the solution component of unknown r = lane + 64 t.
template <int D, int P, int MAXM>
__device__ __forceinline__ void check_and_store(const StencilArgs& a, int64_t node, int64_t off, int n,
                                                const Frame<D, P, MAXM>& F, double (&sol)[(MAXM + 63) / 64][1 + D],
                                                bool ok, int8_t good_status) {
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
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (!(a.op_mask & (1u << q))) continue;
        double s = wave_sum_dpp_d(S[q]);
        double ab = wave_sum_dpp_d(A[q]);
        double lp = 0.0;
#pragma unroll
        for (int l = 0; l < m; ++l) lp += check_coef(l) * MO.lq(l, q);
        double rho = fabs(s - lp) / (ab + fabs(lp));
        ok = ok && (rho <= a.repro_tol);
    }
    const double sc2 = F.inv_s * F.inv_s;
    int ro = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (!(a.op_mask & (1u << q))) continue;
        const double sc = (q == 0) ? sc2 : F.inv_s;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int j = lane + 64 * t - m;
            if (j >= 0 && j < n) a.w[ro * a.nnz + off + j] = ok ? sol[t][q] * sc : __builtin_nan("");
        }
        ++ro;
    }
    if (a.status && lane == 0) a.status[node] = ok ? good_status : (int8_t)RBF_ST_SINGULAR;
}

// LU with partial pivoting of the rows held in registers, eliminating the
// right-hand sides alongside; returns false on a zero / non-finite pivot.
// On return row[t][*] holds row r's U entries (columns >= its pivot step, zeros
// at earlier pivot columns), step[t] its pivot step and invd[t] 1/U_kk.
template <typename T, int NR, int MAXM>
__device__ __forceinline__ bool lu_rows(int M, T (&row)[(MAXM + 63) / 64][MAXM], T (&rhs)[(MAXM + 63) / 64][NR],
                                        int (&step)[(MAXM + 63) / 64], T (&invd)[(MAXM + 63) / 64],
                                        bool keep_l) {
    constexpr int RPL = (MAXM + 63) / 64;
    const int lane = lane_id();
    bool piv[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int r = lane + 64 * t;
        piv[t] = (r >= MAXM);
        step[t] = -1;
        invd[t] = (T)0;
    }
    bool ok = true;
    // every loop below has a constant trip count (bodies are guarded instead of
    // leaving early) so that full unrolling keeps row[][] in registers
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        if (ok && k < M) {
            T best = (T)-1;
#pragma unroll
            for (int t = 0; t < RPL; ++t)
                if (!piv[t]) best = fmax(best, (T)fabs(row[t][k]));
            T mx;
            if constexpr (sizeof(T) == 8) mx = wave_max_d(best);
            else mx = wave_max_f(best);
            if (!(mx > (T)0) || !(mx < (T)INFINITY)) {
                ok = false;
            } else {
                int p = 0, ps = 0;
                uint64_t b0 = __ballot(!piv[0] && fabs(row[0][k]) == mx);
                if (b0) {
                    p = first_lane(b0);
                } else if constexpr (RPL == 2) {
                    uint64_t b1 = __ballot(!piv[RPL - 1] && fabs(row[RPL - 1][k]) == mx);
                    p = first_lane(b1);
                    ps = 1;
                }
                const T pv = readlane_t<T>(ps == 0 ? row[0][k] : row[RPL - 1][k], p);
                const T inv = (T)1 / pv;
                T l[RPL];
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    if (lane == p && t == ps) {
                        piv[t] = true;
                        step[t] = k;
                        invd[t] = inv;
                    }
                    l[t] = piv[t] ? (T)0 : row[t][k] * inv;
                    if (!piv[t]) row[t][k] = keep_l ? l[t] : (T)0;
                }
#pragma unroll
                for (int j = k + 1; j < MAXM; ++j) {
                    if (j < M) {
                        const T u = readlane_t<T>(ps == 0 ? row[0][j] : row[RPL - 1][j], p);
#pragma unroll
                        for (int t = 0; t < RPL; ++t) row[t][j] = fma(-l[t], u, row[t][j]);
                    }
                }
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const T u = readlane_t<T>(ps == 0 ? rhs[0][q] : rhs[RPL - 1][q], p);
#pragma unroll
                    for (int t = 0; t < RPL; ++t) rhs[t][q] = fma(-l[t], u, rhs[t][q]);
                }
            }
        }
    }
    return ok;
}

// Back substitution U x = y (y in rhs, consumed).  sol[t][q] receives x of
// unknown r = lane + 64 t.  Rows with step > k must hold 0 at column k.
template <typename T, int NR, int MAXM>
__device__ __forceinline__ void back_substitute(int M, const T (&row)[(MAXM + 63) / 64][MAXM],
                                                T (&rhs)[(MAXM + 63) / 64][NR], const int (&step)[(MAXM + 63) / 64],
                                                const T (&invd)[(MAXM + 63) / 64], T (&sol)[(MAXM + 63) / 64][NR]) {
    constexpr int RPL = (MAXM + 63) / 64;
    const int lane = lane_id();
#pragma unroll
    for (int t = 0; t < RPL; ++t)
#pragma unroll
        for (int q = 0; q < NR; ++q) sol[t][q] = (T)0;
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
                const T y = (ps == 0) ? rhs[0][q] * invd[0] : rhs[RPL - 1][q] * invd[RPL - 1];
                const T x = readlane_t<T>(y, p);
#pragma unroll
                for (int t = 0; t < RPL; ++t) rhs[t][q] = fma(-row[t][k], x, rhs[t][q]);
                if (lane == (k & 63)) sol[k >> 6][q] = x;
            }
        }
    }
}

template <int D, int P, int MAXM>
__device__ __forceinline__ void stencil_f64(const StencilArgs& a, int64_t node, double* qt) {
    constexpr int m = n_mono(D, P);
    constexpr int RPL = (MAXM + 63) / 64;
    constexpr int NR = 1 + D;
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
    double row[RPL][MAXM];
    double rhs[RPL][NR];
    assemble_rows<D, P, MAXM>(F, n, a.phs_power, qt, row, rhs);
    int step[RPL];
    double invd[RPL];
    bool ok = lu_rows<double, NR, MAXM>(M, row, rhs, step, invd, false);
    double sol[RPL][NR];
    if (ok) {
        back_substitute<double, NR, MAXM>(M, row, rhs, step, invd, sol);
    } else {
#pragma unroll
        for (int t = 0; t < RPL; ++t)
#pragma unroll
            for (int q = 0; q < NR; ++q) sol[t][q] = 0.0;
    }
    check_and_store<D, P, MAXM>(a, node, off, n, F, sol, ok, (int8_t)RBF_ST_OK);
}

}  // namespace rbf
