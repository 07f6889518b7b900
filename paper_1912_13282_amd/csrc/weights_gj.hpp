// FP64 RBF-FD weights, one stencil per wavefront, Gauss-Jordan elimination with
// partial pivoting (the LU of the paper's solver continued upwards, which costs
// nothing extra when every lane holds one row and leaves no back substitution).
//
// Data movement per elimination step: the pivot search is a DPP reduction, the
// pivot row is stored to LDS by its lane and read back by every lane as
// broadcast 16-byte loads (the LDS pipe runs beside the FP64 FMAs).
#pragma once

#include "weights_f64.hpp"

namespace rbf {

// 1/x from the hardware reciprocal estimate refined by Newton steps
// (e' = e (2 - x e)); two steps for float64, one for float32.
__device__ __forceinline__ double recip(double x) {
    double e = __builtin_amdgcn_rcp(x);
    e = fma(e, fma(-x, e, 1.0), e);
    e = fma(e, fma(-x, e, 1.0), e);
    return e;
}
__device__ __forceinline__ float recip(float x) {
    float e = __builtin_amdgcn_rcpf(x);
    return fmaf(e, fmaf(-x, e, 1.0f), e);
}

template <int D, int P, int MAXM>
struct GjLds {
    static constexpr int m = n_mono(D, P);
    static constexpr int NR = 1 + D;
    static constexpr int QW = MAXM - m;
    static constexpr int QT = m * QW;          // Q^T of the polynomial rows (assembly)
    static constexpr int SOL = MAXM * NR;      // solution, permuted to unknown order (end)
    static constexpr int A = ((QT > SOL ? QT : SOL) + 1) & ~1;   // even: keeps 16-byte alignment
    static constexpr int XH = QW * 4;          // scaled offsets, padded to 4 doubles
    static constexpr int PRW = ((MAXM + NR + 1) / 2) * 2 + 2;  // one pivot row + RHS (see gauss_jordan)
    static constexpr int TOTAL = A + XH + 2 * PRW;
};

template <int D, int P, int MAXM, typename T>
__device__ __forceinline__ void assemble_rows_lds(const Frame<D, P, MAXM>& F, int n, int kpow, double* lds,
                                                  T (&row)[MAXM], double (&rhs)[1 + D]) {
    using L = GjLds<D, P, MAXM>;
    constexpr int m = L::m;
    constexpr int NR = L::NR;
    constexpr int QW = L::QW;
    constexpr Mono<D, P> MO{};
    double* qt = lds;
    double* xh = lds + L::A;
    const int r = lane_id();
    const int j = r - m;
    const bool wrow = (j >= 0 && j < n);
    {
        double q[m];
        monomials<D, P>(F.xh[0], q);
#pragma unroll
        for (int c = 0; c < m; ++c) {
            row[c] = (T)(wrow ? q[c] : 0.0);
            if (wrow) qt[c * QW + j] = q[c];
        }
        if (wrow) {
            *reinterpret_cast<double2*>(xh + 4 * j) = make_double2(F.xh[0][0], F.xh[0][1]);
            *reinterpret_cast<double2*>(xh + 4 * j + 2) = make_double2(F.xh[0][2], 0.0);
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int c = m; c < MAXM; ++c) {
        const int k = c - m;
        const double2 p01 = *reinterpret_cast<const double2*>(xh + 4 * k);
        const double2 p2 = *reinterpret_cast<const double2*>(xh + 4 * k + 2);
        double v;
        if (wrow) {
            const double dx = F.xh[0][0] - p01.x, dy = F.xh[0][1] - p01.y;
            double r2 = dx * dx + dy * dy;
            if (D == 3) {
                const double dz = F.xh[0][2] - p2.x;
                r2 += dz * dz;
            }
            v = (k < n) ? phs_from_r2(r2, kpow) : 0.0;
        } else if (r < m) {
            v = (k < n) ? qt[r * QW + k] : 0.0;
        } else {
            v = (r == c) ? 1.0 : 0.0;
        }
        row[c] = (T)v;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) rhs[q] = 0.0;
    if (wrow) {
        const double r2 = F.xh[0][0] * F.xh[0][0] + F.xh[0][1] * F.xh[0][1] + F.xh[0][2] * F.xh[0][2];
        const double rr = sqrt(r2);
        const double pw = (kpow == 5) ? r2 * rr : rr;
        rhs[0] = (double)(kpow * (kpow + D - 2)) * pw;
#pragma unroll
        for (int q = 1; q < NR; ++q) rhs[q] = -(double)kpow * pw * F.xh[0][q - 1];
    } else if (r < m) {
#pragma unroll
        for (int l = 0; l < m; ++l)
            if (r == l) {
#pragma unroll
                for (int q = 0; q < NR; ++q) rhs[q] = MO.lq(l, q);
            }
    }
}

// Gauss-Jordan with partial pivoting on the rows held in registers (one row per
// lane, MAXM <= 64).  All MAXM steps run without branches: padding rows are
// identity rows, so steps k >= M pivot on them and change nothing; a zero or
// non-finite pivot is recorded and reported at the end.  On success x[q] of the
// lane holding unknown r (= row r) is returned through LDS in sol[q].
template <typename T, int NR, int MAXM>
__device__ __forceinline__ bool gauss_jordan(T (&row)[MAXM], T (&rhs)[NR], T* prow, T* sol_lds, T (&sol)[NR],
                                             bool keep_multipliers, int (&step_out), T (&invd_out)) {
    constexpr int V = 16 / sizeof(T);                       // values per 16-byte LDS access
    constexpr int PRW = ((MAXM + NR + V - 1) / V) * V + V;  // one pivot row + RHS, padded
    constexpr int RO = ((MAXM + V - 1) / V) * V;            // RHS offset inside a row buffer
    using V2 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    const int lane = lane_id();
    bool piv = lane >= MAXM;
    int mystep = -1;
    T invd = (T)0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        // pivot search on float magnitudes (partial pivoting needs a large pivot,
        // not the exact maximum); the first lane with the maximum wins
        const float cand = piv ? -1.0f : (float)fabs(row[k]);
        const float mx = wave_max_dpp_f(cand);
        bad = bad || !(mx > 0.0f) || !__builtin_isfinite(mx);
        const uint64_t b = __ballot(!piv && cand == mx);
        const int p = first_lane(b);
        T* buf = static_cast<T*>(__builtin_assume_aligned(prow + (k & 1) * PRW, 16));
        const bool me = (lane == p);
        if (me) {
            piv = true;
            mystep = k;
#pragma unroll
            for (int j = k; j < MAXM; ++j) buf[j] = row[j];
#pragma unroll
            for (int q = 0; q < NR; ++q) buf[RO + q] = rhs[q];
        }
        wave_lds_sync();
        const T inv = recip(buf[k]);
        if (me) invd = inv;
        const T l = me ? (T)0 : row[k] * inv;
        if (keep_multipliers && !me) row[k] = l;
#pragma unroll
        for (int j0 = ((k + 1) / V) * V; j0 < MAXM; j0 += V) {
            const V2 uv = *reinterpret_cast<const V2*>(buf + j0);
            const T* u = reinterpret_cast<const T*>(&uv);
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (j0 + e > k && j0 + e < MAXM) row[j0 + e] = fma(-l, u[e], row[j0 + e]);
        }
#pragma unroll
        for (int q0 = 0; q0 < NR; q0 += V) {
            const V2 uv = *reinterpret_cast<const V2*>(buf + RO + q0);
            const T* u = reinterpret_cast<const T*>(&uv);
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (q0 + e < NR) rhs[q0 + e] = fma(-l, u[e], rhs[q0 + e]);
        }
    }
    step_out = mystep;
    invd_out = invd;
    if (mystep >= 0)
#pragma unroll
        for (int q = 0; q < NR; ++q) sol_lds[mystep * NR + q] = rhs[q] * invd;
    wave_lds_sync();
    if (lane < MAXM)
#pragma unroll
        for (int q = 0; q < NR; ++q) sol[q] = sol_lds[lane * NR + q];
    return __ballot(bad) == 0;
}

template <int D, int P, int MAXM>
__device__ __forceinline__ void stencil_f64_gj(const StencilArgs& a, int64_t node, double* lds) {
    static_assert(MAXM <= 64, "one row per lane");
    using L = GjLds<D, P, MAXM>;
    constexpr int m = L::m;
    constexpr int NR = L::NR;
    const int64_t off = a.offsets[node];
    const int64_t n64 = a.offsets[node + 1] - off;
    if (n64 < 1 || n64 > a.n_max || n64 + m > MAXM) {
        reject_stencil(a, node, off, n64 < 0 ? 0 : n64, RBF_ST_BADSIZE);
        return;
    }
    const int n = (int)n64;
    Frame<D, P, MAXM> F;
    if (!load_frame<D, P, MAXM>(a, off, n, F)) {
        reject_stencil(a, node, off, n, RBF_ST_BADSIZE);
        return;
    }
    double row[MAXM];
    double rhs[NR];
    assemble_rows_lds<D, P, MAXM, double>(F, n, a.phs_power, lds, row, rhs);
    double s1[NR];
    int mystep;
    double invd;
    const bool ok = gauss_jordan<double, NR, MAXM>(row, rhs, lds + L::A + L::XH, lds, s1, false, mystep, invd);
    double sol[1][NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) sol[0][q] = ok ? s1[q] : 0.0;
    check_and_store<D, P, MAXM>(a, node, off, n, F, sol, ok, (int8_t)RBF_ST_OK);
}

}  // namespace rbf
