// RBF-FD weights of one stencil per wavefront (gfx950): assembly of the
// augmented system of eq. (rbf-system-aug), LU with partial pivoting, back
// substitution, back-scaling and the FP64 reproduction check.
//
// Unknown / row order inside the kernel: the m polynomial multipliers first,
// then the n stencil weights, i.e. K' = [0 Q^T; Q A] acting on [lambda; w].
// This is the paper's K with rows and columns permuted alike (same solution);
// it puts the runtime-sized block last so every register index is static.
//
// Row r of K' lives in lane (r & 63), slot (r >> 6) (RPL = rows per lane).
// Padding rows r in [M, MAXM) are identity rows, so one code path serves every
// n with n + m <= MAXM.  Rows are never swapped: a pivoted row is marked with
// its step number and drops out of later updates (multiplier 0).
#pragma once

#include "common.hpp"

namespace rbf {

template <int D, int P>
struct Mono {
    static constexpr int m = n_mono(D, P);
    int e[m > 0 ? m : 1][3];
    constexpr Mono() : e() {
        int c = 0;
        for (int deg = 0; deg <= P; ++deg) {
            if (D == 2) {
                for (int a = deg; a >= 0; --a) {
                    e[c][0] = a;
                    e[c][1] = deg - a;
                    e[c][2] = 0;
                    ++c;
                }
            } else {
                for (int a = deg; a >= 0; --a)
                    for (int b = deg - a; b >= 0; --b) {
                        e[c][0] = a;
                        e[c][1] = b;
                        e[c][2] = deg - a - b;
                        ++c;
                    }
            }
        }
    }
    // (lap q_l)(0) and (d_a q_l)(0)
    constexpr double lq(int l, int op) const {
        int s = e[l][0] + e[l][1] + e[l][2];
        if (op == 0) return (s == 2 && (e[l][0] == 2 || e[l][1] == 2 || e[l][2] == 2)) ? 2.0 : 0.0;
        int a = op - 1;
        return (s == 1 && e[l][a] == 1) ? 1.0 : 0.0;
    }
};

// fixed coefficients of the test polynomial of the reproduction check
__host__ __device__ constexpr double check_coef(int l) { return 1.0 + 0.6180339887498949 * ((l * 7 + 3) % 11) / 11.0; }

template <int e>
__device__ __forceinline__ double ipow(double x) {
    if constexpr (e == 0) return 1.0;
    else if constexpr (e == 1) return x;
    else if constexpr (e == 2) return x * x;
    else if constexpr (e == 3) return x * x * x;
    else return (x * x) * (x * x);
}

// q_l(xh) for a static l
template <int D, int P, int l>
__device__ __forceinline__ double mono_val(const double (&xh)[3]) {
    constexpr Mono<D, P> M{};
    double v = ipow<M.e[l][0]>(xh[0]) * ipow<M.e[l][1]>(xh[1]);
    if constexpr (D == 3) v *= ipow<M.e[l][2]>(xh[2]);
    return v;
}

template <int D, int P, int... L>
__device__ __forceinline__ void mono_all(const double (&xh)[3], double* q, std::integer_sequence<int, L...>) {
    ((q[L] = mono_val<D, P, L>(xh)), ...);
}

template <int D, int P>
__device__ __forceinline__ void monomials(const double (&xh)[3], double* q) {
    mono_all<D, P>(xh, q, std::make_integer_sequence<int, n_mono(D, P)>{});
}

// phi(r) = r^k for odd k in {3, 5}, from r^2
__device__ __forceinline__ double phs_from_r2(double r2, int k) {
    double r = sqrt(r2);
    return (k == 5) ? r2 * r2 * r : r2 * r;
}

struct StencilArgs {
    const double* X;
    int64_t N;
    const int64_t* offsets;
    const int32_t* idx;
    int64_t nnz;
    int n_max;
    unsigned op_mask;
    int phs_power;
    int scale_mode;
    double repro_tol;
    double* w;
    int8_t* status;
};

// Write NaN weights and a status for a stencil that is rejected up front.
__device__ inline void reject_stencil(const StencilArgs& a, int64_t node, int64_t off, int64_t n, int8_t st) {
    int R = __builtin_popcount(a.op_mask);
    for (int r = 0; r < R; ++r)
        for (int64_t e = lane_id(); e < n; e += WAVE) a.w[r * a.nnz + off + e] = __builtin_nan("");
    if (a.status && lane_id() == 0) a.status[node] = st;
}

// Local frame of the stencil: scaled offsets of the nodes held by this lane's rows
// (row r = m + j holds node j), the scale s and its inverse.
template <int D, int P, int MAXM>
struct Frame {
    static constexpr int RPL = (MAXM + 63) / 64;
    double xh[RPL][3];
    double s, inv_s;
};

// Returns false (wave-uniform) if any stencil index is outside [0, N).
template <int D, int P, int MAXM>
__device__ __forceinline__ bool load_frame(const StencilArgs& a, int64_t off, int n, Frame<D, P, MAXM>& F) {
    constexpr int m = n_mono(D, P);
    constexpr int RPL = Frame<D, P, MAXM>::RPL;
    const int lane = lane_id();
    const int c = a.idx[off];
    bool bad = !(c >= 0 && c < a.N);
    double cx[3] = {0, 0, 0};
    if (!bad)
        for (int q = 0; q < D; ++q) cx[q] = a.X[(int64_t)c * D + q];
    double o[RPL][3];
    double r2max = 0.0, r2min = INFINITY;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        int j = lane + 64 * t - m;
        o[t][0] = o[t][1] = o[t][2] = 0.0;
        if (j >= 0 && j < n) {
            int id = a.idx[off + j];
            if (id >= 0 && id < a.N) {
                for (int q = 0; q < D; ++q) o[t][q] = a.X[(int64_t)id * D + q] - cx[q];
            } else {
                bad = true;
            }
            double r2 = o[t][0] * o[t][0] + o[t][1] * o[t][1] + o[t][2] * o[t][2];
            r2max = fmax(r2max, r2);
            if (j >= 1) r2min = fmin(r2min, r2);
        }
    }
    double r2 = (a.scale_mode == 1) ? wave_min_d(r2min) : wave_max_d(r2max);
    F.s = sqrt(r2);
    F.inv_s = 1.0 / F.s;
#pragma unroll
    for (int t = 0; t < RPL; ++t)
        for (int q = 0; q < 3; ++q) F.xh[t][q] = o[t][q] * F.inv_s;
    return __ballot(bad) == 0;
}

// Broadcast of the scaled coordinates of unknown/row index rr (static).
template <int RPL, int rr>
__device__ __forceinline__ void bcast_xh(const double (&xh)[RPL][3], double (&out)[3]) {
    constexpr int t = rr >> 6, ln = rr & 63;
#pragma unroll
    for (int q = 0; q < 3; ++q) out[q] = readlane_d(xh[t][q], ln);
}

}  // namespace rbf
